"""GPU parity: the HIP kernels against the CPU oracle, bit-exact.

Filter words and every lookup byte must equal the oracle's on the same
seeded inputs, for every layout and every compiled execution mapping (the
result of the method does not depend on the mapping, paper Sec. IV-A).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import log, to_device, valid_mappings
from paper_2512_15595_amd import workloads

pytestmark = pytest.mark.gpu

LAYOUTS = [(s, S) for S in (32, 64) for s in (1, 2, 4, 8, 16)]


def _bf():
    from paper_2512_15595_amd import bf

    return bf


def _gpu_run(params, adds, queries, mapping=None, add_offset=0, query_offset=0):
    bf = _bf()
    f = bf.BloomFilter(params["num_blocks"], params["words_per_block"], params["word_bits"],
                       params["k"], params["seed"])
    try:
        if mapping is not None:
            theta, phi, kt, atomic = mapping
            f.set_mapping(bf.BF_OP_ADD, theta, phi, kt, atomic)
            f.set_mapping(bf.BF_OP_CONTAINS, theta, phi, kt, 0)
        if adds.size:
            f.add(to_device(adds, add_offset))
        out = None
        if queries.size:
            out = f.contains(to_device(queries, query_offset)).cpu().numpy()
        words = f.words().cpu().numpy()
        torch.cuda.synchronize()
        return words, out
    finally:
        f.close()


def _oracle(params, adds, queries):
    ref = oracle.OracleFilter(params["num_blocks"], params["words_per_block"],
                              params["word_bits"], params["k"], params["seed"])
    ref.add(adds)
    return ref.bytes.copy(), ref.contains(queries)


def test_correctness_workload_bit_exact():
    """2^20-bit filter (4096 x 8 x 32-bit words), k = 8, seed 0: 20,000
    adds and 1,000,000 lookups (half present), default mappings."""
    params, adds, queries = workloads.correctness_workload()
    log(f"correctness workload {params}")
    words, out = _gpu_run(params, adds, queries)
    want_words, want_out = _oracle(params, adds, queries)
    assert np.array_equal(words, want_words)
    assert np.array_equal(out, want_out)
    assert out.sum() >= 500_000


@pytest.mark.parametrize("s,S", LAYOUTS)
def test_every_mapping_bit_exact(s, S):
    """All layouts x all compiled mappings, on a non-power-of-two block
    count and a ragged key count (several tiles and a partial one)."""
    k = 16 if s == 16 else 8
    params = dict(num_blocks=1009, words_per_block=s, word_bits=S, k=k, seed=0xABCDEF)
    g = workloads.rng(7 + s * S)
    adds = g.integers(0, 2**64, size=3 * 1024 + 37, dtype=np.uint64)
    queries = np.concatenate([adds[::3], g.integers(0, 2**64, size=4000, dtype=np.uint64)])
    want_words, want_out = _oracle(params, adds, queries)
    for mapping in valid_mappings(s, S):
        log(f"layout s={s} S={S} mapping={mapping}")
        words, out = _gpu_run(params, adds, queries, mapping)
        assert np.array_equal(words, want_words), mapping
        assert np.array_equal(out, want_out), mapping


@pytest.mark.parametrize("s,S", [(1, 32), (1, 64), (2, 32), (4, 64), (8, 32), (8, 64), (16, 32)])
def test_k_values_compiled_and_runtime(s, S):
    """Compiled k (4, 6, 8, 12, 16) and runtime-k variants (others)."""
    g = workloads.rng(11 + s)
    adds = g.integers(0, 2**64, size=5000, dtype=np.uint64)
    queries = np.concatenate([adds[::2], g.integers(0, 2**64, size=5000, dtype=np.uint64)])
    for k in (4, 5, 6, 8, 12, 13, 16, 31, 32):
        if k < s:
            continue
        params = dict(num_blocks=777, words_per_block=s, word_bits=S, k=k, seed=k)
        log(f"k={k} s={s} S={S}")
        want_words, want_out = _oracle(params, adds, queries)
        for mapping in (None, (1, 1, 1, 32), (min(s, 4), 1, 2, 32)):
            words, out = _gpu_run(params, adds, queries, mapping)
            assert np.array_equal(words, want_words), (k, mapping)
            assert np.array_equal(out, want_out), (k, mapping)


def test_empty_single_and_misaligned_inputs():
    params = dict(num_blocks=4096, words_per_block=8, word_bits=32, k=8, seed=0)
    bf = _bf()
    f = bf.BloomFilter(4096, 8, 32, 8, 0)
    try:
        empty = torch.zeros(0, dtype=torch.int64, device="cuda")
        f.add(empty)
        assert f.contains(empty).numel() == 0
        assert int(f.words().sum().item()) == 0
    finally:
        f.close()
    g = workloads.rng(3)
    one = g.integers(0, 2**64, size=1, dtype=np.uint64)
    words, out = _gpu_run(params, one, one)
    want_words, want_out = _oracle(params, one, one)
    assert np.array_equal(words, want_words) and np.array_equal(out, want_out)
    # keys starting 8 bytes into an allocation: wide per-lane loads fall back
    adds = g.integers(0, 2**64, size=2051, dtype=np.uint64)
    queries = np.concatenate([adds, g.integers(0, 2**64, size=3001, dtype=np.uint64)])
    want_words, want_out = _oracle(params, adds, queries)
    for mapping in ((1, 8, 4, 32), (4, 2, 2, 64), (2, 4, 4, 32)):
        words, out = _gpu_run(params, adds, queries, mapping, add_offset=1, query_offset=3)
        assert np.array_equal(words, want_words), mapping
        assert np.array_equal(out, want_out), mapping


@pytest.mark.parametrize("s,S", [(1, 32), (8, 32), (16, 64)])
def test_single_block_maximum_contention(s, S):
    """b = 1: every key's atomics hit the same block."""
    k = 16 if s == 16 else 8
    params = dict(num_blocks=1, words_per_block=s, word_bits=S, k=k, seed=99)
    g = workloads.rng(5)
    adds = g.integers(0, 2**64, size=200_000, dtype=np.uint64)
    queries = g.integers(0, 2**64, size=20_000, dtype=np.uint64)
    want_words, want_out = _oracle(params, adds[:2000], queries)
    # the block saturates quickly; compare after few keys, then after many
    for mapping in (None, (1, s, 1, 32), (s if s <= 16 else 16, 1, 1, 32)):
        words, out = _gpu_run(params, adds[:2000], queries, mapping)
        assert np.array_equal(words, want_words), mapping
        assert np.array_equal(out, want_out), mapping
    want_words, _ = _oracle(params, adds, queries[:1])
    words, _ = _gpu_run(params, adds, queries[:1])
    assert np.array_equal(words, want_words)


def test_repeat_runs_and_clear_are_deterministic():
    bf = _bf()
    params, adds, queries = workloads.correctness_workload()
    f = bf.BloomFilter(4096, 8, 32, 8, 0)
    try:
        d_adds = to_device(adds)
        f.add(d_adds)
        first = f.words().cpu().numpy()
        f.add(d_adds)                       # idempotent
        assert np.array_equal(f.words().cpu().numpy(), first)
        f.clear()
        assert int(f.words().sum().item()) == 0
        half = adds.size // 2               # split batches give the same words
        f.add(to_device(adds[:half]))
        f.add(to_device(adds[half:]))
        assert np.array_equal(f.words().cpu().numpy(), first)
        # save / restore round trip
        saved = f.words()
        f.clear()
        f.load_words(saved)
        assert np.array_equal(f.words().cpu().numpy(), first)
        torch.cuda.synchronize()
    finally:
        f.close()


def test_bad_mapping_is_rejected():
    bf = _bf()
    f = bf.BloomFilter(4096, 8, 32, 8, 0)
    try:
        for args in [(3, 1, 1, 0), (1, 16, 1, 0), (4, 4, 1, 0), (32, 1, 1, 0), (1, 8, 3, 0),
                     (1, 1, 1, 64)]:
            with pytest.raises(bf.BfError):
                f.set_mapping(bf.BF_OP_ADD, *args)
        with pytest.raises(bf.BfError):
            f.set_mapping(bf.BF_OP_CONTAINS, 1, 8, 1, 64)
        info = f.info()
        assert info.mapping[bf.BF_OP_ADD].lanes_per_key >= 1
    finally:
        f.close()


@pytest.mark.parametrize("s,S", LAYOUTS)
def test_partitioned_add_bit_exact(s, S):
    """The partitioned construction (keys grouped by 64 KiB chunk, chunks
    updated in LDS) writes exactly the oracle's words: a block count that
    leaves the last chunk partial, ragged key counts, compiled and runtime k."""
    bf = _bf()
    block = s * S // 8
    for nblocks, nkeys, k in ((3 * (65536 // block) + 17, 100_003, 16 if s == 16 else 8),
                              (7, 5_000, max(s, 5)),
                              (200_001, 333_333, max(s, 12))):
        params = dict(num_blocks=nblocks, words_per_block=s, word_bits=S, k=k, seed=nblocks)
        g = workloads.rng(nblocks + s)
        adds = g.integers(0, 2**64, size=nkeys, dtype=np.uint64)
        queries = np.concatenate([adds[:2000], g.integers(0, 2**64, size=3000, dtype=np.uint64)])
        log(f"partitioned s={s} S={S} blocks={nblocks} keys={nkeys} k={k}")
        want_words, want_out = _oracle(params, adds, queries)
        f = bf.BloomFilter(**params)
        try:
            f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
            f.add(to_device(adds))
            assert np.array_equal(f.words().cpu().numpy(), want_words)
            assert np.array_equal(f.contains(to_device(queries)).cpu().numpy(), want_out)
            # a second batch on top (workspace reuse, smaller)
            more = g.integers(0, 2**64, size=nkeys // 3 + 1, dtype=np.uint64)
            f.add(to_device(more))
            ref = oracle.OracleFilter(**params)
            ref.add(adds)
            ref.add(more)
            assert np.array_equal(f.words().cpu().numpy(), ref.bytes)
            torch.cuda.synchronize()
        finally:
            f.close()



@pytest.mark.parametrize("chunks,extra_blocks", [(1024, 0), (1024, 1)])
def test_partitioned_add_at_the_one_pass_limit(chunks, extra_blocks):
    """Filters of exactly 1024 chunks of 64 KiB (partitioned in one pass) and
    of one block more (1025 chunks, the last holding one block: two passes)
    build the oracle's words, with a ragged key count and a second add."""
    bf = _bf()
    nblocks = chunks * (65536 // 32) + extra_blocks
    params = dict(num_blocks=nblocks, words_per_block=8, word_bits=32, k=8, seed=chunks + extra_blocks)
    g = workloads.rng(nblocks)
    adds = g.integers(0, 2**64, size=1_500_001, dtype=np.uint64)
    more = g.integers(0, 2**64, size=700_003, dtype=np.uint64)
    queries = np.concatenate([adds[:5000], g.integers(0, 2**64, size=20_000, dtype=np.uint64)])
    log(f"one-pass limit: {chunks} chunks + {extra_blocks} blocks, {adds.size} + {more.size} keys")
    ref = oracle.OracleFilter(**params)
    ref.add(adds)
    ref.add(more)
    f = bf.BloomFilter(**params)
    try:
        f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
        f.add(to_device(adds))
        f.add(to_device(more))
        assert np.array_equal(f.words().cpu().numpy(), ref.bytes)
        assert np.array_equal(f.contains(to_device(queries)).cpu().numpy(), ref.contains(queries))
        torch.cuda.synchronize()
    finally:
        f.close()

def test_auto_strategy_matches_direct():
    """Auto picks the partitioned path for a dense batch; words equal those
    of the direct path."""
    bf = _bf()
    params = dict(num_blocks=1 << 20, words_per_block=8, word_bits=32, k=8, seed=3)
    adds = workloads.uniform_keys(1 << 21, 17)
    d = to_device(adds)
    words = {}
    for strategy in (bf.BF_STRATEGY_AUTO, bf.BF_STRATEGY_DIRECT, bf.BF_STRATEGY_PARTITIONED):
        f = bf.BloomFilter(**params)
        try:
            f.set_mapping(bf.BF_OP_ADD, strategy=strategy)
            f.add(d)
            words[strategy] = f.words().cpu().numpy()
        finally:
            f.close()
    assert np.array_equal(words[0], words[1]) and np.array_equal(words[1], words[2])
    sel = workloads.rng(4).choice(params["num_blocks"], size=4096, replace=False).astype(np.uint64)
    want = oracle.block_words(params["num_blocks"], 8, 32, 8, 3, adds, sel)
    rows = words[0].reshape(params["num_blocks"], -1)[sel.astype(np.int64)]
    assert np.array_equal(rows, want)


def test_add_strategy_reports_the_construction():
    """bf_add_strategy resolves the automatic choice as bf_add does: direct
    for sparse batches, partitioned for dense ones, at the layout's measured
    crossover (the same rule the host-only bf_tuned_mapping reports); a
    forced strategy wins; the classic layout is measured in keys of k
    records; the chained layout is never partitioned."""
    bf = _bf()
    f = bf.BloomFilter(1 << 20, 8, 32, 8, 3)                 # 32 MiB
    try:
        assert f.add_strategy(0) == bf.BF_STRATEGY_DIRECT
        assert f.add_strategy(1 << 20) == bf.BF_STRATEGY_DIRECT
        assert f.add_strategy(1 << 22) == bf.BF_STRATEGY_PARTITIONED
        for n in (1 << 18, 1 << 20, 3 << 19, 1 << 21, 3 << 20, 1 << 22, 1 << 24):
            st, m = bf.bf_tuned_mapping(bf.BF_OP_ADD, 1 << 20, 8, 32, 8, n)
            assert st == 0 and f.add_strategy(n) == m.strategy
        f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_DIRECT)
        assert f.add_strategy(1 << 22) == bf.BF_STRATEGY_DIRECT
        f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
        assert f.add_strategy(10) == bf.BF_STRATEGY_PARTITIONED
    finally:
        f.close()
    c = bf.ClassicFilter(1 << 28, 8, 1)                      # 32 MiB, 8 records per key
    try:
        assert c.add_strategy(1 << 15) == bf.BF_STRATEGY_DIRECT
        assert c.add_strategy(1 << 20) == bf.BF_STRATEGY_PARTITIONED
    finally:
        c.close()
    h = bf.ChainedHashFilter(1 << 20, 8, 32, 8, 3)
    try:
        assert h.add_strategy(1 << 24) == bf.BF_STRATEGY_DIRECT
    finally:
        h.close()


def test_partitioned_overflow_with_repeated_keys():
    """Repeated keys pile into one chunk beyond its bucket capacity; the
    overflowing records take the direct-atomic fallback and the words still
    equal the oracle's."""
    bf = _bf()
    params = dict(num_blocks=(4 << 20) // 32, words_per_block=8, word_bits=32, k=8, seed=11)
    g = workloads.rng(99)
    few = g.integers(0, 2**64, size=3, dtype=np.uint64)
    adds = np.concatenate([np.repeat(few, 200_000), g.integers(0, 2**64, size=100_000, dtype=np.uint64)])
    adds = adds[g.permutation(adds.size)]
    want_words, _ = _oracle(params, adds, adds[:1])
    f = bf.BloomFilter(**params)
    try:
        f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
        f.add(to_device(adds))
        assert np.array_equal(f.words().cpu().numpy(), want_words)
        torch.cuda.synchronize()
    finally:
        f.close()


def test_filter_over_caller_owned_words():
    """bf_create_in: the caller's tensor is the filter state (adds land in it,
    byte-identical to the oracle) and saved words can be adopted in place."""
    bf = _bf()
    params = dict(num_blocks=3001, words_per_block=4, word_bits=64, k=8, seed=5)
    nbytes = params["num_blocks"] * 4 * 8
    words = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    adds = workloads.rng(90).integers(0, 2**64, size=40_000, dtype=np.uint64)
    queries = np.concatenate([adds[::4], workloads.rng(91).integers(0, 2**64, size=20_000,
                                                                    dtype=np.uint64)])
    want_words, want_out = _oracle(params, adds, queries)
    v = bf.BloomFilterView(words, **params)
    try:
        assert v.info().d_words == words.data_ptr()
        v.add(to_device(adds))
        out = v.contains(to_device(queries)).cpu().numpy()
        torch.cuda.synchronize()
    finally:
        v.close()
    assert np.array_equal(words.cpu().numpy(), want_words)        # the tensor is the state
    assert np.array_equal(out, want_out)
    saved = words.clone()
    w = bf.BloomFilterView(saved, **params)                       # adopt saved words
    try:
        assert np.array_equal(w.contains(to_device(queries)).cpu().numpy(), want_out)
    finally:
        w.close()
    assert words.sum().item() > 0                                  # destroy freed nothing
