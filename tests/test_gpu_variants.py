"""GPU parity of the classic (Sec. II-A-1) and cache-sectorized (Sec. II-A-5)
layouts against the CPU oracle, bit-exact: identical filter bytes and every
lookup byte, for every compiled execution mapping, compiled and runtime k,
power-of-two and other sizes, ragged and misaligned key arrays; and at the
cache-regime scale (256 MiB) on sampled words and lookups.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import log, to_device
from paper_2512_15595_amd import workloads

pytestmark = pytest.mark.gpu


def _bf():
    from paper_2512_15595_amd import bf

    return bf


def _run(f, adds, queries, add_offset=0, query_offset=0):
    if adds.size:
        f.add(to_device(adds, add_offset))
    out = None
    if queries.size:
        out = f.contains(to_device(queries, query_offset)).cpu().numpy()
    words = f.words().cpu().numpy()
    torch.cuda.synchronize()
    return words, out


def _keys(n, seed):
    return workloads.rng(seed).integers(0, 2**64, size=n, dtype=np.uint64)


# --------------------------------------------------------------------------
# Classic
# --------------------------------------------------------------------------

CLASSIC_CASES = [
    # (num_bits, k): powers of two and not, compiled and runtime k
    (1 << 20, 8),
    (64 * 12345, 8),
    (1 << 16, 16),
    (64 * 1000, 5),
    (1 << 23, 4),
    (64 * 777, 12),
    (64, 3),
    (1 << 18, 6),
    (64 * 5003, 32),
]


@pytest.mark.parametrize("m,k", CLASSIC_CASES)
def test_classic_matches_oracle(m, k):
    bf = _bf()
    n = max(1, m // 16) + 37
    adds = _keys(n, m + k)
    queries = np.concatenate([adds[::2], _keys(3 * 1024 + 5, m + k + 1)])
    ref = oracle.ClassicOracle(m, k, seed=0x5EED + k)
    ref.add(adds)
    want_out = ref.contains(queries)
    for kt in (1, 2, 4):
        log(f"classic m={m} k={k} kt={kt}")
        f = bf.ClassicFilter(m, k, 0x5EED + k)
        try:
            f.set_mapping(bf.BF_OP_ADD, 1, 1, kt)
            f.set_mapping(bf.BF_OP_CONTAINS, 1, 1, kt)
            words, out = _run(f, adds, queries)
        finally:
            f.close()
        assert np.array_equal(words, ref.bytes), f"kt={kt}"
        assert np.array_equal(out, want_out), f"kt={kt}"
        assert np.all(out[: adds[::2].size] == 1)


def test_classic_edges():
    """Empty and single-key batches, misaligned key and result arrays, a
    key count one short of a tile, clear and save / restore."""
    bf = _bf()
    m, k = 64 * 4099, 8
    f = bf.ClassicFilter(m, k, 3)
    ref = oracle.ClassicOracle(m, k, 3)
    try:
        empty = np.zeros(0, dtype=np.uint64)
        words, _ = _run(f, empty, empty)
        assert not words.any()
        one = _keys(1, 1)
        ref.add(one)
        words, out = _run(f, one, one)
        assert np.array_equal(words, ref.bytes) and out.tolist() == [1]
        adds = _keys(2 * 256 * 4 - 1, 2)
        ref.add(adds)
        queries = np.concatenate([adds, _keys(5000, 3)])
        words, out = _run(f, adds, queries, add_offset=1, query_offset=1)
        assert np.array_equal(words, ref.bytes)
        assert np.array_equal(out, ref.contains(queries))
        saved = f.words()
        f.clear()
        assert not f.words().cpu().numpy().any()
        f.load_words(saved)
        assert np.array_equal(f.words().cpu().numpy(), ref.bytes)
        info = f.info()
        assert info.layout == bf.BF_LAYOUT_CLASSIC and info.num_bits == m
        assert info.size_bytes == m // 8 and info.mapping[bf.BF_OP_ADD].strategy == bf.BF_STRATEGY_AUTO
        with pytest.raises(bf.BfError):
            f.set_mapping(bf.BF_OP_ADD, 2, 1, 1)
        f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
    finally:
        f.close()
    g = bf.ClassicFilter(m, 5, 3)          # runtime k: no partitioned construction
    try:
        assert g.info().mapping[bf.BF_OP_ADD].strategy == bf.BF_STRATEGY_DIRECT
        with pytest.raises(bf.BfError) as e:
            g.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
        assert e.value.status == bf.BF_EUNSUPPORTED
    finally:
        g.close()


@pytest.mark.parametrize("m,k", [(1 << 20, 8), (64 * 40_003, 6), (1 << 23, 16), (64 * 7777, 12),
                                 (1 << 16, 4), (64 * 1000, 16)])
def test_classic_partitioned_add_bit_exact(m, k):
    """Forced partitioned construction of the classic filter (k records per
    key, grouped by 64 KiB chunk); a quarter of the keys repeat one key, so
    its chunks' buckets overflow into the direct fallback."""
    bf = _bf()
    adds = _keys(300_000, m % 1000 + k)
    adds[: adds.size // 4] = adds[3]
    ref = oracle.ClassicOracle(m, k, 21)
    ref.add(adds)
    queries = np.concatenate([adds[::7], _keys(50_000, 5)])
    log(f"classic partitioned m={m} k={k}")
    f = bf.ClassicFilter(m, k, 21)
    try:
        f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
        words, out = _run(f, adds, queries, add_offset=1)
    finally:
        f.close()
    assert np.array_equal(words, ref.bytes)
    assert np.array_equal(out, ref.contains(queries))


def test_classic_auto_strategy_matches_direct():
    bf = _bf()
    m, k = 1 << 28, 8
    adds = _keys(1 << 21, 44)
    states = []
    for strategy in (bf.BF_STRATEGY_AUTO, bf.BF_STRATEGY_DIRECT):
        f = bf.ClassicFilter(m, k, 9)
        try:
            f.set_mapping(bf.BF_OP_ADD, strategy=strategy)
            f.add(to_device(adds))
            states.append(f.words().cpu().numpy())
        finally:
            f.close()
    assert np.array_equal(states[0], states[1])
    sel = np.unique(workloads.rng(45).integers(0, m // 64, size=4096, dtype=np.uint64))
    want = oracle.classic_words(m, k, 9, adds, sel)
    assert np.array_equal(states[0].view("<u8")[sel.astype(np.int64)], want)


def test_classic_cache_regime_full_size_sampled():
    """256 MiB (2^31 bits), k = 8, c = 16 bits per key: 2^27 adds, then
    lookups of 2^24 inserted and 2^24 fresh keys.  Checked on 2^13 sampled
    64-bit words (oracle from the keys alone), sampled lookups against the
    oracle's rule on the GPU state, and no false negatives anywhere."""
    bf = _bf()
    m, k, seed = 1 << 31, 8, 77
    n = m // 16
    log(f"classic full size m={m} n={n}")
    adds = _keys(n, 101)
    queries = np.concatenate([adds[: 1 << 24], _keys(1 << 24, 102)])
    f = bf.ClassicFilter(m, k, seed)
    try:
        f.add(to_device(adds))
        out = f.contains(to_device(queries)).cpu().numpy()
        state = f.words().cpu().numpy()
    finally:
        f.close()
    assert np.all(out[: 1 << 24] == 1)
    g = workloads.rng(5)
    sel = np.unique(g.integers(0, m // 64, size=1 << 13, dtype=np.uint64))
    want = oracle.classic_words(m, k, seed, adds, sel)
    assert np.array_equal(state.view("<u8")[sel.astype(np.int64)], want)
    ref = oracle.ClassicOracle(m, k, seed)
    ref.bytes = state
    pick = g.integers(0, queries.size, size=1 << 16)
    assert np.array_equal(out[pick], ref.contains(queries[pick]))
    fill = float(np.unpackbits(state[: 1 << 24]).mean())
    assert abs(fill - (1 - np.exp(-k / 16))) < 0.005


# --------------------------------------------------------------------------
# Cache-sectorized
# --------------------------------------------------------------------------

CSBF_LAYOUTS = [(s, S, z) for S in (32, 64) for s in (1, 2, 4, 8, 16)
                for z in (1, 2, 4, 8, 16) if z <= s]


def _csbf_mappings(z):
    out = [(1, 1), (1, 2)]
    theta = 2
    while theta <= z:
        out.append((theta, 1))
        theta *= 2
    return out


@pytest.mark.parametrize("s,S,z", CSBF_LAYOUTS)
def test_csbf_every_mapping_bit_exact(s, S, z):
    bf = _bf()
    g = workloads.rng(300 + 7 * s + S + z)
    ks = sorted({k for k in (4, 8, 16, z, 2 * z, 3 * z) if k >= z and k % z == 0 and k <= 32})
    for k in ks:
        params = dict(num_blocks=1013, words_per_block=s, word_bits=S, groups=z, k=k,
                      seed=int(g.integers(0, 2**63)))
        adds = g.integers(0, 2**64, size=2 * 1024 + 29, dtype=np.uint64)
        queries = np.concatenate([adds[::3], g.integers(0, 2**64, size=3000, dtype=np.uint64)])
        ref = oracle.CsbfOracle(**params)
        ref.add(adds)
        want_out = ref.contains(queries)
        for theta, kt in _csbf_mappings(z):
            log(f"csbf s={s} S={S} z={z} k={k} theta={theta} kt={kt}")
            f = bf.CacheSectorizedFilter(**params)
            try:
                f.set_mapping(bf.BF_OP_ADD, theta, 0, kt)
                f.set_mapping(bf.BF_OP_CONTAINS, theta, 0, kt)
                words, out = _run(f, adds, queries)
            finally:
                f.close()
            assert np.array_equal(words, ref.bytes), (k, theta, kt)
            assert np.array_equal(out, want_out), (k, theta, kt)


def test_csbf_one_word_per_group_equals_sectorized_gpu():
    """z = s on the GPU gives the sectorized filter's words exactly."""
    bf = _bf()
    adds = _keys(50_000, 9)
    queries = np.concatenate([adds[:1000], _keys(20_000, 10)])
    for s, S, k in ((8, 32, 8), (16, 64, 16), (4, 64, 12)):
        a = bf.CacheSectorizedFilter(5000, s, S, s, k, 17)
        b = bf.BloomFilter(5000, s, S, k, 17)
        try:
            wa, oa = _run(a, adds, queries)
            wb, ob = _run(b, adds, queries)
        finally:
            a.close()
            b.close()
        assert np.array_equal(wa, wb) and np.array_equal(oa, ob)


def test_csbf_edges():
    bf = _bf()
    params = dict(num_blocks=777, words_per_block=16, word_bits=64, groups=4, k=8, seed=4)
    f = bf.CacheSectorizedFilter(**params)
    ref = oracle.CsbfOracle(**params)
    try:
        empty = np.zeros(0, dtype=np.uint64)
        words, _ = _run(f, empty, empty)
        assert not words.any()
        adds = _keys(2 * 512 - 1, 11)
        ref.add(adds)
        queries = np.concatenate([adds, _keys(4000, 12)])
        words, out = _run(f, adds, queries, add_offset=1, query_offset=1)
        assert np.array_equal(words, ref.bytes)
        assert np.array_equal(out, ref.contains(queries))
        info = f.info()
        assert info.layout == bf.BF_LAYOUT_CACHE_SECTORIZED and info.groups == 4
        with pytest.raises(bf.BfError):
            f.set_mapping(bf.BF_OP_ADD, 8, 0, 1)          # THETA > z
        with pytest.raises(bf.BfError):
            f.set_mapping(bf.BF_OP_CONTAINS, 2, 0, 2)     # two keys per lane needs THETA = 1
        with pytest.raises(bf.BfError):
            f.set_mapping(bf.BF_OP_ADD, 2, 4, 1)          # PHI must be s / THETA
        # single-block contention: every key lands in one block
        g = bf.CacheSectorizedFilter(1, 8, 32, 2, 4, 0)
        r1 = oracle.CsbfOracle(1, 8, 32, 2, 4, 0)
        try:
            many = _keys(100_000, 13)
            r1.add(many)
            w1, o1 = _run(g, many, many[:1000])
            assert np.array_equal(w1, r1.bytes) and np.all(o1 == 1)
        finally:
            g.close()
    finally:
        f.close()


def test_csbf_rejected_by_batch_and_server():
    bf = _bf()
    f = bf.CacheSectorizedFilter(1024, 8, 32, 2, 4, 0)
    c = bf.ClassicFilter(1 << 16, 4, 0)
    d_keys = torch.zeros(16, dtype=torch.int64, device="cuda")
    try:
        for filt in (f, c):
            with pytest.raises(bf.BfError) as e:
                bf.BatchPlan(bf.BF_OP_ADD, [filt], d_keys, np.array([0, 16]))
            assert e.value.status == bf.BF_EUNSUPPORTED
            with pytest.raises(bf.BfError) as e:
                bf.Server([filt])
            assert e.value.status == bf.BF_EUNSUPPORTED
    finally:
        f.close()
        c.close()


@pytest.mark.parametrize("s,S,z,k", [(8, 32, 2, 4), (16, 64, 4, 8), (4, 64, 4, 12), (2, 32, 1, 6),
                                     (16, 32, 16, 16), (8, 64, 2, 10)])
def test_csbf_partitioned_add_bit_exact(s, S, z, k):
    """Forced partitioned construction (keys grouped by 64 KiB chunk, applied
    in LDS) on a 40-chunk filter with a ragged block count; a quarter of the
    keys repeat one key, so its chunk's buckets overflow into the direct
    fallback.  The automatic choice on a 64 MiB filter must agree too."""
    bf = _bf()
    block = s * S // 8
    b = (40 * 65536) // block - 3
    params = dict(num_blocks=b, words_per_block=s, word_bits=S, groups=z, k=k, seed=123)
    adds = _keys(600_000, 41 + s + z)
    adds[: adds.size // 4] = adds[7]
    ref = oracle.CsbfOracle(**params)
    ref.add(adds)
    queries = np.concatenate([adds[::5], _keys(100_000, 42)])
    log(f"csbf partitioned s={s} S={S} z={z} k={k}")
    f = bf.CacheSectorizedFilter(**params)
    try:
        f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
        assert f.info().mapping[bf.BF_OP_ADD].strategy == bf.BF_STRATEGY_PARTITIONED
        words, out = _run(f, adds, queries)
    finally:
        f.close()
    assert np.array_equal(words, ref.bytes)
    assert np.array_equal(out, ref.contains(queries))


def test_csbf_auto_strategy_matches_direct():
    bf = _bf()
    b = (64 << 20) // 32
    adds = _keys(3 << 20, 43)
    states = []
    for strategy in (bf.BF_STRATEGY_AUTO, bf.BF_STRATEGY_DIRECT):
        f = bf.CacheSectorizedFilter(b, 8, 32, 2, 4, 5)
        try:
            f.set_mapping(bf.BF_OP_ADD, strategy=strategy)
            f.add(to_device(adds))
            states.append(f.words().cpu().numpy())
        finally:
            f.close()
    assert np.array_equal(states[0], states[1])
    sel = np.unique(workloads.rng(44).integers(0, b, size=4096, dtype=np.uint64))
    want = oracle.csbf_block_words(b, 8, 32, 2, 4, 5, adds, sel)
    assert np.array_equal(states[0].reshape(b, 32)[sel.astype(np.int64)], want)


@pytest.mark.parametrize("s,S,z,k", [(8, 32, 2, 4), (16, 64, 4, 16)])
def test_csbf_cache_regime_full_size_sampled(s, S, z, k):
    """256 MiB filters at 16 bits per key: 2^27 adds, 2^25 lookups (half
    inserted); 2^12 sampled blocks against the oracle from the keys alone,
    sampled lookups against the oracle's rule on the GPU state."""
    bf = _bf()
    nbytes = 1 << 28
    b = nbytes // (s * S // 8)
    n = nbytes * 8 // 16
    seed = 99
    log(f"csbf full size s={s} S={S} z={z} k={k} n={n}")
    adds = _keys(n, 201)
    queries = np.concatenate([adds[: 1 << 24], _keys(1 << 24, 202)])
    f = bf.CacheSectorizedFilter(b, s, S, z, k, seed)
    try:
        f.add(to_device(adds))
        out = f.contains(to_device(queries)).cpu().numpy()
        state = f.words().cpu().numpy()
    finally:
        f.close()
    assert np.all(out[: 1 << 24] == 1)
    g = workloads.rng(6)
    sel = np.unique(g.integers(0, b, size=1 << 12, dtype=np.uint64))
    want = oracle.csbf_block_words(b, s, S, z, k, seed, adds, sel)
    blocks = state.reshape(b, s * S // 8)
    assert np.array_equal(blocks[sel.astype(np.int64)], want)
    ref = oracle.CsbfOracle(b, s, S, z, k, seed)
    ref.bytes = state
    pick = g.integers(0, queries.size, size=1 << 16)
    assert np.array_equal(out[pick], ref.contains(queries[pick]))


# --------------------------------------------------------------------------
# Chained pattern hashing (the prior-art baseline of the breakdown)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("s,S", [(s, S) for S in (32, 64) for s in (1, 2, 4, 8, 16)])
def test_chained_bit_exact(s, S):
    bf = _bf()
    g = workloads.rng(500 + s + S)
    for k in sorted({s, 8 if s <= 8 else 16, 16, 11 if s <= 11 else 20}):
        params = dict(num_blocks=1019, words_per_block=s, word_bits=S, k=k,
                      seed=int(g.integers(0, 2**63)))
        adds = g.integers(0, 2**64, size=3 * 256 + 17, dtype=np.uint64)
        queries = np.concatenate([adds[::2], g.integers(0, 2**64, size=2000, dtype=np.uint64)])
        ref = oracle.ChainedOracle(**params)
        ref.add(adds)
        log(f"chained s={s} S={S} k={k}")
        f = bf.ChainedHashFilter(**params)
        try:
            words, out = _run(f, adds, queries, add_offset=1)
            info = f.info()
        finally:
            f.close()
        assert info.layout == bf.BF_LAYOUT_SECTORIZED_CHAINED
        assert np.array_equal(words, ref.bytes), k
        assert np.array_equal(out, ref.contains(queries)), k


def test_chained_mapping_and_strategy_limits():
    bf = _bf()
    f = bf.ChainedHashFilter(256, 8, 32, 8, 1)
    try:
        f.set_mapping(bf.BF_OP_ADD, 1, 8, 1)
        with pytest.raises(bf.BfError):
            f.set_mapping(bf.BF_OP_ADD, 2, 4, 1)
        with pytest.raises(bf.BfError) as e:
            f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
        assert e.value.status == bf.BF_EUNSUPPORTED
        big = _keys(1 << 22, 91)                      # dense: would be partitioned if allowed
        ref = oracle.ChainedOracle(256, 8, 32, 8, 1)
        ref.add(big[:20000])
        words, _ = _run(f, big[:20000], np.zeros(0, dtype=np.uint64))
        assert np.array_equal(words, ref.bytes)
    finally:
        f.close()
