"""GPU parity of the batched persistent launch (include/bf_batch.h).

Every filter of a batch must end with exactly the words the oracle builds
from that filter's keys alone, and every lookup byte must equal the
oracle's; the graph launch, the direct launch and the per-filter launches
must agree with each other bit for bit.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import log
from paper_2512_15595_amd import workloads

pytestmark = pytest.mark.gpu


def _bf():
    from paper_2512_15595_amd import bf

    return bf


def _make_batch(nfilters, total, sizes_extra=(), s=8, S=32, k=8, seed=21):
    block = s * S // 8
    sizes = list(workloads.log_uniform_sizes(nfilters, 4 << 10, 512 << 10, block, seed))
    sizes += list(sizes_extra)
    n = len(sizes)
    counts = workloads.zipf_counts(n, total, 1.1, 0, total // 4, seed + 1)
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    keys = workloads.uniform_keys(int(offsets[-1]), seed + 2)
    fresh = workloads.uniform_keys(int(offsets[-1]), seed + 3)
    queries = workloads.mix(keys, fresh, 0.5, seed + 4)
    params = [dict(num_blocks=int(sz) // block, words_per_block=s, word_bits=S, k=k, seed=1000 + i)
              for i, sz in enumerate(sizes)]
    return params, offsets, keys, queries


def _oracle(params, offsets, keys, queries):
    words, outs = [], np.zeros(queries.size, dtype=np.uint8)
    for i, p in enumerate(params):
        a, b = offsets[i], offsets[i + 1]
        ref = oracle.OracleFilter(**p)
        ref.add(keys[a:b])
        words.append(ref.bytes.copy())
        outs[a:b] = ref.contains(queries[a:b])
    return words, outs


def _run(params, offsets, keys, queries, mode, add_strategy=None):
    bf = _bf()
    filters = [bf.BloomFilter(**p) for p in params]
    if add_strategy is not None:
        filters[0].set_mapping(bf.BF_OP_ADD, strategy=add_strategy)
    d_keys = torch.from_numpy(keys.view(np.int64)).to("cuda")
    d_q = torch.from_numpy(queries.view(np.int64)).to("cuda")
    d_out = torch.full((queries.size,), 7, dtype=torch.uint8, device="cuda")
    add = bf.BatchPlan(bf.BF_OP_ADD, filters, d_keys, offsets)
    con = bf.BatchPlan(bf.BF_OP_CONTAINS, filters, d_q, offsets, d_out)
    try:
        for plan in (add, con):
            getattr(plan, {"graph": "launch", "direct": "launch_direct",
                           "per_filter": "launch_per_filter"}[mode])()
        words = [f.words().cpu().numpy() for f in filters]
        out = d_out.cpu().numpy()
        info = add.info(), con.info()
        torch.cuda.synchronize()
        return words, out, info
    finally:
        add.close()
        con.close()
        for f in filters:
            f.close()


@pytest.mark.parametrize("mode", ["graph", "direct", "per_filter"])
def test_batch_matches_oracle(mode):
    # many small filters plus Infinity-Cache and HBM sized ones: all three
    # per-class mappings run in one launch
    params, offsets, keys, queries = _make_batch(300, 1 << 19, sizes_extra=(8 << 20, 12 << 20, 260 << 20))
    log(f"batch mode={mode}: {len(params)} filters, {keys.size} keys")
    want_words, want_out = _oracle(params, offsets, keys, queries)
    words, out, (ia, ic) = _run(params, offsets, keys, queries, mode)
    for i in range(len(params)):
        assert np.array_equal(words[i], want_words[i]), f"filter {i}"
    assert np.array_equal(out, want_out)
    assert ia.nfilters == len(params) and ia.nkeys == keys.size
    assert ia.grid % 8 == 0
    assert ia.tiles_per_class[0] > 0 and ia.tiles_per_class[1] > 0 and ia.tiles_per_class[2] > 0


@pytest.mark.parametrize("s,S,k", [(1, 64, 8), (4, 32, 5), (16, 64, 16), (8, 64, 12)])
def test_batch_other_layouts(s, S, k):
    params, offsets, keys, queries = _make_batch(120, 1 << 17, sizes_extra=(6 << 20,), s=s, S=S, k=k,
                                                 seed=40 + s)
    log(f"batch layout s={s} S={S} k={k}")
    want_words, want_out = _oracle(params, offsets, keys, queries)
    words, out, _ = _run(params, offsets, keys, queries, "graph")
    for i in range(len(params)):
        assert np.array_equal(words[i], want_words[i]), f"filter {i}"
    assert np.array_equal(out, want_out)


def test_batch_replay_and_empty_filters():
    """Replaying the graph is idempotent for add; filters with no keys are
    untouched; the plan rejects mixed layouts."""
    bf = _bf()
    params, offsets, keys, queries = _make_batch(50, 1 << 15, seed=77)
    counts = np.diff(offsets)
    counts[::7] = 0                                   # some filters get nothing
    offsets = np.concatenate([[0], np.cumsum(counts)])
    keys = keys[: offsets[-1]]
    queries = queries[: offsets[-1]]
    want_words, want_out = _oracle(params, offsets, keys, queries)
    filters = [bf.BloomFilter(**p) for p in params]
    d_keys = torch.from_numpy(keys.view(np.int64)).to("cuda")
    d_q = torch.from_numpy(queries.view(np.int64)).to("cuda")
    d_out = torch.zeros(queries.size, dtype=torch.uint8, device="cuda")
    add = bf.BatchPlan(bf.BF_OP_ADD, filters, d_keys, offsets)
    con = bf.BatchPlan(bf.BF_OP_CONTAINS, filters, d_q, offsets, d_out)
    try:
        for _ in range(3):
            add.launch()
            con.launch()
            torch.cuda.synchronize()
            for i, f in enumerate(filters):
                assert np.array_equal(f.words().cpu().numpy(), want_words[i])
            assert np.array_equal(d_out.cpu().numpy(), want_out)
        other = bf.BloomFilter(1024, 4, 32, 8, 0)
        with pytest.raises(bf.BfError):
            bf.BatchPlan(bf.BF_OP_ADD, filters[:3] + [other], d_keys, offsets[:5])
        other.close()
    finally:
        add.close()
        con.close()
        for f in filters:
            f.close()


@pytest.mark.parametrize("mode", ["graph", "direct"])
def test_batch_partitioned_add(mode):
    """One partitioned construction over all filters of a plan (forced):
    skewed key counts, empty filters, a filter of repeated keys (its chunk
    buckets overflow into the direct fallback), filters of every size class."""
    bf = _bf()
    params, offsets, keys, queries = _make_batch(200, 1 << 19, sizes_extra=(8 << 20, 300 << 20), seed=61)
    counts = np.diff(offsets)
    counts[5] = 0
    counts[17] = 0
    offsets = np.concatenate([[0], np.cumsum(counts)])
    keys = keys[: offsets[-1]].copy()
    queries = queries[: offsets[-1]]
    i = int(np.argmax(counts))                   # the busiest filter gets repeats
    keys[offsets[i]: offsets[i] + counts[i] // 2] = keys[offsets[i]]
    log(f"batch partitioned mode={mode}: {len(params)} filters, {keys.size} keys")
    want_words, want_out = _oracle(params, offsets, keys, queries)
    words, out, (ia, ic) = _run(params, offsets, keys, queries, mode,
                                add_strategy=bf.BF_STRATEGY_PARTITIONED)
    assert ia.strategy == bf.BF_STRATEGY_PARTITIONED
    for j in range(len(params)):
        assert np.array_equal(words[j], want_words[j]), f"filter {j}"
    assert np.array_equal(out, want_out)


@pytest.mark.parametrize("mode", ["graph", "direct"])
def test_batch_auto_add_splits_dense_and_sparse_filters(mode):
    """The automatic add plan partitions the dense filters (at least bytes /
    80 keys) and leaves the sparse ones, and the empty ones, to the tiled
    launch recorded after it; every filter's words equal the oracle's."""
    bf = _bf()
    block = 32
    g = workloads.rng(77)
    dense = [(8 << 20, 300_000 + int(g.integers(0, 1000))) for _ in range(8)]  # 1024 chunks, 2.4 M keys
    sparse = [(64 << 20, 5_000 + int(g.integers(0, 5000))) for _ in range(4)]
    empty = [(1 << 20, 0), (64 << 20, 0)]
    spec = dense[:4] + sparse[:2] + [empty[0]] + dense[4:] + sparse[2:] + [empty[1]]
    counts = np.array([c for _, c in spec], dtype=np.int64)
    offsets = np.zeros(len(spec) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    keys = workloads.uniform_keys(int(offsets[-1]), 78)
    params = [dict(num_blocks=sz // block, words_per_block=8, word_bits=32, k=8, seed=500 + i)
              for i, (sz, _) in enumerate(spec)]
    log(f"batch auto split mode={mode}: {len(spec)} filters, {keys.size} keys")
    want_words, _ = _oracle(params, offsets, keys, np.zeros(0, dtype=np.uint64))
    filters = [bf.BloomFilter(**p) for p in params]
    d_keys = torch.from_numpy(keys.view(np.int64)).to("cuda")
    add = bf.BatchPlan(bf.BF_OP_ADD, filters, d_keys, offsets)
    try:
        info = add.info()
        assert info.strategy == bf.BF_STRATEGY_PARTITIONED
        assert info.ntiles > 0                           # the sparse filters' tiles
        (add.launch if mode == "graph" else add.launch_direct)()
        words = [f.words().cpu().numpy() for f in filters]
        torch.cuda.synchronize()
    finally:
        add.close()
        for f in filters:
            f.close()
    for j in range(len(spec)):
        assert np.array_equal(words[j], want_words[j]), f"filter {j}"


@pytest.mark.parametrize("mode", ["graph", "direct"])
def test_plan_destroy_waits_for_its_own_launches_only(mode):
    """A plan destroyed right after its launch: the launch still completes
    with the oracle's results (the plan's memory is released behind it), and
    the host does not wait for another stream's queued work on an unrelated
    filter, enqueued after the plan's launch."""
    bf = _bf()
    block = 32
    g = workloads.rng(91)
    spec = [(8 << 20, 300_000 + int(g.integers(0, 1000))) for _ in range(8)]   # dense: partitioned
    spec += [(64 << 20, 4_000), (1 << 20, 0), (4 << 20, 2_000)]                 # sparse and empty: tiles
    counts = np.array([c for _, c in spec], dtype=np.int64)
    offsets = np.zeros(len(spec) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    keys = workloads.uniform_keys(int(offsets[-1]), 92)
    queries = workloads.mix(keys, workloads.uniform_keys(keys.size, 93), 0.5, 94)
    params = [dict(num_blocks=sz // block, words_per_block=8, word_bits=32, k=8, seed=700 + i)
              for i, (sz, _) in enumerate(spec)]
    want_words, want_out = _oracle(params, offsets, keys, queries)
    filters = [bf.BloomFilter(**p) for p in params]
    other = bf.BloomFilter((1 << 30) // block, 8, 32, 8, 3)
    d_keys = torch.from_numpy(keys.view(np.int64)).to("cuda")
    d_q = torch.from_numpy(queries.view(np.int64)).to("cuda")
    d_out = torch.full((queries.size,), 7, dtype=torch.uint8, device="cuda")
    d_other = torch.from_numpy(workloads.uniform_keys(1 << 26, 95).view(np.int64)).to("cuda")
    out_other = torch.empty(d_other.numel(), dtype=torch.uint8, device="cuda")
    s_plan, s_other = torch.cuda.Stream(), torch.cuda.Stream()
    try:
        for op in (bf.BF_OP_ADD, bf.BF_OP_CONTAINS):
            plan = (bf.BatchPlan(op, filters, d_keys, offsets) if op == bf.BF_OP_ADD
                    else bf.BatchPlan(op, filters, d_q, offsets, d_out))
            info = plan.info()
            if op == bf.BF_OP_ADD:
                assert info.strategy == bf.BF_STRATEGY_PARTITIONED and info.ntiles > 0
            torch.cuda.synchronize()
            log(f"plan destroy mode={mode} op={op}: plan launched, ~50 ms of other work queued after it")
            (plan.launch if mode == "graph" else plan.launch_direct)(stream=s_plan)
            for _ in range(40):
                other.contains(d_other, out=out_other, stream=s_other)
            done_other = torch.cuda.Event()
            done_other.record(s_other)
            plan.close()
            other_pending = not done_other.query()
            torch.cuda.synchronize()
            log(f"plan destroy mode={mode} op={op}: other work pending at return: {other_pending}")
            assert other_pending, "bf_batch_destroy waited for another stream's work"
        words = [f.words().cpu().numpy() for f in filters]
        out = d_out.cpu().numpy()
    finally:
        for f in filters:
            f.close()
        other.close()
    for j in range(len(params)):
        assert np.array_equal(words[j], want_words[j]), f"filter {j}"
    assert np.array_equal(out, want_out)
