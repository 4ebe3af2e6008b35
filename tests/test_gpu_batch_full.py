"""Parity of the batched launch at the full many-filter shape: 4096 filters
with sizes log-uniform on [4 KiB, 16 MiB] (about 8.5 GB in all), 256-bit
blocks (8 x 32-bit words), k = 8, key counts Zipf(1.1) clipped to
[10^2, 10^7] summing to 2^28, lookups half present, half fresh -- the
workload the batched benchmark times, built by the same generator.

Every filter's words after the graph-replayed add and every lookup byte of
the graph-replayed contains are compared with the CPU oracle building each
filter from its own keys alone (the unchanged single-threaded oracle, one
filter per host thread).  The plain per-filter launches the benchmark
compares against must give the same words and bytes.
"""
from __future__ import annotations

import time

import numpy as np
import pytest
import torch

import oracle
from oracle import parallel as oracle_par
from gpu_helpers import log
from paper_2512_15595_amd import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

NF, TOTAL, S_WORDS, WBITS, K = 4096, 1 << 28, 8, 32, 8
BLOCK = S_WORDS * WBITS // 8


@pytest.fixture(scope="module")
def batch_run():
    from paper_2512_15595_amd import bf

    log(f"batch full: generating {NF} filters and {TOTAL} keys")
    sizes, offsets, keys, queries = workloads.batched_workload(NF, TOTAL, block_bytes=BLOCK)
    filters = [bf.BloomFilter(int(sz) // BLOCK, S_WORDS, WBITS, K, i) for i, sz in enumerate(sizes)]
    d_keys = torch.from_numpy(keys.view(np.int64)).to("cuda")
    d_q = torch.from_numpy(queries.view(np.int64)).to("cuda")
    out_g = torch.full((queries.size,), 7, dtype=torch.uint8, device="cuda")
    out_p = torch.full((queries.size,), 7, dtype=torch.uint8, device="cuda")
    add = bf.BatchPlan(bf.BF_OP_ADD, filters, d_keys, offsets)
    con = bf.BatchPlan(bf.BF_OP_CONTAINS, filters, d_q, offsets, out_g)
    con_p = bf.BatchPlan(bf.BF_OP_CONTAINS, filters, d_q, offsets, out_p)
    try:
        info_add = add.info()
        log(f"batch full: graph add (strategy {info_add.strategy}) and graph contains")
        add.launch()
        con.launch()
        words = [f.words() for f in filters]
        host_words = [w.cpu().numpy() for w in words]
        log("batch full: per-filter plain launches into cleared filters")
        for f in filters:
            f.clear()
        add.launch_per_filter()
        con_p.launch_per_filter()
        per_filter_equal = all(bool(torch.equal(f.words(), w)) for f, w in zip(filters, words))
        out_equal = bool(torch.equal(out_g, out_p))
        out = out_g.cpu().numpy()
        torch.cuda.synchronize()
    finally:
        for plan in (add, con, con_p):
            plan.close()
        for f in filters:
            f.close()
    del d_keys, d_q, out_g, out_p, words
    torch.cuda.empty_cache()
    return dict(sizes=sizes, offsets=offsets, keys=keys, queries=queries, words=host_words,
                out=out, info_add=info_add, per_filter_equal=per_filter_equal,
                out_equal=out_equal)


def test_workload_has_the_full_shape(batch_run):
    sizes, offsets = batch_run["sizes"], batch_run["offsets"]
    counts = np.diff(offsets)
    assert sizes.size == NF and int(offsets[-1]) == TOTAL
    assert sizes.min() >= 4 << 10 and sizes.max() <= 16 << 20
    assert counts.min() >= 100 and counts.max() <= 10_000_000
    # the automatic plan splits dense (partitioned) from sparse (tiled) filters
    from paper_2512_15595_amd import bf

    info = batch_run["info_add"]
    assert info.strategy == bf.BF_STRATEGY_PARTITIONED and info.ntiles > 0


def test_every_filter_and_lookup_equals_oracle(batch_run):
    sizes, offsets = batch_run["sizes"], batch_run["offsets"]
    keys, queries = batch_run["keys"], batch_run["queries"]
    words, out = batch_run["words"], batch_run["out"]
    want_out = np.zeros(queries.size, dtype=np.uint8)

    def one(i):
        a, b = int(offsets[i]), int(offsets[i + 1])
        ref = oracle.OracleFilter(int(sizes[i]) // BLOCK, S_WORDS, WBITS, K, i)
        ref.add(keys[a:b])
        want_out[a:b] = ref.contains(queries[a:b])
        return bool(np.array_equal(ref.bytes, words[i]))

    # largest jobs first so the pool drains evenly
    order = np.argsort(-np.diff(offsets), kind="stable")
    t0 = time.perf_counter()
    ok = dict(zip(order.tolist(), oracle_par.per_filter(order.tolist(), one)))
    log(f"batch full: oracle over {NF} filters in {time.perf_counter() - t0:.1f}s")
    bad = [i for i in range(NF) if not ok[i]]
    assert not bad, f"{len(bad)} filters differ from the oracle, e.g. {bad[:8]}"
    if not np.array_equal(out, want_out):
        diff = np.flatnonzero(out != want_out)
        pytest.fail(f"{diff.size} lookup bytes differ from the oracle (first {diff[:8]})")


def test_per_filter_launches_agree(batch_run):
    assert batch_run["per_filter_equal"]
    assert batch_run["out_equal"]
