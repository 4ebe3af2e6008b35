"""Parity at the full DRAM-resident size, in the launch configuration the
benchmark times: a 1 GiB filter (2^25 blocks of 8 x 32-bit words, k = 8),
2^28 adds, 2^28 lookups at each of 0 / 50 / 100 % hits.

Every one of the 2^30 filter bytes and every one of the 3 x 2^28 lookup
bytes is compared with the CPU oracle.  The oracle is the unchanged
single-threaded C definition, run on host threads over disjoint block
ranges (words) and query slices (lookups) by oracle/parallel.py.  The
construction the benchmark times (the default strategy, partitioned at this
density) is compared with the oracle; the paper's direct construction at the
same size must then give the same words.
"""
from __future__ import annotations

import math
import time

import numpy as np
import pytest
import torch

import fpr_model
from oracle import parallel as oracle_par
from gpu_helpers import log
from paper_2512_15595_amd import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

NB, S_WORDS, WBITS, K, SEED = 1 << 25, 8, 32, 8, 0
N = 1 << 28


@pytest.fixture(scope="module")
def dram_run():
    from paper_2512_15595_amd import bf

    log("dram: generating 2^28 keys and 3 x 2^28 queries")
    adds, queries = workloads.dram_workload(N)
    f = bf.BloomFilter(NB, S_WORDS, WBITS, K, SEED)
    strategy = f.add_strategy(N)
    d_adds = torch.from_numpy(adds.view(np.int64)).to("cuda")
    log(f"dram: bf_add of 2^28 keys (default strategy {strategy}) into 1 GiB")
    f.add(d_adds)                      # default strategy, as benchmarked
    outs = {}
    for h, q in queries.items():
        log(f"dram: bf_contains of 2^28 queries at {h} % hits")
        d_q = torch.from_numpy(q.view(np.int64)).to("cuda")
        outs[h] = f.contains(d_q).cpu().numpy()
        del d_q
    words_dev = f.words()
    # the paper's construction (one atomic OR group per key) at the same size
    log("dram: bf_add of the same keys with the direct strategy into a second filter")
    g = bf.BloomFilter(NB, S_WORDS, WBITS, K, SEED)
    g.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_DIRECT)
    g.add(d_adds)
    direct_equal = bool(torch.equal(g.words(), words_dev))
    words = words_dev.cpu().numpy()
    torch.cuda.synchronize()
    g.close()
    f.close()
    del d_adds, words_dev
    torch.cuda.empty_cache()
    return dict(adds=adds, queries=queries, outs=outs, words=words, strategy=strategy,
                direct_equal=direct_equal)


@pytest.fixture(scope="module")
def oracle_words(dram_run):
    t0 = time.perf_counter()
    w = oracle_par.filter_words(NB, S_WORDS, WBITS, K, SEED, dram_run["adds"])
    log(f"dram: oracle words of all 2^25 blocks in {time.perf_counter() - t0:.1f}s "
        f"({oracle_par.workers()} threads)")
    return w


def test_benchmarked_add_is_partitioned(dram_run):
    from paper_2512_15595_amd import bf

    assert dram_run["strategy"] == bf.BF_STRATEGY_PARTITIONED


def test_all_filter_words_equal_oracle(dram_run, oracle_words):
    words = dram_run["words"]
    assert words.size == oracle_words.size == NB * S_WORDS * WBITS // 8
    if not np.array_equal(words, oracle_words):
        bad = np.flatnonzero(words.reshape(NB, -1).view(np.uint64).any(axis=1) !=
                             oracle_words.reshape(NB, -1).view(np.uint64).any(axis=1))
        diff = np.flatnonzero((words != oracle_words).reshape(NB, -1).any(axis=1))
        pytest.fail(f"{diff.size} blocks differ from the oracle (first {diff[:8]}); "
                    f"{bad.size} differ in emptiness")


def test_direct_construction_gives_the_same_words(dram_run):
    assert dram_run["direct_equal"]


@pytest.mark.parametrize("hits", [0, 50, 100])
def test_every_lookup_equals_oracle(dram_run, oracle_words, hits):
    q = dram_run["queries"][hits]
    t0 = time.perf_counter()
    want = oracle_par.contains(oracle_words, NB, S_WORDS, WBITS, K, SEED, q)
    log(f"dram: oracle lookups of 2^28 queries at {hits} % hits in "
        f"{time.perf_counter() - t0:.1f}s")
    got = dram_run["outs"][hits]
    assert got.dtype == np.uint8 and got.size == N
    if not np.array_equal(got, want):
        diff = np.flatnonzero(got != want)
        pytest.fail(f"{diff.size} lookups differ from the oracle (first {diff[:8]}, "
                    f"got {got[diff[:8]]}, want {want[diff[:8]]})")


def test_no_false_negatives_at_full_size(dram_run):
    outs, queries = dram_run["outs"], dram_run["queries"]
    assert outs[100].all()
    hit_pos = queries[50] == queries[100]
    assert outs[50][hit_pos].all()


def test_false_positive_rate_at_full_size(dram_run):
    outs, words = dram_run["outs"], dram_run["words"]
    p = fpr_model.sbf_fpr(N, NB, S_WORDS, WBITS, K)
    got = outs[0].mean()
    # 2^28 independent-ish queries on one filter: binomial spread plus the
    # model's 2 % allowance for filter-to-filter variation
    sd = math.sqrt(p * (1 - p) / N)
    assert abs(got - p) <= 6 * sd + 0.02 * p, (got, p)
    fill = np.unpackbits(words[: 1 << 24]).mean()
    want_fill = fpr_model.sbf_fill_fraction(N, NB, S_WORDS, WBITS, K)
    assert abs(fill - want_fill) <= 0.002 * want_fill + 5 * math.sqrt(want_fill / (8 << 24))
