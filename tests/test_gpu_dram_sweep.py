"""Parity over the DRAM-resident layout sweep: 1 GiB filters of every block
shape the sweep covers -- words per block s in {1, 2, 4, 8, 16} x word width
S in {32, 64} bits (block sizes 32 to 1024 bits), k = 8 (raised to s = 16
where k < s) -- each built from the workload's 2^28 uniform keys with the
automatic construction (partitioned at this density) and with the direct
one, then looked up with every lanes-per-key count of the sweep (1, 2, 4, 8,
where <= s) on 2^26 queries, half of them present.

Every byte of every filter and every lookup byte is compared with the CPU
oracle (the unchanged single-threaded C, on host threads over block ranges
and query slices: oracle/parallel.py).  The 256-bit layout with the full
3 x 2^28 lookups at 0 / 50 / 100 % hits is tests/test_gpu_dram.py.
"""
from __future__ import annotations

import time

import numpy as np
import pytest
import torch

from gpu_helpers import log
from oracle import parallel as oracle_par
from paper_2512_15595_amd import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

FILTER_BYTES = 1 << 30
N_ADD, N_Q = 1 << 28, 1 << 26
LAYOUTS = [(s, S) for S in (32, 64) for s in (1, 2, 4, 8, 16)]


@pytest.fixture(scope="module")
def keys():
    adds = workloads.uniform_keys(N_ADD, 31)
    queries = workloads.mix(adds[:N_Q], workloads.uniform_keys(N_Q, 32), 0.5, 33)
    return adds, queries


@pytest.mark.parametrize("s,S", LAYOUTS, ids=[f"{s}x{S}" for s, S in LAYOUTS])
def test_layout_at_1gib_equals_oracle(keys, s, S):
    from paper_2512_15595_amd import bf

    adds, queries = keys
    k = max(8, s)
    nb = FILTER_BYTES // (s * S // 8)
    seed = 100 + s * S
    f = bf.BloomFilter(nb, s, S, k, seed)
    g = bf.BloomFilter(nb, s, S, k, seed)
    d_adds = torch.from_numpy(adds.view(np.int64)).to("cuda")
    d_q = torch.from_numpy(queries.view(np.int64)).to("cuda")
    try:
        strategy = f.add_strategy(N_ADD)
        log(f"dram sweep {s}x{S} k={k}: bf_add of 2^28 keys into 1 GiB (strategy {strategy}) "
            f"and the direct construction")
        assert strategy == bf.BF_STRATEGY_PARTITIONED
        f.add(d_adds)
        g.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_DIRECT)
        g.add(d_adds)
        direct_equal = bool(torch.equal(f.words(), g.words()))
        outs = {}
        theta = 1
        while theta <= min(s, 8):
            f.set_mapping(bf.BF_OP_CONTAINS, theta, s // theta, 2)
            outs[theta] = f.contains(d_q).cpu().numpy()
            theta *= 2
        words = f.words().cpu().numpy()
        torch.cuda.synchronize()
    finally:
        f.close()
        g.close()
    assert direct_equal, "direct and partitioned construction differ"
    t0 = time.perf_counter()
    want_words = oracle_par.filter_words(nb, s, S, k, seed, adds)
    want = oracle_par.contains(want_words, nb, s, S, k, seed, queries)
    log(f"dram sweep {s}x{S}: oracle in {time.perf_counter() - t0:.1f}s")
    if not np.array_equal(words, want_words):
        bad = np.flatnonzero((words != want_words).reshape(nb, -1).any(axis=1))
        pytest.fail(f"{bad.size} blocks differ from the oracle (first {bad[:8]})")
    for theta, got in outs.items():
        assert np.array_equal(got, want), f"lookups with {theta} lanes per key differ"
    assert outs[1][queries == adds[:N_Q]].all()  # no false negatives
