"""GPU tests of the request loop (include/bf_serve.h).

A served mix of interleaved add / contains requests must give every request
the result it has when the requests run one by one in submission order
(tolerance 0): checked against the CPU oracle replaying the same sequence
per filter, and against the server's own serial replay.
"""
from __future__ import annotations

import ctypes

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


def _scenario(nfilters=6, nreq=240, seed=5, max_keys=20_000, s=8, S=32, k=8):
    g = workloads.rng(seed)
    block = s * S // 8
    sizes = workloads.log_uniform_sizes(nfilters, 64 << 10, 2 << 20, block, seed + 1)
    params = [dict(num_blocks=int(sz) // block, words_per_block=s, word_bits=S, k=k, seed=500 + i)
              for i, sz in enumerate(sizes)]
    # pre-populated at 32 bits per key
    prepop = [workloads.splitmix64(900 + i, 0, int(sz) // 4) for i, sz in enumerate(sizes)]
    ops = np.where(g.random(nreq) < 0.1, 0, 1)              # 1 add : 9 contains
    filt = g.integers(0, nfilters, size=nreq)
    ns = np.exp(np.log(100) + g.random(nreq) * (np.log(max_keys) - np.log(100))).astype(np.int64)
    keys, starts = [], [0]
    for i in range(nreq):
        f = int(filt[i])
        if ops[i] == 0:
            kk = workloads.splitmix64(5000 + i, 0, int(ns[i]))
        else:
            kk = workloads.mixed_queries(int(ns[i]), 900 + f, 0, prepop[f].size, 7000 + i, 0, 0.5,
                                         8000 + i)
        keys.append(kk)
        starts.append(starts[-1] + int(ns[i]))
    # bursty arrivals so that many requests are in flight together
    arrivals = np.cumsum(g.exponential(20_000, size=nreq)).astype(np.int64)
    return params, prepop, ops, filt, ns, np.concatenate(keys), np.array(starts), arrivals


def _expected(params, prepop, ops, filt, ns, keys, starts):
    refs = []
    for p, pk in zip(params, prepop):
        r = oracle.OracleFilter(**p)
        r.add(pk)
        refs.append(r)
    out = np.zeros(keys.size, dtype=np.uint8)
    for i in range(len(ops)):
        a, b = starts[i], starts[i + 1]
        if ops[i] == 0:
            refs[filt[i]].add(keys[a:b])
        else:
            out[a:b] = refs[filt[i]].contains(keys[a:b])
    return [r.bytes.copy() for r in refs], out


def _run(params, prepop, ops, filt, ns, keys, starts, arrivals, serial, **cfg):
    bf = _bf()
    filters = [bf.BloomFilter(**p) for p in params]
    for f, pk in zip(filters, prepop):
        f.add(torch.from_numpy(pk.view(np.int64)).to("cuda"))
    d_keys = torch.from_numpy(keys.view(np.int64)).to("cuda")
    d_out = torch.full((keys.size,), 9, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    srv = bf.Server(filters, **cfg)
    try:
        kp = [d_keys.data_ptr() + 8 * int(starts[i]) for i in range(len(ops))]
        op_ptr = [d_out.data_ptr() + int(starts[i]) if ops[i] == 1 else 0 for i in range(len(ops))]
        reqs = srv.requests(ops, filt, kp, ns, op_ptr, arrivals)
        res = srv.replay(reqs, serial=serial)
        stats = srv.stats()
        torch.cuda.synchronize()
        out = d_out.cpu().numpy()
        words = [f.words().cpu().numpy() for f in filters]
        return res, stats, out, words
    finally:
        srv.close()
        for f in filters:
            f.close()


@pytest.mark.parametrize("cfg", [
    dict(),                                                   # defaults: coalescing on
    dict(coalesce_max_keys=0, nstreams=4, max_inflight=8),    # one launch per request
    dict(hbm_budget_bytes=600_000, max_inflight=3, nstreams=2, coalesce_max_requests=4,
         coalesce_max_tiles=64),                              # tight budget and slots
], ids=["coalesce", "no_coalesce", "tight_budget"])
def test_served_results_equal_sequential_oracle(cfg):
    sc = _scenario()
    params, prepop, ops, filt, ns, keys, starts, arrivals = sc
    log(f"serve cfg={cfg}: {len(ops)} requests, {keys.size} keys")
    want_words, want_out = _expected(params, prepop, ops, filt, ns, keys, starts)
    res, stats, out, words = _run(*sc, serial=False, **cfg)
    assert all(r.status == 0 for r in res)
    mask = np.repeat(ops == 1, ns)
    assert np.array_equal(out[mask], want_out[mask])
    for i in range(len(params)):
        assert np.array_equal(words[i], want_words[i]), i
    assert stats.requests == len(ops)
    # every request's times are ordered
    for r in res:
        assert r.arrival_ns <= r.admit_ns <= r.complete_ns
    if cfg.get("coalesce_max_keys", 65536):
        assert stats.coalesced_launches > 0
    if "hbm_budget_bytes" in cfg:
        assert stats.peak_inflight_bytes <= cfg["hbm_budget_bytes"]
        assert stats.peak_inflight_launches <= cfg["max_inflight"]


def test_serial_replay_matches_too():
    sc = _scenario(nreq=120, seed=9)
    params, prepop, ops, filt, ns, keys, starts, arrivals = sc
    want_words, want_out = _expected(params, prepop, ops, filt, ns, keys, starts)
    res, _, out, words = _run(*sc, serial=True)
    mask = np.repeat(ops == 1, ns)
    assert np.array_equal(out[mask], want_out[mask])
    for i in range(len(params)):
        assert np.array_equal(words[i], want_words[i]), i


def test_device_key_generators_match_host():
    from paper_2512_15595_amd import bf as bfmod

    lib = ctypes.CDLL(bfmod.LIB_PATH)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    lib.bfb_fill_splitmix64.argtypes = [vp, u64, u64, u64, vp]
    lib.bfb_fill_mixed_queries.argtypes = [vp, u64, u64, u64, u32, u64, u64, u32, u64, vp]
    n = 100_003
    d = torch.empty(n, dtype=torch.int64, device="cuda")
    assert lib.bfb_fill_splitmix64(d.data_ptr(), n, 77, 1000, None) == 0
    got = d.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, workloads.splitmix64(77, 1000, n))
    hit = 0.5
    assert lib.bfb_fill_mixed_queries(d.data_ptr(), n, 5, 10, 4096, 6, 20,
                                      int(hit * 2**32), 9, None) == 0
    got = d.cpu().numpy().view(np.uint64)
    want = workloads.mixed_queries(n, 5, 10, 4096, 6, 20, hit, 9)
    assert np.array_equal(got, want)


def test_oversized_request_is_refused():
    bf = _bf()
    f = bf.BloomFilter(1024, 8, 32, 8, 0)
    srv = bf.Server([f], hbm_budget_bytes=1000, max_inflight=2, nstreams=1)
    try:
        keys = torch.zeros(1000, dtype=torch.int64, device="cuda")
        reqs = srv.requests([0], [0], [keys.data_ptr()], [1000], [0], [0])
        res = srv.replay(reqs)
        assert res[0].status == bf.BF_ENOMEM
    finally:
        srv.close()
        f.close()


def _dense_scenario(nfilters=8, nreq=48, seed=31):
    """Served mix whose adds take the partitioned construction: 4-16 MiB
    filters, adds of 2-4 M keys (above the measured automatic crossover,
    about 1.7 M keys at 16 MiB), lookups of 10^3 - 2 * 10^6 keys, one add per
    three requests, all arriving within a few hundred microseconds."""
    g = workloads.rng(seed)
    block = 32
    sizes = workloads.log_uniform_sizes(nfilters, 4 << 20, 16 << 20, block, seed + 1)
    params = [dict(num_blocks=int(sz) // block, words_per_block=8, word_bits=32, k=8, seed=700 + i)
              for i, sz in enumerate(sizes)]
    prepop = [workloads.splitmix64(1900 + i, 0, int(sz) // 4) for i, sz in enumerate(sizes)]
    ops = np.where(g.random(nreq) < 1 / 3, 0, 1)
    filt = g.integers(0, nfilters, size=nreq)
    lo_hi = np.where(ops == 0, 2e6, 1e3), np.where(ops == 0, 4e6, 2e6)
    ns = np.exp(np.log(lo_hi[0]) + g.random(nreq) * (np.log(lo_hi[1]) - np.log(lo_hi[0]))).astype(np.int64)
    keys, starts = [], [0]
    for i in range(nreq):
        f = int(filt[i])
        if ops[i] == 0:
            kk = workloads.splitmix64(15000 + i, 0, int(ns[i]))
        else:
            kk = workloads.mixed_queries(int(ns[i]), 1900 + f, 0, prepop[f].size, 17000 + i, 0, 0.5,
                                         18000 + i)
        keys.append(kk)
        starts.append(starts[-1] + int(ns[i]))
    arrivals = np.cumsum(g.exponential(5_000, size=nreq)).astype(np.int64)
    return params, prepop, ops, filt, ns, np.concatenate(keys), np.array(starts), arrivals


def _expected_by_filter(params, prepop, ops, filt, ns, keys, starts):
    """The sequential oracle replay, one host thread per filter (filters are
    independent; each replays its own requests in submission order)."""
    from oracle import parallel as oracle_par

    out = np.zeros(keys.size, dtype=np.uint8)

    def replay(j):
        r = oracle.OracleFilter(**params[j])
        r.add(prepop[j])
        for i in np.flatnonzero(filt == j):
            a, b = starts[i], starts[i + 1]
            if ops[i] == 0:
                r.add(keys[a:b])
            else:
                out[a:b] = r.contains(keys[a:b])
        return r.bytes

    words = oracle_par.per_filter(list(range(len(params))), replay)
    return words, out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("cfg", [dict(), dict(nstreams=3, max_inflight=4)], ids=["default", "few_slots"])
def test_served_partitioned_adds_equal_sequential_oracle(cfg):
    bf = _bf()
    sc = _dense_scenario()
    params, prepop, ops, filt, ns, keys, starts, arrivals = sc
    # every served add takes the partitioned construction (host-only query)
    probes = [bf.BloomFilter(**p) for p in params]
    try:
        for i in np.flatnonzero(ops == 0):
            assert probes[int(filt[i])].add_strategy(int(ns[i])) == bf.BF_STRATEGY_PARTITIONED
    finally:
        for pr in probes:
            pr.close()
    log(f"serve dense cfg={cfg}: {len(ops)} requests ({int((ops == 0).sum())} partitioned adds), "
        f"{keys.size} keys")
    want_words, want_out = _expected_by_filter(params, prepop, ops, filt, ns, keys, starts)
    res, stats, out, words = _run(*sc, serial=False, **cfg)
    assert all(r.status == 0 for r in res)
    mask = np.repeat(ops == 1, ns)
    assert np.array_equal(out[mask], want_out[mask])
    for i in range(len(params)):
        assert np.array_equal(words[i], want_words[i]), i
    # requests overlapped on the device
    assert stats.peak_inflight_launches > 1
