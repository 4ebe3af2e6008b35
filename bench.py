#!/usr/bin/env python3
"""Benchmark: bulk add + bulk contains on a 1 GiB DRAM-resident sectorized
Bloom filter on one MI355X, against a random-access bound measured on the
same GPU.

One step = clear the filter, add 2^28 uniform uint64 keys, then look up
2^28 queries at 0 %, 50 % and 100 % hit ratio (256-bit blocks of 8 x 32-bit
words, k = 8, 2^25 blocks).  The value is keys processed per second over the
whole step (adds + lookups), inputs already resident in HBM.

Beside it, in the same run: the random-access bounds of this GPU (the
denominators), a 1 GiB streaming copy, the paper's direct construction
timed against the atomic-OR bound, a bounded served leg (Poisson requests
at 0.9x and 2x the serial capacity: served and serial p50 / p99 and their
throughput ratio), the batched leg (4096 filters, one graph launch per op
against one plain launch per filter), and the CPU oracle on one core and on
every core of the host.

Prints one JSON line, e.g.
  python bench.py --steps 20 --warmup 3
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gkeys/s add+contains, 1 GiB blocked BF, % random-gather bound; p99 served"
PEAK_HBM_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")
# the timed kernels (lookups; direct and partitioned adds) and their mappings
KERNEL_SOURCES = ["bf_kernels.hpp", "bf_hash.hpp", "bf_tuned_defaults.inc", "bf_partition.hpp"]


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2512_15595_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse_mapping(text: str | None):
    if not text:
        return None
    parts = [int(x) for x in text.split(",")]
    while len(parts) < 5:
        parts.append(0)
    return parts


class Timer:
    """HIP events on torch's current stream (the stream the kernels run on)."""

    def __init__(self, torch):
        self.torch = torch
        self.start = torch.cuda.Event(enable_timing=True)
        self.stop = torch.cuda.Event(enable_timing=True)

    def __enter__(self):
        self.start.record()
        return self

    def __exit__(self, *exc):
        self.stop.record()

    def ms(self) -> float:
        return self.start.elapsed_time(self.stop)


def measure_bounds(torch, nbytes: int, seg: int, n_access: int, reps: int = 3) -> dict:
    """Random-access rates (G accesses/s) over an nbytes buffer."""
    import ctypes

    from paper_2512_15595_amd import bf as bfmod

    lib = ctypes.CDLL(bfmod.LIB_PATH)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    lib.bfb_random_read.argtypes = [vp, u64, u32, u32, u64, u32, vp, vp]
    lib.bfb_random_atomic_or.argtypes = [vp, u64, u32, u32, u64, u32, vp]
    lib.bfb_gups.argtypes = [vp, u64, u64, u32, vp]
    lib.bfb_fill_random_index.argtypes = [vp, u64, u64, u32, vp]
    lib.bfb_random_read_indexed.argtypes = [vp, u64, u32, vp, u64, vp, vp]
    lib.bfb_random_read_policy.argtypes = [vp, u64, u32, u32, u64, u32, vp, vp]

    stream = torch.cuda.current_stream().cuda_stream
    buf = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    idx = torch.empty(n_access, dtype=torch.int64, device="cuda")
    out = torch.empty(n_access, dtype=torch.uint8, device="cuda")
    rc = lib.bfb_fill_random_index(idx.data_ptr(), n_access, nbytes // seg, 77, stream)
    assert rc == 0

    def best(fn):
        rates = []
        for r in range(reps):
            with Timer(torch) as t:
                rc = fn(r)
            assert rc == 0, rc
            torch.cuda.synchronize()
            rates.append(n_access / (t.ms() * 1e-3) / 1e9)
        return max(rates)

    res = {}
    for s_bytes, lanes in ((8, 1), (seg, 1), (seg, 2)):
        res[f"read_{s_bytes}B_x{lanes}"] = best(
            lambda r, s_bytes=s_bytes, lanes=lanes: lib.bfb_random_read(
                buf.data_ptr(), nbytes, s_bytes, lanes, n_access, 1000 + r, sink.data_ptr(), stream))
    # the same reads issued with explicit cache policies, eight loads in
    # flight per thread (segments of 32 or 128 bytes only)
    if seg in (32, 128):
        for pol, name in ((1, "nt"), (2, "sc1"), (3, "sc0sc1"), (4, "ntsc1")):
            res[f"read_{seg}B_{name}"] = best(
                lambda r, pol=pol: lib.bfb_random_read_policy(
                    buf.data_ptr(), nbytes, seg, pol, n_access, 1500 + r, sink.data_ptr(), stream))
    res[f"read_{seg}B_indexed"] = best(
        lambda r: lib.bfb_random_read_indexed(buf.data_ptr(), nbytes, seg, idx.data_ptr(), n_access,
                                              out.data_ptr(), stream))
    res["gups_8B"] = best(lambda r: lib.bfb_gups(buf.data_ptr(), nbytes, n_access, 2000 + r, stream))
    for s_bytes, lanes in ((8, 1), (seg, 1), (seg, seg // 8)):
        res[f"atomic_or_{s_bytes}B_x{lanes}"] = best(
            lambda r, s_bytes=s_bytes, lanes=lanes: lib.bfb_random_atomic_or(
                buf.data_ptr(), nbytes, s_bytes, lanes, n_access, 3000 + r, stream))
    del buf, idx, out
    torch.cuda.empty_cache()
    read_keys = [k for k in res if k.startswith("read_")]
    # a direct add is one random atomic-OR group per key: its bound is the
    # best random atomic-OR rate (8-byte words, or the block's segment
    # covered by one or several lanes); GUPS (load + store, not atomic) is
    # reported beside it
    write_keys = [k for k in res if k.startswith("atomic_")]
    return {
        "rates_g_per_s": {k: round(v, 3) for k, v in res.items()},
        "contains_bound": max(res[k] for k in read_keys),
        "contains_bound_shape": max(read_keys, key=lambda k: res[k]),
        "add_bound": max(res[k] for k in write_keys),
        "add_bound_shape": max(write_keys, key=lambda k: res[k]),
    }


def streaming_copy(torch, nbytes: int) -> float:
    """One streaming copy of nbytes (the byte-counter calibration kernel);
    returns read+write GB/s of the last of three runs."""
    import ctypes

    from paper_2512_15595_amd import bf as bfmod

    lib = ctypes.CDLL(bfmod.LIB_PATH)
    lib.bfb_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    for _ in range(3):
        with Timer(torch) as t:
            assert lib.bfb_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream) == 0
        torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / (t.ms() * 1e-3) / 1e9


def committed_traffic(kernel: str, sample_keys: int):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(PROFILE_DIR, "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    if data.get("kernel_source_hash") != kernel_source_hash():
        return None
    entry = data.get("kernels", {}).get(kernel)
    if not entry or entry.get("keys_per_launch") != sample_keys:
        return None
    return entry.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline_all_cores(adds, queries, params, n: int, single_bytes) -> dict:
    """The same oracle on every host core the process may use (at most 16,
    the box's share): words built block range by block range and lookups
    answered slice by slice, one unchanged single-threaded oracle call per
    thread; the words must equal the single-thread run's."""
    import numpy as np

    from oracle import parallel

    p = params
    threads = parallel.workers()
    t0 = time.perf_counter()
    words = parallel.filter_words(p["num_blocks"], p["words_per_block"], p["word_bits"], p["k"],
                                  p["seed"], adds[:n], threads=threads)
    t_add = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = parallel.contains(words, p["num_blocks"], p["words_per_block"], p["word_bits"], p["k"],
                          p["seed"], queries[:n], threads=threads)
    t_contains = time.perf_counter() - t0
    same = bool(np.array_equal(words, single_bytes)) if single_bytes is not None else None
    return {
        "value": round(2 * n / (t_add + t_contains) / 1e9, 6),
        "unit": "Gkeys/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"{n} adds then {n} lookups (50% hits) on the full 1 GiB filter in host memory, "
                   f"{threads} threads; add {n / t_add / 1e6:.2f} Mkeys/s, contains "
                   f"{n / t_contains / 1e6:.2f} Mkeys/s, {int(np.sum(r))} positives"),
        "words_equal_single_thread": same,
    }


def cpu_baseline(adds, queries, params, budget_s: float, keep_words: bool = False):
    """The CPU oracle (single thread) on a bounded sample of the workload.
    Returns the summary, the sample size and (keep_words) the oracle bytes."""
    import numpy as np

    import oracle

    ref = oracle.OracleFilter(params["num_blocks"], params["words_per_block"],
                              params["word_bits"], params["k"], params["seed"])
    # calibrate on a small slice, then size the sample to the time budget
    probe = 1 << 16
    t0 = time.perf_counter()
    ref.add(adds[:probe])
    ref.contains(queries[:probe])
    per_key = (time.perf_counter() - t0) / (2 * probe)
    n = int(min(adds.size, max(probe, budget_s / per_key / 2)))
    n = 1 << max(16, n.bit_length() - 1)
    ref.clear()
    t0 = time.perf_counter()
    ref.add(adds[:n])
    t_add = time.perf_counter() - t0
    t0 = time.perf_counter()
    r = ref.contains(queries[:n])
    t_contains = time.perf_counter() - t0
    words = ref.bytes if keep_words else None
    del ref
    return {
        "value": round(2 * n / (t_add + t_contains) / 1e9, 6),
        "unit": "Gkeys/s",
        "cores": 1,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"{n} adds then {n} lookups (50% hits) on the full 1 GiB filter in host memory; "
                   f"add {n / t_add / 1e6:.2f} Mkeys/s, contains {n / t_contains / 1e6:.2f} Mkeys/s, "
                   f"{int(np.sum(r))} positives"),
    }, n, words


def run_batched(args) -> dict:
    """Many filters: one persistent graph launch per op against one plain
    launch per filter, same filters, keys and results."""
    import numpy as np
    import torch

    from paper_2512_15595_amd import workloads
    from paper_2512_15595_amd.bf import BF_OP_ADD, BF_OP_CONTAINS, BatchPlan, BloomFilter

    nf, total = args.batch_filters, 1 << args.log2_keys
    s, S, k = args.words_per_block, args.word_bits, args.k
    block = s * S // 8
    log(f"[bench] batched workload: {nf} filters, {total} keys; generating")
    sizes, offsets, keys, queries = workloads.batched_workload(nf, total, block_bytes=block)
    filters = [BloomFilter(int(sz) // block, s, S, k, i) for i, sz in enumerate(sizes)]
    d_keys = torch.from_numpy(keys.view(np.int64)).to("cuda")
    d_q = torch.from_numpy(queries.view(np.int64)).to("cuda")
    out_b = torch.zeros(queries.size, dtype=torch.uint8, device="cuda")
    out_p = torch.zeros(queries.size, dtype=torch.uint8, device="cuda")
    add = BatchPlan(BF_OP_ADD, filters, d_keys, offsets)
    con = BatchPlan(BF_OP_CONTAINS, filters, d_q, offsets, out_b)
    con_p = BatchPlan(BF_OP_CONTAINS, filters, d_q, offsets, out_p)
    torch.cuda.synchronize()

    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            with Timer(torch) as t:
                fn()
            torch.cuda.synchronize()
            ts.append(t.ms())
        return float(np.median(ts))

    for _ in range(max(1, args.warmup)):
        add.launch(); con.launch(); add.launch_per_filter(); con_p.launch_per_filter()
    torch.cuda.synchronize()
    reps = max(3, args.steps)
    ms = {
        "add_graph": timed(add.launch, reps),
        "contains_graph": timed(con.launch, reps),
        "add_direct": timed(add.launch_direct, reps),
        "contains_direct": timed(con.launch_direct, reps),
        "add_per_filter": timed(add.launch_per_filter, reps),
        "contains_per_filter": timed(con_p.launch_per_filter, reps),
    }
    same = bool(torch.equal(out_b, out_p))
    hits = int(out_b.sum().item())
    info_a, info_c = add.info(), con.info()
    batched = ms["add_graph"] + ms["contains_graph"]
    plain = ms["add_per_filter"] + ms["contains_per_filter"]
    res = {
        "metric": "Gkeys/s batched add+contains over many filters (one graph launch per op)",
        "value": round(2 * total / (batched * 1e-3) / 1e9, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": reps,
        "warmup": args.warmup,
        "higher_is_better": True,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"batched_{nf}_filters_4KiB_16MiB_zipf1.1_sbf_{s}x{S}_k{k}",
                   "filters": nf, "filter_bytes_total": int(sizes.sum()), "keys": total,
                   "grid": info_a.grid, "tiles_add": info_a.ntiles, "tiles_contains": info_c.ntiles,
                   "tiles_per_class_add": list(info_a.tiles_per_class),
                   "mapping_per_class_add": [info_a.mapping[c].as_dict() for c in range(3)],
                   "mapping_per_class_contains": [info_c.mapping[c].as_dict() for c in range(3)]},
        "ms": {key: round(v, 4) for key, v in ms.items()},
        "plain_per_filter_gkeys_s": round(2 * total / (plain * 1e-3) / 1e9, 3),
        "speedup_vs_per_filter": round(plain / batched, 3),
        "add_speedup": round(ms["add_per_filter"] / ms["add_graph"], 3),
        "contains_speedup": round(ms["contains_per_filter"] / ms["contains_graph"], 3),
        "results_equal_batched_vs_per_filter": same,
        "positives": hits,
    }
    for plan in (add, con, con_p):
        plan.close()
    for f in filters:
        f.close()
    return res


def water_fill_sizes(n: int, total: int, lo: int, hi: int, align: int, seed: int):
    """Log-uniform sizes on [lo, hi], scaled to sum to `total` with every
    size clipped to hi (scale, clip, repeat), rounded down to `align`."""
    import numpy as np

    from paper_2512_15595_amd import workloads

    sizes = workloads.log_uniform_sizes(n, lo, hi, align, seed).astype(np.float64)
    for _ in range(100):
        free = sizes < hi
        rest = total - sizes[~free].sum()
        sizes[free] *= rest / sizes[free].sum()
        sizes = np.minimum(sizes, hi)
        if abs(sizes.sum() - total) < align * n:
            break
    return (np.floor(sizes / align) * align).astype(np.int64)


def latency_summary(res, ns) -> dict:
    import numpy as np

    arr = np.array([r.arrival_ns for r in res], dtype=np.float64)
    done = np.array([r.complete_ns for r in res], dtype=np.float64)
    lat = (done - arr) / 1e6
    span = (done.max() - arr.min()) / 1e9
    return {"throughput_gkeys_s": round(float(np.sum(ns)) / span / 1e9, 3),
            "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_ms": round(float(lat.mean()), 3), "makespan_s": round(span, 4)}


def run_serve(args) -> dict:
    """64 device-resident filters (32 GiB), a Poisson stream of contains and
    add requests (9:1, sizes log-uniform 1e3..1.6e7 keys, 50 % hits), served
    with continuous batching under a 48 GiB working budget, against serial
    execution of the same schedule."""
    import ctypes

    import numpy as np
    import torch

    from paper_2512_15595_amd import bf as bfmod
    from paper_2512_15595_amd import workloads
    from paper_2512_15595_amd.bf import BloomFilter, Server

    lib = ctypes.CDLL(bfmod.LIB_PATH)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    lib.bfb_fill_splitmix64.argtypes = [vp, u64, u64, u64, vp]
    lib.bfb_fill_mixed_queries.argtypes = [vp, u64, u64, u64, u32, u64, u64, u32, u64, vp]
    stream = torch.cuda.current_stream().cuda_stream
    s, S, k = args.words_per_block, args.word_bits, args.k
    block = s * S // 8
    nf = args.serve_filters
    total_bytes = args.serve_total_gib << 30
    sizes = water_fill_sizes(nf, total_bytes, 64 << 20, 1 << 30, block, 5)
    log(f"[bench] serve: {nf} filters, {sizes.sum() / 2**30:.2f} GiB; pre-populating at 32 bits/key")
    filters = [BloomFilter(int(sz) // block, s, S, k, 100 + i) for i, sz in enumerate(sizes)]
    chunk = 1 << 27
    buf = torch.empty(chunk, dtype=torch.int64, device="cuda")
    prepop = [int(sz) // 4 for sz in sizes]
    for i, f in enumerate(filters):
        for first in range(0, prepop[i], chunk):
            m = min(chunk, prepop[i] - first)
            assert lib.bfb_fill_splitmix64(buf.data_ptr(), m, 900 + i, first, stream) == 0
            f.add(buf[:m])
    del buf
    max_n = 16_000_000
    pool_n = max_n + 1024
    pools = torch.empty((nf, pool_n), dtype=torch.int64, device="cuda")
    outs = torch.empty((nf, pool_n), dtype=torch.uint8, device="cuda")
    for i in range(nf):
        assert lib.bfb_fill_mixed_queries(pools[i].data_ptr(), pool_n, 900 + i, 0, min(prepop[i], 2**32 - 1),
                                          3000 + i, 0, 1 << 31, 4000 + i, stream) == 0
    torch.cuda.synchronize()
    log("[bench] serve: filters and request pools resident")

    g = workloads.rng(11)
    nreq = args.serve_requests
    ops = np.where(g.random(nreq) < 0.1, 0, 1)
    filt = g.integers(0, nf, size=nreq)
    ns = np.exp(np.log(1e3) + g.random(nreq) * (np.log(1.6e7) - np.log(1e3))).astype(np.int64)
    offs = (g.integers(0, pool_n - ns) // 2) * 2
    kp = [pools[filt[i]].data_ptr() + 8 * int(offs[i]) for i in range(nreq)]
    op_ = [outs[filt[i]].data_ptr() + int(offs[i]) if ops[i] == 1 else 0 for i in range(nreq)]
    budget = (48 << 30) - int(sizes.sum())
    srv = Server(filters, hbm_budget_bytes=budget, max_inflight=args.serve_inflight,
                 nstreams=args.serve_streams, coalesce_max_keys=args.serve_coalesce_keys)

    # serial capacity: every request present at time 0, one after another
    ncap = min(nreq, 2000)
    reqs0 = srv.requests(ops[:ncap], filt[:ncap], kp[:ncap], ns[:ncap], op_[:ncap], np.zeros(ncap))
    cap_res = srv.replay(reqs0, serial=True)
    cap = latency_summary(cap_res, ns[:ncap])["throughput_gkeys_s"] * 1e9
    log(f"[bench] serve: serial capacity {cap / 1e9:.2f} Gkeys/s")
    # the device's capacity for this mix: the same requests all present at
    # time 0, served with overlap; then lookups alone and adds alone (their
    # rates at these request sizes bound any mix: 1 / (share / rate summed))
    sat = latency_summary(srv.replay(reqs0), ns[:ncap])["throughput_gkeys_s"]
    per_op = {}
    for opv, name in ((1, "contains"), (0, "add")):
        idx = np.flatnonzero(ops[:ncap] == opv)
        r = srv.requests(ops[idx], filt[idx], [kp[i] for i in idx], ns[idx], [op_[i] for i in idx],
                         np.zeros(idx.size))
        per_op[name] = latency_summary(srv.replay(r), ns[idx])["throughput_gkeys_s"]
    key_share_add = float(ns[:ncap][ops[:ncap] == 0].sum() / ns[:ncap].sum())
    ceiling = 1.0 / (key_share_add / per_op["add"] + (1.0 - key_share_add) / per_op["contains"])
    log(f"[bench] serve: saturated {sat:.2f} Gkeys/s; contains alone {per_op['contains']:.2f}, "
        f"adds alone {per_op['add']:.2f}; mix ceiling {ceiling:.2f}")
    runs = {}
    mean_n = float(ns.mean())
    for load in args.serve_loads:
        rate = load * cap / mean_n  # requests per second
        arr = np.cumsum(workloads.rng(20 + int(load * 10)).exponential(1.0 / rate, size=nreq)) * 1e9
        reqs = srv.requests(ops, filt, kp, ns, op_, arr.astype(np.int64))
        served = latency_summary(srv.replay(reqs), ns)
        serial = latency_summary(srv.replay(reqs, serial=True), ns)
        runs[str(load)] = {"served": served, "serial": serial,
                           "throughput_ratio": round(served["throughput_gkeys_s"] / serial["throughput_gkeys_s"], 3),
                           "p99_ratio_serial_over_served": round(serial["p99_ms"] / max(served["p99_ms"], 1e-9), 3)}
        log(f"[bench] serve load {load}: {runs[str(load)]}")
    st = srv.stats().as_dict()
    srv.close()
    hi_load = runs[str(max(args.serve_loads))]
    res = {
        "metric": "served Gkeys/s and p50/p99 latency, 64 filters x 32 GiB, Poisson contains:add 9:1",
        "value": hi_load["served"]["throughput_gkeys_s"],
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"serve_{nf}_filters_{sizes.sum() >> 30}GiB_sbf_{s}x{S}_k{k}",
                   "requests": nreq, "mean_keys_per_request": round(mean_n), "hbm_budget_bytes": budget,
                   "max_inflight": args.serve_inflight, "streams": args.serve_streams,
                   "coalesce_max_keys": args.serve_coalesce_keys},
        "serial_capacity_gkeys_s": round(cap / 1e9, 3),
        "saturated": {"served_gkeys_s": sat, "contains_only_gkeys_s": per_op["contains"],
                      "adds_only_gkeys_s": per_op["add"], "add_key_share": round(key_share_add, 4),
                      "mix_ceiling_gkeys_s": round(ceiling, 3)},
        "loads": runs,
        "server_stats": st,
    }
    for f in filters:
        f.close()
    return res


CACHE_LAYOUTS = ("rbbf_1x64", "rbbf_1x32", "sbf_8x32", "classic")


def make_cache_filter(bfmod, layout: str, nbytes: int, k: int, seed: int):
    """The four layouts of the cache-regime sweep at one size.  An 8-word
    sectorized filter needs k >= 8; below that the cache-sectorized filter
    with the most groups that divide k takes its place (z = 4 for k = 4,
    z = 2 for k = 6)."""
    if layout == "rbbf_1x64":
        return bfmod.BloomFilter(nbytes // 8, 1, 64, k, seed), layout
    if layout == "rbbf_1x32":
        return bfmod.BloomFilter(nbytes // 4, 1, 32, k, seed), layout
    if layout == "sbf_8x32":
        if k >= 8:
            return bfmod.BloomFilter(nbytes // 32, 8, 32, k, seed), layout
        z = 4 if k % 4 == 0 else 2
        return bfmod.CacheSectorizedFilter(nbytes // 32, 8, 32, z, k, seed), f"csbf_8x32_z{z}"
    if layout == "classic":
        return bfmod.ClassicFilter(nbytes * 8, k, seed), layout
    raise ValueError(layout)


def run_cache(args) -> dict:
    """Cache-resident regime and layout sweep: filters of 1 MiB .. 256 MiB,
    k in {4, 6, 8, 12, 16}, register-blocked (one 64- or 32-bit word),
    sectorized (8 x 32-bit) and classic layouts.  Throughput: add of N
    uniform keys into a cleared filter, then lookup of the same N keys (all
    present), N = 2^log2_keys, timed with HIP events on the launch stream.
    Accuracy at matched bits per key c in {8, 16, 32}: n = m / c distinct
    keys inserted into a 64 MiB filter, 2^22 fresh keys looked up.  A second
    throughput pass uses 2-bit packed 31-mers of a random sequence with 10 %
    repeated segments (one size, k = 8)."""
    import ctypes

    import numpy as np
    import torch

    from paper_2512_15595_amd import bf as bfmod
    from paper_2512_15595_amd import workloads

    lib = ctypes.CDLL(bfmod.LIB_PATH)
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    lib.bfb_fill_splitmix64.argtypes = [vp, u64, u64, u64, vp]
    stream = torch.cuda.current_stream().cuda_stream
    n = 1 << args.cache_log2_keys
    keys = torch.empty(n, dtype=torch.int64, device="cuda")
    assert lib.bfb_fill_splitmix64(keys.data_ptr(), n, 31, 0, stream) == 0
    out = torch.empty(n, dtype=torch.uint8, device="cuda")
    sizes = [1 << e for e in args.cache_log2_sizes]
    ks = tuple(args.cache_ks)
    layouts = tuple(args.cache_layouts)

    def timed(fn, reps):
        fn()
        t = Timer(torch)
        with t:
            for _ in range(reps):
                fn()
        torch.cuda.synchronize()
        return t.ms() / reps

    def throughput(f, qkeys, reps):
        f.clear()
        add_ms = timed(lambda: f.add(qkeys), reps)
        con_ms = timed(lambda: f.contains(qkeys, out=out[: qkeys.numel()]), reps)
        found = int(out[: qkeys.numel()].sum().item())
        assert found == qkeys.numel(), "false negative"
        return qkeys.numel() / add_ms / 1e6, qkeys.numel() / con_ms / 1e6

    rows = []
    for nbytes in sizes:
        for layout in layouts:
            for k in ks:
                f, name = make_cache_filter(bfmod, layout, nbytes, k, 7)
                try:
                    a, c = throughput(f, keys, args.steps)
                finally:
                    f.close()
                rows.append({"layout": name, "bytes": nbytes, "k": k, "add_gkeys_s": round(a, 3),
                             "contains_gkeys_s": round(c, 3)})
                log(f"[cache] {name} {nbytes >> 20} MiB k={k}: add {a:.2f} contains {c:.2f} Gkeys/s")

    fpr_rows = []
    fbytes = 64 << 20
    fresh = torch.empty(1 << 22, dtype=torch.int64, device="cuda")
    assert lib.bfb_fill_splitmix64(fresh.data_ptr(), fresh.numel(), 32, 0, stream) == 0
    for c_bits in ((8, 16, 32) if args.cache_fpr else ()):
        ins = fbytes * 8 // c_bits
        assert ins <= n, "the accuracy pass needs 2^26 keys"
        for layout in layouts:
            for k in ks:
                f, name = make_cache_filter(bfmod, layout, fbytes, k, 9)
                try:
                    f.add(keys[:ins])
                    f.contains(fresh, out=out[: fresh.numel()])
                    fp = int(out[: fresh.numel()].sum().item())
                finally:
                    f.close()
                eq1 = (1 - np.exp(-k / c_bits)) ** k
                fpr_rows.append({"layout": name, "bits_per_key": c_bits, "k": k,
                                 "fpr": fp / fresh.numel(), "classic_eq1": float(eq1)})

    kmer_rows = []
    kmer_sizes = (1 << 22, 1 << 28) if args.cache_kmer else ()
    if kmer_sizes:
        kmers = workloads.kmer_keys(n + 30, 33)
        d_kmers = torch.from_numpy(kmers.view(np.int64)).to("cuda")
    for nbytes in kmer_sizes:
        for layout in layouts:
            f, name = make_cache_filter(bfmod, layout, nbytes, 8, 11)
            try:
                a, c = throughput(f, d_kmers, args.steps)
            finally:
                f.close()
            kmer_rows.append({"layout": name, "bytes": nbytes, "k": 8, "add_gkeys_s": round(a, 3),
                              "contains_gkeys_s": round(c, 3)})

    sbf = [r["contains_gkeys_s"] for r in rows if r["layout"] == "sbf_8x32" and r["k"] == 8]
    best = max(sbf) if sbf else None
    return {
        "metric": "Gkeys/s add / contains, cache-resident filters, per layout",
        "value": best,
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "cache_regime_1MiB_256MiB", "keys_per_op": n,
                   "sizes_bytes": sizes, "k": list(ks), "layouts": list(layouts),
                   "value_is": "best sbf_8x32 k=8 contains rate over sizes"},
        "throughput": rows,
        "fpr_64MiB": fpr_rows,
        "kmer31_throughput": kmer_rows,
    }


def run_breakdown(args) -> dict:
    """Optimization breakdown (the analog of the paper's Sec. V-E figure) at
    the paper's parameters, S = 64, k = 16, B = 256 (s = 4), for an
    L2-resident (2 MiB) and an HBM-resident (1 GiB) filter: add then lookup of
    2^log2_keys uniform keys, each step of the sequence measured on its own:
      1 classic filter of the same size, direct (atomic) construction;
      2 sectorized, chained pattern hashing, one lane per key, direct add;
      3 + multiplicative pattern hashing (one lane per key, direct add);
      4 + horizontal add with the hash shared by the group (best THETA in
        {2, 4}, direct add); lookup keeps one lane per key;
      5 + MI355X: keys per lane and, for dense adds, partitioned construction
        (the library defaults)."""
    import ctypes

    import torch

    from paper_2512_15595_amd import bf as bfmod

    lib = ctypes.CDLL(bfmod.LIB_PATH)
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    lib.bfb_fill_splitmix64.argtypes = [vp, u64, u64, u64, vp]
    stream = torch.cuda.current_stream().cuda_stream
    n = 1 << args.breakdown_log2_keys
    keys = torch.empty(n, dtype=torch.int64, device="cuda")
    assert lib.bfb_fill_splitmix64(keys.data_ptr(), n, 41, 0, stream) == 0
    out = torch.empty(n, dtype=torch.uint8, device="cuda")
    s, S, k = 4, 64, 16
    A, C = bfmod.BF_OP_ADD, bfmod.BF_OP_CONTAINS
    DIRECT = bfmod.BF_STRATEGY_DIRECT

    def timed(fn):
        fn()
        t = Timer(torch)
        with t:
            for _ in range(args.steps):
                fn()
        torch.cuda.synchronize()
        return t.ms() / args.steps

    def rates(f):
        f.clear()
        a = n / timed(lambda: f.add(keys)) / 1e6
        c = n / timed(lambda: f.contains(keys, out=out)) / 1e6
        assert int(out.sum().item()) == n, "false negative"
        return a, c

    rows = []
    for nbytes in (2 << 20, 1 << 30):
        b = nbytes // (s * S // 8)
        res = {}
        f = bfmod.ClassicFilter(nbytes * 8, k, 3)
        f.set_mapping(A, strategy=DIRECT)  # the baseline: one atomic per position
        res["1_classic"] = rates(f)
        f.close()
        f = bfmod.ChainedHashFilter(b, s, S, k, 3)
        res["2_sectorized_chained_hash"] = rates(f)
        f.close()
        f = bfmod.BloomFilter(b, s, S, k, 3)
        f.set_mapping(A, 1, s, 1, 0, 0, DIRECT)
        f.set_mapping(C, 1, s, 1)
        res["3_multiplicative_hash"] = rates(f)
        best = None
        for theta in (2, 4):
            f.set_mapping(A, theta, s // theta, 1, 0, 0, DIRECT)
            a, _ = rates(f)
            if best is None or a > best[0]:
                best = (a, theta)
        res["4_horizontal_shared_add"] = (best[0], res["3_multiplicative_hash"][1])
        f.set_mapping(A, 0, 0, 0)
        f.set_mapping(C, 0, 0, 0)
        res["5_mi355x_defaults"] = rates(f)
        info = f.info()
        f.close()
        base = res["1_classic"]
        for step, (a, c) in res.items():
            rows.append({"filter_bytes": nbytes, "step": step, "add_gkeys_s": round(a, 3),
                         "contains_gkeys_s": round(c, 3),
                         "add_vs_classic": round(a / base[0], 2),
                         "contains_vs_classic": round(c / base[1], 2)})
            log(f"[breakdown] {nbytes >> 20} MiB {step}: add {a:.2f} contains {c:.2f} Gkeys/s")
        rows[-2]["theta"] = best[1]
        rows[-1]["mapping"] = {"add": info.mapping[A].as_dict(), "contains": info.mapping[C].as_dict()}
    return {
        "metric": "Gkeys/s add / contains along the optimization sequence",
        "value": rows[-1]["add_gkeys_s"],
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "breakdown_sbf_4x64_k16_2MiB_1GiB", "keys_per_op": n,
                   "value_is": "1 GiB add rate with the library defaults"},
        "rows": rows,
    }


def run_layouts(args) -> dict:
    """Layout tables and the throughput / accuracy frontier at the paper's
    parameters (S = 64, k = 16, N = 10^9 uniform keys, Sec. V-A), for a 1 GiB
    (HBM) and a 32 MiB (Infinity Cache) filter.
    Tables (the analogs of the paper's 1 GB and 32 MB layout tables): for
    B = 64 ... 1024 bits (s = 1 ... 16) and every THETA, PHI = s / THETA, one
    key per lane: lookup of the N keys after adding them, and direct-strategy
    construction (one atomic group per key).
    Frontier: per configuration (sectorized B = 64 ... 1024; cache-sectorized
    B = 512 with z = 2, 4 and B = 1024 with z = 2, 4, 8; classic) the
    false-positive rate after inserting the space- and rate-optimal number of
    distinct keys n = m ln2 / k (Eq. (1)), measured on 2^27 fresh keys, beside
    the best lookup and construction rates over the compiled mappings and the
    library's default (which may construct by partitioning)."""
    import ctypes
    import math

    import torch

    from paper_2512_15595_amd import bf as bfmod

    lib = ctypes.CDLL(bfmod.LIB_PATH)
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    lib.bfb_fill_splitmix64.argtypes = [vp, u64, u64, u64, vp]
    stream = torch.cuda.current_stream().cuda_stream
    n = args.layouts_keys
    keys = torch.empty(n, dtype=torch.int64, device="cuda")
    assert lib.bfb_fill_splitmix64(keys.data_ptr(), n, 51, 0, stream) == 0
    fresh = torch.empty(1 << 27, dtype=torch.int64, device="cuda")
    assert lib.bfb_fill_splitmix64(fresh.data_ptr(), fresh.numel(), 52, 0, stream) == 0
    out = torch.empty(n, dtype=torch.uint8, device="cuda")
    S, k = 64, 16
    A, C = bfmod.BF_OP_ADD, bfmod.BF_OP_CONTAINS
    DIRECT = bfmod.BF_STRATEGY_DIRECT

    def timed(fn):
        fn()
        t = Timer(torch)
        with t:
            for _ in range(args.steps):
                fn()
        torch.cuda.synchronize()
        return t.ms() / args.steps

    def add_rate(f):
        f.clear()
        return n / timed(lambda: f.add(keys)) / 1e6

    def contains_rate(f):
        f.clear()
        f.add(keys)
        r = n / timed(lambda: f.contains(keys, out=out)) / 1e6
        assert int(out.sum().item()) == n, "false negative"
        return r

    def thetas(s, cap):
        t, res = 1, []
        while t <= min(s, cap):
            res.append(t)
            t *= 2
        return res

    tables = []
    for nbytes in (1 << 30, 32 << 20):
        for s in (1, 2, 4, 8, 16):
            b = nbytes // (s * S // 8)
            f = bfmod.BloomFilter(b, s, S, k, 5)
            for theta in thetas(s, 16):
                f.set_mapping(C, theta, s // theta, 1)
                f.set_mapping(A, theta, s // theta, 1, 0, 0, DIRECT)
                row = {"filter_bytes": nbytes, "B": s * S, "theta": theta, "phi": s // theta,
                       "contains_gkeys_s": round(contains_rate(f), 3),
                       "add_direct_gkeys_s": round(add_rate(f), 3)}
                tables.append(row)
                log(f"[layouts] {nbytes >> 20} MiB B={s * S} theta={theta}: "
                    f"contains {row['contains_gkeys_s']} add {row['add_direct_gkeys_s']}")
            f.close()

    def fpr(f, m_bits):
        ins = int(m_bits * math.log(2) / k)
        assert ins <= n
        f.clear()
        f.add(keys[:ins])
        f.contains(fresh, out=out[: fresh.numel()])
        return int(out[: fresh.numel()].sum().item()) / fresh.numel(), ins

    configs = [("sbf", s, None) for s in (1, 2, 4, 8, 16)]
    configs += [("csbf", 8, z) for z in (2, 4)] + [("csbf", 16, z) for z in (2, 4, 8)]
    configs += [("classic", None, None)]
    frontier = []
    for nbytes in (1 << 30, 32 << 20):
        for kind, s, z in configs:
            if kind == "classic":
                f = bfmod.ClassicFilter(nbytes * 8, k, 7)
                maps = [(1, 1, 2)]
                label = "classic"
            elif kind == "sbf":
                f = bfmod.BloomFilter(nbytes // (s * S // 8), s, S, k, 7)
                maps = [(t, s // t, kt) for t in thetas(s, 16) for kt in (1, 2, 4)]
                label = f"sbf_B{s * S}"
            else:
                f = bfmod.CacheSectorizedFilter(nbytes // (s * S // 8), s, S, z, k, 7)
                maps = [(t, s // t, 1) for t in thetas(z, 16)] + [(1, s, 2)]
                label = f"csbf_B{s * S}_z{z}"
            rate, ins = fpr(f, nbytes * 8)
            best_c = best_a = 0.0
            for theta, phi, kt in maps:
                f.set_mapping(C, theta, phi, kt)
                f.set_mapping(A, theta, phi, kt, 0, 0, DIRECT)
                best_c = max(best_c, contains_rate(f))
                best_a = max(best_a, add_rate(f))
            f.set_mapping(A, 0, 0, 0)
            f.set_mapping(C, 0, 0, 0)
            row = {"filter_bytes": nbytes, "config": label, "fpr": rate, "inserted": ins,
                   "best_contains_gkeys_s": round(best_c, 3), "best_add_direct_gkeys_s": round(best_a, 3),
                   "default_add_gkeys_s": round(add_rate(f), 3),
                   "default_contains_gkeys_s": round(contains_rate(f), 3)}
            f.close()
            frontier.append(row)
            log(f"[frontier] {nbytes >> 20} MiB {label}: fpr {rate:.3g} contains {row['best_contains_gkeys_s']} "
                f"add {row['best_add_direct_gkeys_s']} / default {row['default_add_gkeys_s']}")
    return {
        "metric": "Gkeys/s per layout (S = 64, k = 16) and FPR at the optimal load",
        "value": max(r["default_contains_gkeys_s"] for r in frontier if r["filter_bytes"] == 1 << 30),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "layouts_frontier_S64_k16_1GiB_32MiB", "keys_per_op": n,
                   "fresh_lookups_for_fpr": fresh.numel(),
                   "value_is": "best default lookup rate at 1 GiB"},
        "tables": tables,
        "frontier": frontier,
    }


def run_parquet(args) -> dict:
    """The Parquet split-block filter (include/bf_parquet.h).  Bulk rates on
    the format's largest filter (128 MiB; 2^27 values, lookups at 50 % hits),
    and the pruning step of a Parquet scan: `literals` values looked up in
    the filter of every row group (1 MiB filters of 2^19 values each, the
    size a writer picks for that many distinct values at 1 % FPR), as one
    batched graph launch against one launch per row group."""
    import ctypes

    import numpy as np
    import torch

    from paper_2512_15595_amd import bf as bfmod
    from paper_2512_15595_amd.bf import BF_OP_ADD, BF_OP_CONTAINS, BatchPlan, ParquetFilter

    lib = ctypes.CDLL(bfmod.LIB_PATH)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    lib.bfb_fill_splitmix64.argtypes = [vp, u64, u64, u64, vp]
    lib.bfb_fill_mixed_queries.argtypes = [vp, u64, u64, u64, u32, u64, u64, u32, u64, vp]
    stream = torch.cuda.current_stream().cuda_stream
    reps = max(3, args.steps)

    def median_ms(fn, before=None):
        ts = []
        for _ in range(reps):
            if before is not None:
                before()
            with Timer(torch) as t:
                fn()
            torch.cuda.synchronize()
            ts.append(t.ms())
        return float(np.median(ts))

    nbytes, n = 128 << 20, 1 << 27
    log(f"[bench] parquet: {n} values into the format's largest filter (128 MiB)")
    vals = torch.empty(n, dtype=torch.int64, device="cuda")
    qs = torch.empty(n, dtype=torch.int64, device="cuda")
    assert lib.bfb_fill_splitmix64(vals.data_ptr(), n, 301, 0, stream) == 0
    assert lib.bfb_fill_mixed_queries(qs.data_ptr(), n, 301, 0, n, 302, 0, 1 << 31, 303, stream) == 0
    out = torch.empty(n, dtype=torch.uint8, device="cuda")
    f = ParquetFilter(nbytes)
    f.add(vals)
    f.contains(qs, out)
    torch.cuda.synchronize()
    add_ms = median_ms(lambda: f.add(vals), before=f.clear)
    con_ms = median_ms(lambda: f.contains(qs, out))
    strategy = f.add_strategy(n)
    f.close()
    del vals, qs, out

    rgs, per_rg, lits = 1024, 1 << 19, 16
    log(f"[bench] parquet pruning: {rgs} row-group filters of 1 MiB, {lits} literals each")
    filters = [ParquetFilter(1 << 20) for _ in range(rgs)]
    vals = torch.empty(rgs * per_rg, dtype=torch.int64, device="cuda")
    assert lib.bfb_fill_splitmix64(vals.data_ptr(), vals.numel(), 311, 0, stream) == 0
    # a literal is a value of its row group with probability 1/16
    qs = torch.empty(rgs * lits, dtype=torch.int64, device="cuda")
    for i in range(rgs):
        assert lib.bfb_fill_mixed_queries(qs[i * lits:].data_ptr(), lits, 311, i * per_rg, per_rg, 312,
                                          i * lits, 1 << 28, 313 + i, stream) == 0
    offs_v = [i * per_rg for i in range(rgs + 1)]
    offs_q = [i * lits for i in range(rgs + 1)]
    out_g = torch.zeros(rgs * lits, dtype=torch.uint8, device="cuda")
    out_p = torch.zeros(rgs * lits, dtype=torch.uint8, device="cuda")
    build = BatchPlan(BF_OP_ADD, filters, vals, offs_v)
    prune = BatchPlan(BF_OP_CONTAINS, filters, qs, offs_q, out_g)
    prune_p = BatchPlan(BF_OP_CONTAINS, filters, qs, offs_q, out_p)
    build.launch()
    prune.launch()
    prune_p.launch_per_filter()
    torch.cuda.synchronize()
    build_ms = median_ms(build.launch, before=lambda: [g.clear() for g in filters])
    graph_ms = median_ms(prune.launch)
    direct_ms = median_ms(prune.launch_direct)
    per_filter_ms = median_ms(prune_p.launch_per_filter)
    hits = out_g.view(rgs, lits).any(dim=1)
    res = {
        "workload": "parquet_sbbf_128MiB_and_pruning_1024_row_groups_1MiB",
        "filter_bytes": nbytes, "values": n,
        "add_gkeys_s": round(n / (add_ms * 1e-3) / 1e9, 3),
        "contains_gkeys_s": round(n / (con_ms * 1e-3) / 1e9, 3),
        "add_strategy": "partitioned" if strategy == bfmod.BF_STRATEGY_PARTITIONED else "direct",
        "ms": {"add": round(add_ms, 4), "contains": round(con_ms, 4)},
        "pruning": {
            "row_groups": rgs, "values_per_row_group": per_rg, "literals_per_row_group": lits,
            "build_gkeys_s": round(rgs * per_rg / (build_ms * 1e-3) / 1e9, 3),
            "graph_us": round(graph_ms * 1e3, 2), "direct_us": round(direct_ms * 1e3, 2),
            "per_filter_us": round(per_filter_ms * 1e3, 2),
            "speedup_vs_per_filter": round(per_filter_ms / graph_ms, 2),
            "direct_speedup_vs_per_filter": round(per_filter_ms / direct_ms, 2),
            "row_groups_per_s": round(rgs / (min(graph_ms, direct_ms) * 1e-3), 1),
            "row_groups_kept": int(hits.sum().item()),
            "results_equal": bool(torch.equal(out_g, out_p)),
        },
    }
    for plan in (build, prune, prune_p):
        plan.close()
    for g in filters:
        g.close()
    return res


def run_bounds(args) -> dict:
    """The random-access microbenchmarks versus footprint (1 MiB .. 4 GiB):
    random aligned 8-byte and 32-byte reads (one and two lanes per segment),
    32-byte reads through an 8 B/access streamed index, GUPS-style 8-byte
    read-modify-writes and random atomic ORs, 2^26 accesses each."""
    import torch

    rows = []
    for lg in args.bounds_log2_bytes:
        b = measure_bounds(torch, 1 << lg, 32, 1 << 26)
        rows.append({"footprint_bytes": 1 << lg, **b["rates_g_per_s"],
                     "contains_bound": round(b["contains_bound"], 3),
                     "add_bound": round(b["add_bound"], 3)})
        log(f"[bounds] 2^{lg} B: read 32 B {b['rates_g_per_s']['read_32B_x1']:.1f}, "
            f"indexed {b['rates_g_per_s']['read_32B_indexed']:.1f}, "
            f"atomic {b['rates_g_per_s']['atomic_or_8B_x1']:.1f} G/s")
    return {
        "metric": "G random accesses/s vs footprint",
        "value": rows[-1]["contains_bound"],
        "unit": "G accesses/s",
        "n_gpus": 1,
        "steps": 3,
        "warmup": 0,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "random_access_bounds_1MiB_4GiB", "accesses": 1 << 26,
                   "value_is": "largest footprint's contains bound"},
        "rows": rows,
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--serve-filters", type=int, default=64)
    ap.add_argument("--serve-total-gib", type=int, default=32)
    ap.add_argument("--serve-requests", type=int, default=6000)
    ap.add_argument("--serve-loads", type=float, nargs="+", default=[0.5, 0.9, 2.0])
    ap.add_argument("--serve-inflight", type=int, default=16)
    ap.add_argument("--serve-streams", type=int, default=8)
    ap.add_argument("--serve-coalesce-keys", type=int, default=65536)
    ap.add_argument("--workload",
                    choices=["dram", "batched", "serve", "cache", "breakdown", "layouts", "bounds", "parquet"],
                    default="dram")
    ap.add_argument("--bounds-log2-bytes", type=int, nargs="+", default=[20, 22, 24, 26, 28, 30, 32])
    ap.add_argument("--layouts-keys", type=int, default=10**9)
    ap.add_argument("--breakdown-log2-keys", type=int, default=26)
    ap.add_argument("--cache-log2-keys", type=int, default=26)
    ap.add_argument("--cache-log2-sizes", type=int, nargs="+", default=list(range(20, 29)))
    ap.add_argument("--cache-ks", type=int, nargs="+", default=[4, 6, 8, 12, 16])
    ap.add_argument("--cache-layouts", type=str, nargs="+", default=list(CACHE_LAYOUTS))
    ap.add_argument("--cache-fpr", type=int, default=1, help="0 skips the accuracy pass")
    ap.add_argument("--cache-kmer", type=int, default=1, help="0 skips the 31-mer pass")
    ap.add_argument("--batch-filters", type=int, default=4096)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2-keys", type=int, default=28)
    ap.add_argument("--filter-log2-bytes", type=int, default=30)
    ap.add_argument("--words-per-block", type=int, default=8)
    ap.add_argument("--word-bits", type=int, default=32)
    ap.add_argument("--k", type=int, default=8)
    ap.add_argument("--map-add", type=str, default=None, help="theta,phi,kt[,atomic_bits,max_wg]")
    ap.add_argument("--map-contains", type=str, default=None, help="theta,phi,kt[,0,max_wg]")
    ap.add_argument("--no-bound", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=12.0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="(the 1 GiB streaming copy now runs by default; kept for old commands)")
    ap.add_argument("--no-copy", action="store_true", help="skip the 1 GiB streaming copy")
    ap.add_argument("--no-direct-add", action="store_true", help="skip the direct-construction timing")
    ap.add_argument("--no-serve", action="store_true", help="skip the served leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched leg")
    ap.add_argument("--no-parquet", action="store_true", help="skip the Parquet split-block leg")
    ap.add_argument("--line-serve-requests", type=int, default=2000,
                    help="requests per load in the served leg of the benchmark line")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU: this library runs on a single MI355X and has no "
              "multi-GPU path; use --gpus 1.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2512_15595_amd import workloads
    from paper_2512_15595_amd.bf import (BF_OP_ADD, BF_OP_CONTAINS, BF_STRATEGY_DIRECT,
                                         BF_STRATEGY_PARTITIONED, BloomFilter)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "batched":
        print(json.dumps(run_batched(args)), flush=True)
        return 0
    if args.workload == "serve":
        print(json.dumps(run_serve(args)), flush=True)
        return 0
    if args.workload == "cache":
        print(json.dumps(run_cache(args)), flush=True)
        return 0
    if args.workload == "breakdown":
        print(json.dumps(run_breakdown(args)), flush=True)
        return 0
    if args.workload == "layouts":
        print(json.dumps(run_layouts(args)), flush=True)
        return 0
    if args.workload == "bounds":
        print(json.dumps(run_bounds(args)), flush=True)
        return 0
    if args.workload == "parquet":
        print(json.dumps(run_parquet(args)), flush=True)
        return 0
    n = 1 << args.log2_keys
    s, S, k = args.words_per_block, args.word_bits, args.k
    block_bytes = s * S // 8
    filter_bytes = 1 << args.filter_log2_bytes
    num_blocks = filter_bytes // block_bytes
    params = dict(num_blocks=num_blocks, words_per_block=s, word_bits=S, k=k, seed=0)
    workload = f"dram_{filter_bytes >> 20}MiB_sbf_{s}x{S}_k{k}"
    log(f"[bench] workload {workload}: {n} adds, 3 x {n} lookups; generating keys")

    t0 = time.perf_counter()
    adds, queries = workloads.dram_workload(n)
    log(f"[bench] keys generated in {time.perf_counter() - t0:.1f}s; uploading")
    d_adds = torch.from_numpy(adds.view(np.int64)).to("cuda")
    d_q = {h: torch.from_numpy(q.view(np.int64)).to("cuda") for h, q in queries.items()}
    d_out = torch.empty(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()

    bounds = None
    if not args.no_bound:
        log("[bench] measuring the random-access bound on a 1 GiB buffer")
        bounds = measure_bounds(torch, filter_bytes, block_bytes, n)
        log(f"[bench] bounds: {bounds}")

    copy_gbs = None
    if not args.no_copy:
        copy_gbs = streaming_copy(torch, 1 << 30)
        log(f"[bench] streaming copy of 1 GiB: {copy_gbs:.0f} GB/s (read + write)")

    f = BloomFilter(num_blocks, s, S, k, 0)
    ma, mc = parse_mapping(args.map_add), parse_mapping(args.map_contains)
    if ma:
        f.set_mapping(BF_OP_ADD, *ma)
    if mc:
        f.set_mapping(BF_OP_CONTAINS, *mc)
    info = f.info()
    mapping = {"add": info.mapping[BF_OP_ADD].as_dict(),
               "contains": info.mapping[BF_OP_CONTAINS].as_dict()}
    add_partitioned = f.add_strategy(n) == BF_STRATEGY_PARTITIONED

    times = {"clear": [], "add": [], "contains": []}

    def step(record: bool):
        tc, ta = Timer(torch), Timer(torch)
        with tc:
            f.clear()
        with ta:
            f.add(d_adds)
        tq = []
        for h in (0, 50, 100):
            t = Timer(torch)
            with t:
                f.contains(d_q[h], out=d_out)
            tq.append(t)
        if record:
            times["clear"].append(tc)
            times["add"].append(ta)
            times["contains"].extend(tq)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps); timing {args.steps} steps")
    whole_start, whole_stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    whole_start.record()
    for _ in range(args.steps):
        step(True)
    whole_stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = whole_start.elapsed_time(whole_stop)

    # check the last step's results: 100 % hits must all be found
    f.contains(d_q[100], out=d_out)
    found = int(d_out.sum().item())
    f.contains(d_q[0], out=d_out)
    fp = int(d_out.sum().item())
    torch.cuda.synchronize()
    assert found == n, f"false negatives: {n - found}"

    # the paper's construction, one atomic-OR group per key (Sec. IV), timed
    # on its own after the steps: a cleared filter, the same keys
    direct_ms = None
    if not args.no_direct_add:
        g = BloomFilter(num_blocks, s, S, k, 0)
        g.set_mapping(BF_OP_ADD, strategy=BF_STRATEGY_DIRECT)
        dts = []
        for _ in range(3):
            g.clear()
            t = Timer(torch)
            with t:
                g.add(d_adds)
            torch.cuda.synchronize()
            dts.append(t.ms())
        direct_ms = float(np.median(dts))
        direct_same = bool(torch.equal(g.words(), f.words()))
        g.close()
        assert direct_same, "direct and partitioned construction differ"

    ms = {key: float(np.mean([t.ms() for t in v])) for key, v in times.items()}
    keys_per_step = 4 * n
    ms_per_step = total_ms / args.steps
    value = keys_per_step / (ms_per_step * 1e-3) / 1e9
    add_rate = n / (ms["add"] * 1e-3) / 1e9
    contains_rate = n / (ms["contains"] * 1e-3) / 1e9

    # dominant kernel = the op with the larger share of a step
    add_share, contains_share = ms["add"], 3 * ms["contains"]
    if add_share >= contains_share:
        dom, per_key, dom_ms = "add", 8 + 2 * block_bytes, ms["add"]
    else:
        dom, per_key, dom_ms = "contains", 8 + block_bytes + 1, ms["contains"]
    achieved = per_key * n / (dom_ms * 1e-3) / 1e9
    traffic = committed_traffic(dom, n)
    roofline = {"bound": "hbm", "kernel": f"bf_{dom}_kernel", "achieved": round(achieved, 1),
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": traffic, "algorithmic_bytes_per_key": per_key,
                "avg_launch_ms": round(dom_ms, 4)}
    if traffic:
        # every random block read fetches a whole 128-byte line: what the
        # memory system moves, against the HBM peak
        roofline["traffic_gbs"] = round(traffic / (dom_ms * 1e-3) / 1e9, 1)
        roofline["traffic_frac_of_peak"] = round(traffic / (dom_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)

    # the default add: a partitioned construction streams keys, records and
    # each touched 64 KiB chunk, so its bound is streaming bandwidth; it is
    # reported by the HBM bytes it moves (counters) against the 1 GiB copy
    add_traffic = committed_traffic("add", n) if add_partitioned else None
    roofline_add = {"bound": "hbm", "strategy": "partitioned" if add_partitioned else "direct",
                    "kernels": ("part_scatter1 + part_scatter2 + part_apply" if add_partitioned
                                else "bf_add_kernel"),
                    "avg_launch_ms": round(ms["add"], 4), "unit": "GB/s",
                    "algorithmic_bytes_per_key": 8 + 2 * block_bytes,
                    "achieved_algorithmic": round((8 + 2 * block_bytes) * n / (ms["add"] * 1e-3) / 1e9, 1),
                    "traffic": add_traffic}
    if add_traffic:
        moved = add_traffic / (ms["add"] * 1e-3) / 1e9
        roofline_add.update({"traffic_bytes_per_key": round(add_traffic / n, 2),
                             "achieved_traffic": round(moved, 1), "peak": PEAK_HBM_GBS,
                             "frac_of_peak": round(moved / PEAK_HBM_GBS, 4)})
        if copy_gbs:
            roofline_add.update({"copy_1GiB": round(copy_gbs, 1),
                                 "frac_of_copy": round(moved / copy_gbs, 4)})

    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": workload,
            "filter_bytes": filter_bytes, "num_blocks": num_blocks, "words_per_block": s,
            "word_bits": S, "k": k, "adds_per_step": n, "lookups_per_step": 3 * n,
            "hit_ratios_pct": [0, 50, 100], "mapping": mapping,
        },
        "add_gkeys_s": round(add_rate, 3),
        "contains_gkeys_s": round(contains_rate, 3),
        "ms": {key: round(v, 4) for key, v in ms.items()},
        "false_positive_rate_0pct_hits": fp / n,
        "wall_s_timed": round(wall, 3),
        "roofline": roofline,
        "roofline_add": roofline_add,
    }
    if direct_ms is not None:
        result["direct_add_gkeys_s"] = round(n / (direct_ms * 1e-3) / 1e9, 3)
        result["ms"]["direct_add"] = round(direct_ms, 4)
    if copy_gbs is not None:
        result["copy_1GiB_gbs"] = round(copy_gbs, 1)
    if bounds:
        result["random_access_bound"] = bounds
        pct = {"contains": round(100 * contains_rate / bounds["contains_bound"], 2)}
        if direct_ms is not None:
            pct["add_direct"] = round(100 * result["direct_add_gkeys_s"] / bounds["add_bound"], 2)
        if add_traffic and copy_gbs:
            pct["add_partitioned_traffic_vs_copy"] = round(100 * roofline_add["frac_of_copy"], 2)
        result["pct_of_bound"] = pct
    f.close()
    del d_adds, d_q, d_out
    torch.cuda.empty_cache()

    if not args.no_serve:
        log("[bench] served leg: Poisson requests at 0.9x and 2x the serial capacity")
        result["served"] = serve_summary(run_serve(argparse.Namespace(
            **{**vars(args), "serve_requests": args.line_serve_requests, "serve_loads": [0.9, 2.0]})))
        torch.cuda.empty_cache()
    if not args.no_batched:
        log("[bench] batched leg: 4096 filters, graph launch vs one launch per filter")
        result["batched"] = batched_summary(run_batched(argparse.Namespace(
            **{**vars(args), "steps": 5, "warmup": 1})))
        torch.cuda.empty_cache()
    if not args.no_parquet:
        log("[bench] parquet leg: the format's largest filter, and row-group pruning")
        result["parquet"] = run_parquet(argparse.Namespace(**{**vars(args), "steps": 5}))
        torch.cuda.empty_cache()

    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample (one core, then all cores)")
        single, n_cpu, single_words = cpu_baseline(adds, queries[50], params, args.cpu_budget_s,
                                                   keep_words=True)
        result["cpu_baseline"] = single
        result["cpu_baseline_all_cores"] = cpu_baseline_all_cores(adds, queries[50], params, n_cpu,
                                                                  single_words)
    print(json.dumps(result), flush=True)
    return 0


def serve_summary(res: dict) -> dict:
    """The served leg's figures for the benchmark line."""
    out = {"workload": res["config"]["workload"], "requests": res["config"]["requests"],
           "serial_capacity_gkeys_s": res["serial_capacity_gkeys_s"], "saturated": res["saturated"]}
    for load, r in res["loads"].items():
        out[f"load_{load}x"] = {
            "served_gkeys_s": r["served"]["throughput_gkeys_s"],
            "serial_gkeys_s": r["serial"]["throughput_gkeys_s"],
            "throughput_ratio": r["throughput_ratio"],
            "served_p50_ms": r["served"]["p50_ms"], "served_p99_ms": r["served"]["p99_ms"],
            "serial_p50_ms": r["serial"]["p50_ms"], "serial_p99_ms": r["serial"]["p99_ms"],
        }
    return out


def batched_summary(res: dict) -> dict:
    """The batched leg's figures for the benchmark line."""
    return {"workload": res["config"]["workload"], "gkeys_s": res["value"],
            "per_filter_gkeys_s": res["plain_per_filter_gkeys_s"],
            "speedup_vs_per_filter": res["speedup_vs_per_filter"],
            "add_speedup": res["add_speedup"], "contains_speedup": res["contains_speedup"],
            "ms": res["ms"], "results_equal": res["results_equal_batched_vs_per_filter"]}


if __name__ == "__main__":
    sys.exit(main())
