"""Autotuner: measures the execution mappings of add and contains and the
crossover between the two constructions of add, and writes the table the
library compiles in as its defaults (``csrc/bf_tuned_defaults.inc``).

The paper's point is that no fixed mapping is best across operations, block
sizes, memory regimes and GPUs (Sec. IV-A, V-B, V-C, V-D): lookup favours
vertical layouts and construction horizontal ones on B200, and the optimum
moves between architectures.  This module measures the same space on the
local GPU, keyed by
  (op, word bits S, words per block s, filter size class, k, batch class),
over lanes per key THETA, words per lane PHI, keys per lane KT, the atomic
width of add and the workgroup size (64 / 128 / 256 threads).  Size classes
follow the MI355X memory hierarchy: a filter that fits one XCD's 4 MiB L2,
one that fits the 256 MiB Infinity Cache, and one that only fits HBM.  Batch
classes: at most 2^16 keys (latency bound) or more.

It also measures, per layout (sectorized (s, S), cache-sectorized (s, S, z),
classic at k), the cost of a direct add (one atomic group per key) and of a
partitioned one (keys grouped by 64 KiB chunk) over filter sizes and key
counts, and fits
  partitioned ~ a + b * MiB + c * n,   direct ~ e + d[size class] * n
(relative least squares); the library partitions when n * (d - c) > a - e +
b * MiB.

Usage (on the GPU):
  python -m paper_2512_15595_amd.tune --out tuning.json
  python -m paper_2512_15595_amd.tune --emit-inc tuning.json   # writes the .inc
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
INC_PATH = os.path.join(HERE, "csrc", "bf_tuned_defaults.inc")

SIZE_CLASSES = [  # (name, upper bound in bytes, inclusive)
    ("l2", 4 << 20),
    ("mall", 256 << 20),
    ("hbm", 1 << 62),
]
SMALL_BATCH_KEYS = 1 << 16
TUNED_KS = (4, 8, 16)
WG_SIZES = (64, 128, 256)
SBF_LAYOUTS = [(s, wb) for wb in (32, 64) for s in (1, 2, 4, 8, 16)]
CSBF_LAYOUTS = [(8, 32, 2), (8, 32, 4), (16, 32, 4), (16, 64, 2), (16, 64, 4), (16, 64, 8),
                (4, 64, 2), (8, 64, 4)]
CLASSIC_KS = (8, 16)


def size_class(nbytes: int) -> int:
    for i, (_, bound) in enumerate(SIZE_CLASSES):
        if nbytes <= bound:
            return i
    return len(SIZE_CLASSES) - 1


def n_class(n: int) -> int:
    return 0 if n <= SMALL_BATCH_KEYS else 1


def mappings(s: int, word_bits: int, op: str):
    """(theta, phi, kt, atomic_bits) of every compiled mapping."""
    out = []
    theta = 1
    while theta <= min(s, 16):
        phi = 1
        while theta * phi <= s:
            for kt in (1, 2, 4):
                if op == "add":
                    out.append((theta, phi, kt, 32))
                    if word_bits == 32 and phi >= 2:
                        out.append((theta, phi, kt, 64))
                else:
                    out.append((theta, phi, kt, 0))
            phi *= 2
        theta *= 2
    return out


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def time_launches(torch, fn, launches: int, reps: int) -> float:
    """Best over reps of the mean time (ms) of `launches` back-to-back calls."""
    fn()
    torch.cuda.synchronize()
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(launches):
            fn()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / launches
        best = ms if best is None or ms < best else best
    return best


def sweep_mappings(torch, d_keys, d_q, d_out, sizes, ks, ns, reps, layouts=SBF_LAYOUTS,
                   wg_top: int = 3):
    """Stage 1: every mapping at 256-thread workgroups; stage 2: the best
    `wg_top` of them at 64 and 128 threads.  One record per measurement."""
    from .bf import BF_OP_ADD, BF_OP_CONTAINS, BF_STRATEGY_DIRECT, BloomFilter

    records = []
    t0 = time.time()
    for (s, wb) in layouts:
        block = s * wb // 8
        for nbytes in sizes:
            for k in ks:
                if k < s:
                    continue
                f = BloomFilter(nbytes // block, s, wb, k, 0)
                f.add(d_keys)               # a filled filter: lookups see the working load
                torch.cuda.synchronize()
                try:
                    for n in ns:
                        # small batches: 16 launches back to back between two
                        # events, the way a stream of small requests runs
                        # (device bound: ~7 us per launch against ~4 us of
                        # host enqueue)
                        launches = max(1, (1 << 19) // n)
                        nreps = reps if n > SMALL_BATCH_KEYS else 2 * reps + 1
                        for op in ("add", "contains"):
                            code = BF_OP_ADD if op == "add" else BF_OP_CONTAINS
                            strat = BF_STRATEGY_DIRECT if op == "add" else 0
                            keys = d_keys[:n] if op == "add" else d_q[:n]

                            def run(m, wg, keys=keys, op=op):
                                f.set_mapping(code, *m, 0, strat, wg)
                                fn = (lambda: f.add(keys)) if op == "add" else \
                                    (lambda: f.contains(keys, out=d_out))
                                ms = time_launches(torch, fn, launches, nreps)
                                rec = {"op": op, "word_bits": wb, "words_per_block": s, "k": k,
                                       "filter_bytes": nbytes, "size_class": size_class(nbytes),
                                       "n_keys": n, "n_class": n_class(n), "lanes_per_key": m[0],
                                       "words_per_lane": m[1], "keys_per_lane": m[2],
                                       "atomic_bits": m[3], "max_workgroups": 0,
                                       "workgroup_threads": wg, "ms": round(ms, 5),
                                       "gkeys_s": round(n / (ms * 1e-3) / 1e9, 3)}
                                records.append(rec)
                                return rec

                            stage1 = [run(m, 256) for m in mappings(s, wb, op)]
                            stage1.sort(key=lambda r: -r["gkeys_s"])
                            for r in stage1[:wg_top]:
                                m = (r["lanes_per_key"], r["words_per_lane"], r["keys_per_lane"],
                                     r["atomic_bits"])
                                for wg in WG_SIZES:
                                    if wg != 256:
                                        run(m, wg)
                            f.set_mapping(code)
                finally:
                    f.close()
                best = best_per_key([r for r in records if r["words_per_block"] == s and
                                     r["word_bits"] == wb and r["filter_bytes"] == nbytes and
                                     r["k"] == k])
                for key, r in sorted(best.items()):
                    log(f"[tune] {s}x{wb} {nbytes >> 20} MiB k={k} {key[0]:8s} n={r['n_keys']:>9} "
                        f"best {r['gkeys_s']:8.2f} Gkeys/s theta={r['lanes_per_key']} "
                        f"phi={r['words_per_lane']} kt={r['keys_per_lane']} atom={r['atomic_bits']} "
                        f"wg={r['workgroup_threads']} ({time.time() - t0:.0f}s)")
    return records


def _simplicity(r):
    # fewer cooperating lanes, wider per-lane chunks, two keys per lane, full
    # 256-thread workgroups first
    return (r["lanes_per_key"], -r["words_per_lane"], abs(r["keys_per_lane"] - 2),
            -r["atomic_bits"], -r["workgroup_threads"], r["max_workgroups"])


def _mapping_of(r):
    return (r["lanes_per_key"], r["words_per_lane"], r["keys_per_lane"], r["atomic_bits"],
            r.get("workgroup_threads", 256), r["max_workgroups"])


def _class_scores(rs):
    """Per mapping measured at every filter size of the group: the mean over
    those sizes of its rate relative to the best rate at that size (a size
    class spans sizes whose best mappings can differ)."""
    by_size = {}
    for r in rs:
        by_size.setdefault(r.get("filter_bytes", 0), {})[_mapping_of(r)] = r
    common = set.intersection(*(set(v) for v in by_size.values()))
    tops = {sz: max(r["gkeys_s"] for r in v.values()) for sz, v in by_size.items()}
    rep = max(by_size, key=lambda sz: len(by_size[sz]))  # a record to report, per mapping
    out = []
    for m in common:
        score = sum(by_size[sz][m]["gkeys_s"] / tops[sz] for sz in by_size) / len(by_size)
        out.append((score, by_size[rep][m]))
    return out


def best_per_key(records, tolerance: float = 0.01, small_tolerance: float = 0.10):
    """Best mapping per (op, word bits, words per block, size class, k, batch
    class): the highest mean relative rate over the filter sizes measured in
    the class; mappings within `tolerance` of the best count as ties and the
    simplest of them is taken, so run-to-run noise does not pick exotic
    layouts.  Small batches are launch-latency bound and their rates noisier
    (a launch of 2^15 keys takes ~7 us of device time, most of it
    dispatch): their band is `small_tolerance`, and the large-batch mapping
    is kept when it is inside it."""
    groups = {}
    for r in records:
        key = (r["op"], r["word_bits"], r["words_per_block"], r["size_class"], r["k"],
               r.get("n_class", 1))
        groups.setdefault(key, []).append(r)
    best = {}
    for key, rs in groups.items():
        if key[5] == 0:
            continue
        scored = _class_scores(rs)
        top = max(sc for sc, _ in scored)
        ties = [r for sc, r in scored if sc >= (1.0 - tolerance) * top]
        best[key] = min(ties, key=_simplicity)
    # a small batch keeps the large-batch mapping unless another one is
    # clearly faster at its size
    for key, rs in groups.items():
        if key[5] != 0:
            continue
        scored = _class_scores(rs)
        top = max(sc for sc, _ in scored)
        ties = [r for sc, r in scored if sc >= (1.0 - small_tolerance) * top]
        large = best.get(key[:5] + (1,))
        same = [r for r in ties if large is not None and _mapping_of(r) == _mapping_of(large)]
        best[key] = same[0] if same else min(ties, key=_simplicity)
    return best


# --------------------------------------------------------------------------
# construction crossover
# --------------------------------------------------------------------------

def make_layout(bfmod, kind: str, spec, nbytes: int):
    if kind == "sbf":
        s, wb = spec
        k = max(8, s)
        return bfmod.BloomFilter(nbytes // (s * wb // 8), s, wb, k, 0)
    if kind == "csbf":
        s, wb, z = spec
        k = max(8, z)
        return bfmod.CacheSectorizedFilter(nbytes // (s * wb // 8), s, wb, z, k, 0)
    return bfmod.ClassicFilter(nbytes * 8, spec, 0)


def sweep_crossover(torch, d_keys, sizes, ns, reps):
    """Direct and partitioned add times per layout, filter size and key count."""
    from . import bf as bfmod

    jobs = [("sbf", x) for x in SBF_LAYOUTS] + [("csbf", x) for x in CSBF_LAYOUTS] + \
           [("classic", k) for k in CLASSIC_KS]
    records = []
    t0 = time.time()
    for kind, spec in jobs:
        for nbytes in sizes:
            f = make_layout(bfmod, kind, spec, nbytes)
            try:
                for n in ns:
                    keys = d_keys[:n]
                    row = {"kind": kind, "spec": list(spec) if isinstance(spec, tuple) else [spec],
                           "filter_bytes": nbytes, "size_class": size_class(nbytes), "n_keys": n}
                    for strat, name in ((bfmod.BF_STRATEGY_DIRECT, "direct_ms"),
                                        (bfmod.BF_STRATEGY_PARTITIONED, "partitioned_ms")):
                        f.set_mapping(bfmod.BF_OP_ADD, strategy=strat)
                        row[name] = round(time_launches(torch, lambda: f.add(keys), 1, reps), 5)
                    records.append(row)
            finally:
                f.close()
        log(f"[tune] crossover {kind} {spec}: {len([r for r in records if r['kind'] == kind])} "
            f"points ({time.time() - t0:.0f}s)")
    return records


def _wls(rows, cols, target):
    """Least squares of target ~ rows @ coef with relative weights (1/t)."""
    import numpy as np

    A = np.array([[r[c] for c in cols] for r in rows], dtype=np.float64)
    y = np.array([r[target] for r in rows], dtype=np.float64)
    w = 1.0 / np.maximum(y, 1e-6)
    coef, *_ = np.linalg.lstsq(A * w[:, None], y * w, rcond=None)
    return coef


def fit_crossover(records):
    """Per layout: (a_us, b_us_per_mib, c_ps, d_ps[3]) with the direct
    intercept folded into a."""
    fits = {}
    groups = {}
    for r in records:
        groups.setdefault((r["kind"], tuple(r["spec"])), []).append(r)
    for key, rs in groups.items():
        pts = [{"one": 1.0, "mib": r["filter_bytes"] / 2**20, "n": float(r["n_keys"]),
                "t": r["partitioned_ms"] * 1e3} for r in rs]
        a, b, c = _wls(pts, ("one", "mib", "n"), "t")          # us, us/MiB, us/key
        d = []
        e_all = []
        for cls in range(3):
            cr = [r for r in rs if r["size_class"] == cls]
            if not cr:
                d.append(None)
                continue
            dp = [{"one": 1.0, "n": float(r["n_keys"]), "t": r["direct_ms"] * 1e3} for r in cr]
            e, dd = _wls(dp, ("one", "n"), "t")
            d.append(dd)
            e_all.append(e)
        known = [x for x in d if x is not None]
        d = [x if x is not None else known[-1] for x in d]
        e = min(e_all) if e_all else 0.0
        fits[key] = {"a_us": max(a - e, 0.0), "b_us_per_mib": max(b, 0.0), "c_ps": max(c, 0.0) * 1e6,
                     "d_ps": [max(x, 0.0) * 1e6 for x in d]}
    return fits


def emit_inc(records, xover_records=None, path: str = INC_PATH) -> str:
    """Writes the compiled-in table from measured records."""
    best = best_per_key(records)
    lines = [
        "// bf_tuned_defaults.inc -- generated by paper_2512_15595_amd/tune.py from",
        "// measured sweeps on gfx950.  Do not edit by hand.",
        "// BF_TUNED(op, word_bits, words_per_block, size_class (0 L2, 1 MALL, 2 HBM), k,",
        "//          batch class (0: <= 2^16 keys, 1: more), lanes_per_key, words_per_lane,",
        "//          keys_per_lane, atomic_bits, max_workgroups, workgroup_threads)  /* Gkeys/s */",
        "// BF_CROSSOVER(kind (0 sectorized, 1 classic, 2 cache-sectorized), word_bits,",
        "//          words_per_block, groups, k, a_us, b_us_per_MiB, c_ps_per_key,",
        "//          d_ps_per_key for size classes 0, 1, 2)",
    ]
    for key in sorted(best):
        r = best[key]
        lines.append(
            "BF_TUNED({op}, {wb}, {s}, {c}, {k}, {nc}, {t}, {p}, {kt}, {ab}, {cap}, {wg}) /* {g} */".format(
                op=0 if r["op"] == "add" else 1, wb=r["word_bits"], s=r["words_per_block"],
                c=r["size_class"], k=r["k"], nc=r.get("n_class", 1), t=r["lanes_per_key"],
                p=r["words_per_lane"], kt=r["keys_per_lane"], ab=r["atomic_bits"],
                cap=r["max_workgroups"], wg=r.get("workgroup_threads", 256), g=r["gkeys_s"]))
    if xover_records:
        for (kind, spec), v in sorted(fit_crossover(xover_records).items()):
            if kind == "sbf":
                s, wb = spec
                head = f"0, {wb}, {s}, 0, 0"
            elif kind == "csbf":
                s, wb, z = spec
                head = f"2, {wb}, {s}, {z}, 0"
            else:
                head = f"1, 32, 1, 0, {spec[0]}"
            d0, d1, d2 = v["d_ps"]
            lines.append(f"BF_CROSSOVER({head}, {v['a_us']:.3f}, {v['b_us_per_mib']:.4f}, "
                         f"{v['c_ps']:.3f}, {d0:.3f}, {d1:.3f}, {d2:.3f})")
    text = "\n".join(lines) + "\n"
    with open(path, "w") as fh:
        fh.write(text)
    return text


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes-log2", type=int, nargs="+", default=[21, 24, 26, 30],
                    help="filter sizes for the mapping sweep (a class may hold several)")
    ap.add_argument("--ks", type=int, nargs="+", default=list(TUNED_KS))
    ap.add_argument("--ns-log2", type=int, nargs="+", default=[15, 26],
                    help="batch sizes (one per batch class) for the mapping sweep")
    ap.add_argument("--layouts", type=str, default=",".join(f"{s}x{wb}" for s, wb in SBF_LAYOUTS))
    ap.add_argument("--xover-sizes-log2", type=int, nargs="+", default=[22, 26, 30])
    ap.add_argument("--xover-ns-log2", type=int, nargs="+", default=[18, 20, 22, 24, 26])
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--no-mappings", action="store_true")
    ap.add_argument("--no-crossover", action="store_true")
    ap.add_argument("--out", type=str, default=None)
    ap.add_argument("--emit-inc", type=str, default=None, help="write the .inc from a JSON file")
    args = ap.parse_args()

    if args.emit_inc:
        with open(args.emit_inc) as fh:
            data = json.load(fh)
        print(emit_inc(data["records"], data.get("crossover")))
        return 0

    import numpy as np
    import torch

    from . import workloads

    n = 1 << max(max(args.ns_log2), max(args.xover_ns_log2))
    adds = workloads.uniform_keys(n, 1)
    q = workloads.mix(adds, workloads.uniform_keys(n, 2), 0.5, 4)
    d_keys = torch.from_numpy(adds.view(np.int64)).to("cuda")
    d_q = torch.from_numpy(q.view(np.int64)).to("cuda")
    d_out = torch.empty(n, dtype=torch.uint8, device="cuda")
    layouts = [tuple(int(x) for x in lay.split("x")) for lay in args.layouts.split(",")]
    out = {"arch": torch.cuda.get_device_properties(0).gcnArchName, "records": [],
           "crossover": []}
    if not args.no_mappings:
        out["records"] = sweep_mappings(torch, d_keys, d_q, d_out,
                                        [1 << x for x in args.sizes_log2], args.ks,
                                        [1 << x for x in args.ns_log2], args.reps, layouts)
    if not args.no_crossover:
        out["crossover"] = sweep_crossover(torch, d_keys, [1 << x for x in args.xover_sizes_log2],
                                           [1 << x for x in args.xover_ns_log2], args.reps)
        for key, v in sorted(fit_crossover(out["crossover"]).items()):
            log(f"[tune] crossover fit {key}: {v}")
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh)
    else:
        print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
