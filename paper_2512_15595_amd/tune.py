"""Autotuner: measures every execution mapping of add and contains and picks
the fastest per (op, word width, words per block, size class).

The paper's point is that no fixed mapping is best across operations, block
sizes, memory regimes and GPUs (Sec. IV-A, V-B, V-C, V-D): lookup favours
vertical layouts and construction horizontal ones on B200, and the optimum
moves between architectures.  This module measures the same space on the
local GPU -- lanes per key THETA, words per lane PHI, keys per lane KT, the
atomic width of add and the grid cap -- and writes a table that the library
compiles in as its defaults (``csrc/bf_tuned_defaults.inc``).

Size classes follow the MI355X memory hierarchy: a filter that fits one
XCD's 4 MiB L2, one that fits the 256 MiB Infinity Cache, and one that only
fits HBM.

Usage:
  python -m paper_2512_15595_amd.tune --filter-log2-bytes 30 25 21 --out tuning.json
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


def size_class(nbytes: int) -> str:
    for name, bound in SIZE_CLASSES:
        if nbytes <= bound:
            return name
    return SIZE_CLASSES[-1][0]


def mappings(s: int, word_bits: int, op: str, grid_caps=(0,)):
    out = []
    theta = 1
    while theta <= min(s, 16):
        phi = 1
        while theta * phi <= s:
            for kt in (1, 2, 4):
                for cap in grid_caps:
                    if op == "add":
                        out.append((theta, phi, kt, 32, cap))
                        if word_bits == 32 and phi >= 2:
                            out.append((theta, phi, kt, 64, cap))
                    else:
                        out.append((theta, phi, kt, 0, cap))
            phi *= 2
        theta *= 2
    return out


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def sweep_layout(torch, s: int, word_bits: int, k: int, filter_bytes: int, n_keys: int,
                 reps: int, ops=("add", "contains"), grid_caps=(0,), d_keys=None, d_q=None):
    from . import workloads
    from .bf import BF_OP_ADD, BF_OP_CONTAINS, BF_STRATEGY_DIRECT, BloomFilter

    block_bytes = s * word_bits // 8
    num_blocks = filter_bytes // block_bytes
    if d_keys is None:
        import numpy as np

        adds = workloads.uniform_keys(n_keys, 1)
        misses = workloads.uniform_keys(n_keys, 2)
        q = workloads.mix(adds, misses, 0.5, 4)
        d_keys = torch.from_numpy(adds.view(np.int64)).to("cuda")
        d_q = torch.from_numpy(q.view(np.int64)).to("cuda")
    d_out = torch.empty(n_keys, dtype=torch.uint8, device="cuda")
    f = BloomFilter(num_blocks, s, word_bits, k, 0)
    f.add(d_keys)  # a filled filter: lookups then see the working load
    records = []
    try:
        for op in ops:
            opcode = BF_OP_ADD if op == "add" else BF_OP_CONTAINS
            for m in mappings(s, word_bits, op, grid_caps):
                # the table holds the direct path's mappings (a dense add would
                # otherwise take the partitioned strategy, where they do not apply)
                f.set_mapping(opcode, *m, strategy=BF_STRATEGY_DIRECT if op == "add" else 0)
                best = None
                for _ in range(reps + 1):  # first run is a warm-up
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    if op == "add":
                        f.add(d_keys)
                    else:
                        f.contains(d_q, out=d_out)
                    b.record()
                    torch.cuda.synchronize()
                    ms = a.elapsed_time(b)
                    best = ms if best is None or ms < best else best
                rate = n_keys / (best * 1e-3) / 1e9
                records.append({"op": op, "word_bits": word_bits, "words_per_block": s, "k": k,
                                "filter_bytes": filter_bytes, "size_class": size_class(filter_bytes),
                                "n_keys": n_keys, "lanes_per_key": m[0], "words_per_lane": m[1],
                                "keys_per_lane": m[2], "atomic_bits": m[3], "max_workgroups": m[4],
                                "ms": round(best, 4), "gkeys_s": round(rate, 3)})
            f.set_mapping(opcode)  # back to the default
    finally:
        f.close()
    return records


def _simplicity(r):
    # fewer cooperating lanes, wider per-lane chunks, two keys per lane first
    return (r["lanes_per_key"], -r["words_per_lane"], abs(r["keys_per_lane"] - 2),
            -r["atomic_bits"], r["max_workgroups"])


def best_per_class(records, tolerance: float = 0.01):
    """Fastest mapping per (op, word bits, words per block, size class);
    mappings within `tolerance` of the fastest count as ties and the simplest
    of them is taken, so run-to-run noise does not pick exotic layouts."""
    groups = {}
    for r in records:
        key = (r["op"], r["word_bits"], r["words_per_block"], r["size_class"])
        groups.setdefault(key, []).append(r)
    best = {}
    for key, rs in groups.items():
        top = max(r["gkeys_s"] for r in rs)
        ties = [r for r in rs if r["gkeys_s"] >= (1.0 - tolerance) * top]
        best[key] = min(ties, key=_simplicity)
    return best


def emit_inc(records, path: str = INC_PATH) -> str:
    """Writes the compiled-in default table from measured records."""
    best = best_per_class(records)
    lines = [
        "// bf_tuned_defaults.inc -- generated by paper_2512_15595_amd/tune.py from",
        "// measured sweeps on gfx950; one row per (op, word bits, words per block,",
        "// size class): the fastest mapping found.  Do not edit by hand.",
        "// op, word_bits, words_per_block, size_class(0=L2,1=MALL,2=HBM),",
        "//   lanes_per_key, words_per_lane, keys_per_lane, atomic_bits, max_workgroups, Gkeys/s",
    ]
    cls = {name: i for i, (name, _) in enumerate(SIZE_CLASSES)}
    for key in sorted(best):
        r = best[key]
        lines.append(
            "BF_TUNED({op}, {wb}, {s}, {c}, {t}, {p}, {kt}, {ab}, {cap}) /* {g} */".format(
                op=0 if r["op"] == "add" else 1, wb=r["word_bits"], s=r["words_per_block"],
                c=cls[r["size_class"]], t=r["lanes_per_key"], p=r["words_per_lane"],
                kt=r["keys_per_lane"], ab=r["atomic_bits"], cap=r["max_workgroups"],
                g=r["gkeys_s"]))
    text = "\n".join(lines) + "\n"
    with open(path, "w") as fh:
        fh.write(text)
    return text


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--filter-log2-bytes", type=int, nargs="+", default=[30])
    ap.add_argument("--layouts", type=str, default="1x32,2x32,4x32,8x32,16x32,1x64,2x64,4x64,8x64,16x64")
    ap.add_argument("--k", type=int, default=8, help="pattern bits (raised to s where k < s)")
    ap.add_argument("--log2-keys", type=int, default=26)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--ops", type=str, default="add,contains")
    ap.add_argument("--grid-caps", type=str, default="0")
    ap.add_argument("--out", type=str, default=None)
    ap.add_argument("--emit-inc", type=str, default=None, help="write the .inc from a JSON file")
    args = ap.parse_args()

    if args.emit_inc:
        with open(args.emit_inc) as fh:
            records = json.load(fh)["records"]
        print(emit_inc(records))
        return 0

    import numpy as np
    import torch

    from . import workloads

    n = 1 << args.log2_keys
    adds = workloads.uniform_keys(n, 1)
    q = workloads.mix(adds, workloads.uniform_keys(n, 2), 0.5, 4)
    d_keys = torch.from_numpy(adds.view(np.int64)).to("cuda")
    d_q = torch.from_numpy(q.view(np.int64)).to("cuda")
    caps = tuple(int(x) for x in args.grid_caps.split(","))
    records = []
    t0 = time.time()
    for lb in args.filter_log2_bytes:
        for lay in args.layouts.split(","):
            s, wb = (int(x) for x in lay.split("x"))
            k = max(args.k, s)
            recs = sweep_layout(torch, s, wb, k, 1 << lb, n, args.reps,
                                tuple(args.ops.split(",")), caps, d_keys, d_q)
            records.extend(recs)
            for key, r in sorted(best_per_class(recs).items()):
                log(f"[tune] {lb=} {lay} k={k} {key[0]:8s} best {r['gkeys_s']:8.2f} Gkeys/s "
                    f"theta={r['lanes_per_key']} phi={r['words_per_lane']} kt={r['keys_per_lane']} "
                    f"atom={r['atomic_bits']} ({time.time() - t0:.0f}s)")
    out = {"arch": torch.cuda.get_device_properties(0).gcnArchName, "n_keys": n, "records": records}
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh)
    else:
        print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
