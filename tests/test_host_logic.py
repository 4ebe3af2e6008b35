"""Host-side logic without a GPU: the seeded workload generators, the
autotuner's selection and table output, and the benchmark's helpers."""
from __future__ import annotations

import math
from types import SimpleNamespace

import numpy as np
import pytest

import bench
from paper_2512_15595_amd import tune, workloads


# --------------------------------------------------------------------------
# Workload generators
# --------------------------------------------------------------------------

def test_splitmix64_published_sequence():
    """SplitMix64 from state 0 (Steele, Lea, Flood 2014; Vigna's reference
    implementation) begins e220a8397b1dcdaf, 6e789e6aa1b965f4,
    06c45d188009454f, f88bb8a8724c81ec."""
    got = [int(v) for v in workloads.splitmix64(0, 0, 4)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    # element i of stream s is independent of where the range starts
    assert np.array_equal(workloads.splitmix64(7, 5, 10), workloads.splitmix64(7, 0, 15)[5:])


@pytest.mark.parametrize("n", [0, 1, 2, 7, 1000, 65536, 99991])
def test_affine_permutation_is_a_bijection(n):
    p = workloads.affine_permutation(n, 3)
    assert p.size == n
    assert np.array_equal(np.sort(p), np.arange(n))


def test_mix_takes_the_requested_share():
    hits = np.arange(1, 200_001, dtype=np.uint64)
    misses = np.zeros(200_000, dtype=np.uint64)
    for frac in (0.0, 0.25, 0.5, 1.0):
        m = workloads.mix(hits, misses, frac, 9)
        share = float(np.mean(m != 0))
        assert abs(share - frac) < 0.01
        assert np.all((m == 0) | (m == hits))


def test_correctness_workload_shape():
    params, adds, queries = workloads.correctness_workload()
    assert params == dict(num_blocks=4096, words_per_block=8, word_bits=32, k=8, seed=0)
    assert adds.size == 20_000 and queries.size == 1_000_000
    present = np.isin(queries, adds)
    assert abs(present.mean() - 0.5) < 0.001


def test_kmer_keys_are_packed_rolling_31mers():
    keys = workloads.kmer_keys(5000, 5)
    assert keys.size == 5000 - 31 + 1
    assert np.all(keys >> np.uint64(62) == 0)                       # 62 bits used
    # consecutive k-mers overlap in 30 bases: drop the first base, shift, append
    low60 = np.uint64((1 << 60) - 1)
    assert np.array_equal(keys[1:] >> np.uint64(2), keys[:-1] & low60)
    # with every later segment copied, only the first segment's k-mers are new
    rep = workloads.kmer_keys(100 * 200, 6, segment=100, repeat_p=1.0)
    assert np.unique(rep).size < 100 * 2


def test_zipf_counts_sum_clip_and_shape():
    c = workloads.zipf_counts(4096, 2**28, 1.1, 100, 10_000_000, 4)
    assert int(c.sum()) == 2**28
    assert c.min() >= 100 and c.max() <= 10_000_000
    s = np.sort(c)[::-1].astype(np.float64)
    # in the unclipped middle, count ~ r^-1.1
    r1, r2 = 100, 1000
    assert abs(math.log(s[r1 - 1] / s[r2 - 1]) / math.log(r2 / r1) - 1.1) < 0.02


def test_log_uniform_sizes_range_and_alignment():
    s = workloads.log_uniform_sizes(10_000, 4 << 10, 16 << 20, 32, 4)
    assert np.all(s % 32 == 0)
    assert s.min() >= 4 << 10 and s.max() <= 16 << 20
    # log-uniform: about half below the geometric mean
    gm = math.sqrt((4 << 10) * (16 << 20))
    assert abs(np.mean(s < gm) - 0.5) < 0.02


def test_mixed_queries_host_twin():
    src = workloads.splitmix64(11, 100, 5000)
    q = workloads.mixed_queries(50_000, 11, 100, 5000, 12, 0, 0.5, 13)
    hit = np.isin(q, src)
    assert abs(hit.mean() - 0.5) < 0.01
    fresh = workloads.splitmix64(12, 0, 50_000)
    assert np.all(hit | (q == fresh))


# --------------------------------------------------------------------------
# Autotuner
# --------------------------------------------------------------------------

def _rec(theta, phi, kt, rate, op="contains", cls=2, atomic=0, k=8, ncls=1, wg=256):
    return {"op": op, "word_bits": 32, "words_per_block": 8, "size_class": cls, "k": k,
            "n_class": ncls, "lanes_per_key": theta, "words_per_lane": phi, "keys_per_lane": kt,
            "atomic_bits": atomic, "max_workgroups": 0, "workgroup_threads": wg, "gkeys_s": rate}


def test_tuner_prefers_simple_mappings_within_the_tie_band():
    recs = [_rec(4, 2, 1, 50.0), _rec(1, 8, 2, 49.8), _rec(2, 4, 4, 45.0), _rec(1, 8, 2, 49.9, wg=64)]
    best = tune.best_per_key(recs)[("contains", 32, 8, 2, 8, 1)]
    assert (best["lanes_per_key"], best["words_per_lane"], best["keys_per_lane"]) == (1, 8, 2)
    assert best["workgroup_threads"] == 256                      # full workgroups on ties
    recs = [_rec(4, 2, 1, 50.0), _rec(1, 8, 2, 48.0)]           # outside the 1 % band
    best = tune.best_per_key(recs)[("contains", 32, 8, 2, 8, 1)]
    assert best["lanes_per_key"] == 4


def test_tuner_emits_one_row_per_key(tmp_path):
    recs = [_rec(1, 8, 2, 50.0, cls=c) for c in (0, 1, 2)]
    recs += [_rec(4, 2, 2, 20.0, op="add", cls=c, atomic=64) for c in (0, 1, 2)]
    recs += [_rec(1, 8, 1, 9.0, k=16, ncls=0, wg=128)]
    xover = [{"kind": "sbf", "spec": [8, 32], "filter_bytes": b, "size_class": tune.size_class(b),
              "n_keys": n, "partitioned_ms": (30 + 0.5 * b / 2**20 + 1e-5 * n) / 1e3,
              "direct_ms": (5 + 4e-5 * n) / 1e3}
             for b in (4 << 20, 64 << 20, 1 << 30) for n in (1 << 18, 1 << 20, 1 << 22, 1 << 24)]
    text = tune.emit_inc(recs, xover, str(tmp_path / "t.inc"))
    rows = [line for line in text.splitlines() if line.startswith("BF_TUNED(")]
    assert len(rows) == 7
    assert "BF_TUNED(1, 32, 8, 2, 8, 1, 1, 8, 2, 0, 0, 256)" in text   # contains, HBM class
    assert "BF_TUNED(0, 32, 8, 0, 8, 1, 4, 2, 2, 64, 0, 256)" in text  # add, L2 class
    assert "BF_TUNED(1, 32, 8, 2, 16, 0, 1, 8, 1, 0, 0, 128)" in text  # small batch, k = 16
    cross = [line for line in text.splitlines() if line.startswith("BF_CROSSOVER(")]
    assert len(cross) == 1
    vals = [float(x) for x in cross[0][len("BF_CROSSOVER("):-1].split(",")]
    a, b, c, d0 = vals[5:9]
    # the fit recovers the generating model (direct intercept folded into a)
    assert abs(a - 25) < 0.5 and abs(b - 0.5) < 0.01 and abs(c - 10) < 0.2 and abs(d0 - 40) < 0.5


def test_tuner_mapping_space_is_valid():
    for s in (1, 2, 4, 8, 16):
        for wb in (32, 64):
            for op in ("add", "contains"):
                for theta, phi, kt, atomic in tune.mappings(s, wb, op):
                    assert theta * phi <= s and theta <= 16 and kt in (1, 2, 4)
                    assert atomic in ((32, 64) if op == "add" else (0,))
                    if atomic == 64:
                        assert wb == 32 and phi >= 2


def _table():
    """The compiled-in rows, parsed from the generated .inc."""
    tuned, cross = [], []
    for line in open(tune.INC_PATH):
        if line.startswith("BF_TUNED("):
            tuned.append([int(x) for x in line[len("BF_TUNED("):line.index(")")].split(",")])
        elif line.startswith("BF_CROSSOVER("):
            vals = line[len("BF_CROSSOVER("):line.index(")")].split(",")
            cross.append([int(x) for x in vals[:5]] + [float(x) for x in vals[5:]])
    return tuned, cross


def _expected_row(tuned, op, wb, s, cls, k, ncls):
    rows = [r for r in tuned if r[:4] == [op, wb, s, cls]]
    if any(r[5] == ncls for r in rows):
        rows = [r for r in rows if r[5] == ncls]
    if not rows:
        return None
    ratio = lambda r: max(r[4], k) * 4096 // min(r[4], k)            # noqa: E731
    return min(rows, key=lambda r: (ratio(r), -r[4]))


def test_tuned_mapping_follows_the_compiled_table():
    from paper_2512_15595_amd import bf

    tuned, _ = _table()
    assert tuned, "the table has rows"
    g = workloads.rng(5)
    for _ in range(400):
        s = int(g.choice([1, 2, 4, 8, 16]))
        wb = int(g.choice([32, 64]))
        k = int(g.integers(s, 17))
        op = int(g.integers(0, 2))
        nbytes = int(2 ** g.uniform(12, 33)) // (s * wb // 8) * (s * wb // 8) or s * wb // 8
        n = int(2 ** g.uniform(4, 30))
        cls = 0 if nbytes <= 4 << 20 else 1 if nbytes <= 256 << 20 else 2
        ncls = 0 if n <= 1 << 16 else 1
        st, m = bf.bf_tuned_mapping(op, nbytes // (s * wb // 8), s, wb, k, n)
        assert st == 0
        row = _expected_row(tuned, op, wb, s, cls, k, ncls)
        if row is None:
            continue
        if k in (4, 6, 8, 12, 16):                      # compiled k: the row's mapping
            assert (m.lanes_per_key, m.words_per_lane, m.keys_per_lane) == tuple(row[6:9])
            assert m.workgroup_threads == row[11]
            if op == 0:
                assert m.atomic_bits == (row[9] or 32)
        else:                                            # runtime k: one lane, one key
            assert (m.lanes_per_key, m.words_per_lane, m.keys_per_lane) == (1, s, 1)


def test_tuned_strategy_follows_the_measured_crossover():
    from paper_2512_15595_amd import bf

    _, cross = _table()
    for r in cross:
        if r[0] != 0:
            continue
        wb, s = r[1], r[2]
        a, b, c, d = r[5], r[6], r[7], r[8:11]
        for nbytes in (1 << 20, 4 << 20, 64 << 20, 1 << 30, 4 << 30):
            cls = 0 if nbytes <= 4 << 20 else 1 if nbytes <= 256 << 20 else 2
            for n in (1 << 14, 1 << 18, 1 << 20, 3 << 20, 1 << 22, 1 << 24, 1 << 26):
                st, m = bf.bf_tuned_mapping(0, nbytes // (s * wb // 8), s, wb, max(8, s), n)
                assert st == 0
                want = (d[cls] - c) > 0 and n * (d[cls] - c) * 1e-6 > a + b * nbytes / 2**20
                assert m.strategy == (bf.BF_STRATEGY_PARTITIONED if want else bf.BF_STRATEGY_DIRECT), \
                    (s, wb, nbytes, n)


def test_tuned_mapping_rejects_bad_parameters():
    from paper_2512_15595_amd import bf

    for args in [(2, 1024, 8, 32, 8, 100), (0, 0, 8, 32, 8, 100), (0, 1024, 3, 32, 8, 100),
                 (0, 1024, 8, 16, 8, 100), (1, 1024, 8, 32, 7, 100), (1, 2**32 + 1, 8, 32, 8, 1)]:
        st, _ = bf.bf_tuned_mapping(*args)
        assert st == bf.BF_EINVAL


# --------------------------------------------------------------------------
# Benchmark helpers
# --------------------------------------------------------------------------

def test_water_fill_sizes_meet_the_total():
    sizes = bench.water_fill_sizes(64, 32 << 30, 64 << 20, 1 << 30, 32, 5)
    assert sizes.max() <= 1 << 30 and np.all(sizes % 32 == 0)
    assert abs(int(sizes.sum()) - (32 << 30)) <= 32 * 64


def test_latency_summary():
    res = [SimpleNamespace(arrival_ns=i * 1_000_000, complete_ns=i * 1_000_000 + (i + 1) * 100_000)
           for i in range(100)]
    out = bench.latency_summary(res, [10**6] * 100)
    lat = [(i + 1) * 0.1 for i in range(100)]
    assert out["p50_ms"] == round(float(np.percentile(lat, 50)), 3)
    assert out["p99_ms"] == round(float(np.percentile(lat, 99)), 3)
    span = (99 * 1_000_000 + 100 * 100_000) / 1e9
    assert math.isclose(out["throughput_gkeys_s"], round(1e8 / span / 1e9, 3))


def test_parse_mapping():
    assert bench.parse_mapping(None) is None
    assert bench.parse_mapping("4,2,2") == [4, 2, 2, 0, 0]
    assert bench.parse_mapping("1,8,2,0,512") == [1, 8, 2, 0, 512]


def test_bench_refuses_several_gpus(capsys, monkeypatch):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    assert bench.main() == 2
    assert "single MI355X" in capsys.readouterr().err
