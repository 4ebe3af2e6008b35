"""GPU parity of the Parquet split-block filter (include/bf_parquet.h), the
Arrow / Parquet-compatible configuration of the paper's Sec. I and Sec. VI:
bit-exact against the CPU oracle (whose bitset tests/test_parquet.py pins to
Apache Arrow's) for every execution mapping and both constructions, ragged
and misaligned value arrays, sizes from the format's smallest filter to its
largest (128 MiB, every byte and every lookup); and end to end against the
bloom filters pyarrow writes into Parquet files.
"""
from __future__ import annotations

import io
import time

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import log, to_device, valid_mappings
from oracle import parallel as oracle_par
from paper_2512_15595_amd import workloads

pytestmark = pytest.mark.gpu


def _bf():
    from paper_2512_15595_amd import bf

    return bf


def _values(n, seed):
    return workloads.rng(seed).integers(0, 2**64, size=n, dtype=np.uint64)


def _run(f, adds, queries, add_offset=0, query_offset=0):
    if adds.size:
        f.add(to_device(adds, add_offset))
    out = f.contains(to_device(queries, query_offset)).cpu().numpy() if queries.size else None
    words = f.words().cpu().numpy()
    torch.cuda.synchronize()
    return words, out


SIZES = [32, 96, 4096, 1 << 20, (1 << 20) + 32 * 77, 16 << 20]


@pytest.mark.parametrize("num_bytes", SIZES)
@pytest.mark.parametrize("strategy", ["direct", "partitioned"])
def test_parquet_matches_oracle(num_bytes, strategy):
    bf = _bf()
    n = max(num_bytes // 8, 1000) + 37                 # ~8 bits per value, ragged tail
    adds, queries = _values(n, 1), workloads.mix(_values(n, 1), _values(n, 2), 0.5, 3)
    f = bf.ParquetFilter(num_bytes)
    try:
        assert f.info().layout == bf.BF_LAYOUT_PARQUET
        f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_DIRECT if strategy == "direct"
                      else bf.BF_STRATEGY_PARTITIONED)
        log(f"parquet {num_bytes} B {strategy}: {n} adds, {queries.size} lookups")
        words, out = _run(f, adds, queries)
    finally:
        f.close()
    ref = oracle.ParquetOracle(num_bytes)
    ref.add(adds)
    assert np.array_equal(words, ref.bytes)
    assert np.array_equal(out, ref.contains(queries))


def test_parquet_every_mapping_bit_exact():
    bf = _bf()
    num_bytes = 1 << 18
    adds, queries = _values(40_000 + 13, 4), _values(30_000 + 5, 5)
    ref = oracle.ParquetOracle(num_bytes)
    ref.add(adds)
    want = ref.contains(np.concatenate([queries, adds[:5000]]))
    q_all = np.concatenate([queries, adds[:5000]])
    for theta, phi, kt, ab in valid_mappings(8, 32):
        f = bf.ParquetFilter(num_bytes)
        try:
            f.set_mapping(bf.BF_OP_ADD, theta, phi, kt, atomic_bits=ab, strategy=bf.BF_STRATEGY_DIRECT)
            if ab == 32:
                f.set_mapping(bf.BF_OP_CONTAINS, theta, phi, kt)
            words, out = _run(f, adds, q_all, add_offset=1, query_offset=3)
        finally:
            f.close()
        assert np.array_equal(words, ref.bytes), f"add mapping {(theta, phi, kt, ab)}"
        assert np.array_equal(out, want), f"contains mapping {(theta, phi, kt)}"


def test_parquet_noalloc_and_strategy_agree():
    bf = _bf()
    num_bytes = 8 << 20
    adds = _values(3_000_000, 6)
    a, b = bf.ParquetFilter(num_bytes), bf.ParquetFilter(num_bytes)
    try:
        assert a.add_strategy(adds.size) == bf.BF_STRATEGY_PARTITIONED
        d = to_device(adds)
        a.add(d)
        b.add_noalloc(d)
        wa, wb = a.words().cpu().numpy(), b.words().cpu().numpy()
        torch.cuda.synchronize()
    finally:
        a.close()
        b.close()
    ref = oracle.ParquetOracle(num_bytes)
    ref.add(adds)
    assert np.array_equal(wa, ref.bytes) and np.array_equal(wb, ref.bytes)


def _row_groups(nfilters, total, dense=(), seed=31):
    """Filters of a Parquet scan's row groups: power-of-two sizes 1 KiB ..
    1 MiB, Zipf-skewed value counts, plus `dense` (num_bytes, values) ones."""
    g = workloads.rng(seed)
    sizes = [1 << int(e) for e in g.integers(10, 21, size=nfilters)] + [nb for nb, _ in dense]
    counts = list(workloads.zipf_counts(nfilters, total, 1.1, 0, total // 4, seed + 1)) + [n for _, n in dense]
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    values = _values(int(offsets[-1]), seed + 2)
    queries = workloads.mix(values, _values(values.size, seed + 3), 0.5, seed + 4)
    return sizes, offsets, values, queries


@pytest.mark.parametrize("mode", ["launch", "launch_per_filter"])
def test_parquet_batched_plans_equal_oracle(mode):
    """A plan over row-group filters (and three dense ones, which take the
    multi-filter partitioned construction) with the format's salts."""
    bf = _bf()
    sizes, offsets, values, queries = _row_groups(200, 1 << 18, dense=[(16 << 20, 2_000_000)] * 3)
    filters = [bf.ParquetFilter(nb) for nb in sizes]
    d_v = to_device(values)
    d_q = to_device(queries)
    d_out = torch.full((queries.size,), 7, dtype=torch.uint8, device="cuda")
    add = bf.BatchPlan(bf.BF_OP_ADD, filters, d_v, offsets)
    con = bf.BatchPlan(bf.BF_OP_CONTAINS, filters, d_q, offsets, d_out)
    try:
        log(f"parquet plans ({mode}): {len(filters)} filters, {values.size} values")
        if mode == "launch":
            assert add.info().strategy == bf.BF_STRATEGY_PARTITIONED
        getattr(add, mode)()
        getattr(con, mode)()
        words = [f.words().cpu().numpy() for f in filters]
        out = d_out.cpu().numpy()
        torch.cuda.synchronize()
    finally:
        add.close()
        con.close()
        for f in filters:
            f.close()
    want_out = np.zeros(queries.size, dtype=np.uint8)
    for i, nb in enumerate(sizes):
        a, b = offsets[i], offsets[i + 1]
        ref = oracle.ParquetOracle(nb)
        ref.add(values[a:b])
        assert np.array_equal(words[i], ref.bytes), f"filter {i} ({nb} B)"
        want_out[a:b] = ref.contains(queries[a:b])
    assert np.array_equal(out, want_out)


def test_parquet_plans_and_servers_take_one_salt_table():
    bf = _bf()
    f = bf.ParquetFilter(4096)
    g = bf.BloomFilter(4096 // 32, 8, 32, 8, 0)
    keys = to_device(_values(100, 7))
    try:
        st, _ = bf.bf_batch_plan(bf.BF_OP_ADD, [f.handle, g.handle], keys.data_ptr(), [0, 50, 100])
        assert st == bf.BF_EINVAL
        with pytest.raises(bf.BfError) as e:
            bf.Server([f, g])
        assert e.value.status == bf.BF_EINVAL
    finally:
        f.close()
        g.close()


def test_parquet_served_requests_equal_sequential_oracle():
    """Interleaved adds and lookups on row-group filters through the
    server (coalesced small requests, and adds large enough for the
    partitioned construction), against the oracle replaying them in order."""
    bf = _bf()
    g = workloads.rng(41)
    sizes = [64 << 10, 256 << 10, 1 << 20, 2 << 20, 4 << 20]
    nreq = 200
    ops = np.where(g.random(nreq) < 0.15, 0, 1)
    filt = g.integers(0, len(sizes), size=nreq)
    ns = np.exp(np.log(50) + g.random(nreq) * (np.log(40_000) - np.log(50))).astype(np.int64)
    ns[:3] = 2_500_000                      # dense adds: partitioned
    ops[:3] = 0
    filt[:3] = [2, 3, 4]
    keys = _values(int(ns.sum()), 42)
    starts = np.concatenate([[0], np.cumsum(ns)])
    for i in range(nreq):                   # half of each lookup's values were added earlier
        if ops[i] == 1 and i > 0:
            prev = np.flatnonzero((ops[:i] == 0) & (filt[:i] == filt[i]))
            if prev.size:
                j = prev[-1]
                m = min(ns[i] // 2, ns[j])
                keys[starts[i]:starts[i] + m] = keys[starts[j]:starts[j] + m]
    arrivals = np.cumsum(g.exponential(20_000, size=nreq)).astype(np.int64)
    refs = [oracle.ParquetOracle(nb) for nb in sizes]
    want = np.zeros(keys.size, dtype=np.uint8)
    for i in range(nreq):
        a, b = starts[i], starts[i + 1]
        if ops[i] == 0:
            refs[filt[i]].add(keys[a:b])
        else:
            want[a:b] = refs[filt[i]].contains(keys[a:b])
    filters = [bf.ParquetFilter(nb) for nb in sizes]
    d_keys = to_device(keys)
    d_out = torch.full((keys.size,), 9, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    srv = bf.Server(filters)
    try:
        log(f"parquet server: {nreq} requests, {keys.size} values")
        kp = [d_keys.data_ptr() + 8 * int(starts[i]) for i in range(nreq)]
        op_ptr = [d_out.data_ptr() + int(starts[i]) if ops[i] == 1 else 0 for i in range(nreq)]
        res = srv.replay(srv.requests(ops, filt, kp, ns, op_ptr, arrivals))
        torch.cuda.synchronize()
        out = d_out.cpu().numpy()
        words = [f.words().cpu().numpy() for f in filters]
    finally:
        srv.close()
        for f in filters:
            f.close()
    assert all(r.status == 0 for r in res)
    mask = np.repeat(ops == 1, ns)
    assert np.array_equal(out[mask], want[mask])
    for i, r in enumerate(refs):
        assert np.array_equal(words[i], r.bytes), f"filter {i}"


# ---- the format's largest filter, every byte and every lookup ----------------

def test_parquet_128mib_full_size_equals_oracle():
    bf = _bf()
    num_bytes = 128 << 20                               # the format's maximum
    n = 1 << 27                                         # 8 bits per value: the partitioned add
    adds = workloads.uniform_keys(n, 71)
    queries = workloads.mix(adds[: 1 << 25], workloads.uniform_keys(1 << 25, 72), 0.5, 73)
    f = bf.ParquetFilter(num_bytes)
    g = bf.ParquetFilter(num_bytes)
    try:
        assert f.add_strategy(n) == bf.BF_STRATEGY_PARTITIONED
        d = to_device(adds)
        log("parquet 128 MiB: 2^27 adds partitioned and direct, 2^25 lookups")
        f.add(d)
        g.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_DIRECT)
        g.add(d)
        same = bool(torch.equal(f.words(), g.words()))
        out = f.contains(to_device(queries)).cpu().numpy()
        words = f.words().cpu().numpy()
        torch.cuda.synchronize()
    finally:
        f.close()
        g.close()
    assert same, "direct and partitioned construction differ"
    t0 = time.perf_counter()
    want_words = oracle_par.parquet_filter_words(num_bytes, adds)
    want = oracle_par.parquet_contains(want_words, num_bytes, queries)
    log(f"parquet 128 MiB: oracle in {time.perf_counter() - t0:.1f}s")
    if not np.array_equal(words, want_words):
        bad = np.flatnonzero((words != want_words).reshape(-1, 32).any(axis=1))
        pytest.fail(f"{bad.size} blocks differ from the oracle (first {bad[:8]})")
    assert np.array_equal(out, want)


# ---- end to end against the files Apache Arrow writes ------------------------

def _arrow_blob(column, ndv, fpp):
    pa = pytest.importorskip("pyarrow")
    pq = pytest.importorskip("pyarrow.parquet")
    buf = io.BytesIO()
    pq.write_table(pa.table({"x": column}), buf, row_group_size=len(column),  # one filter for all
                   bloom_filter_options={"x": {"ndv": ndv, "fpp": fpp}})
    data = buf.getvalue()
    c = pq.ParquetFile(io.BytesIO(data)).metadata.row_group(0).column(0)
    return data[c.bloom_filter_offset:c.bloom_filter_offset + c.bloom_filter_length]


@pytest.mark.parametrize("n,ndv,fpp", [(1000, 1000, 0.01), (400_000, 400_000, 0.01),
                                       (3_000_000, 1_000_000, 0.05)])
def test_gpu_built_blob_equals_arrow(n, ndv, fpp):
    pa = pytest.importorskip("pyarrow")
    bf = _bf()
    values = workloads.rng(n).integers(-(2**63), 2**63 - 1, size=n, dtype=np.int64)
    blob = _arrow_blob(pa.array(values), ndv, fpp)
    st, num_bytes, _ = bf.bf_parquet_parse_header(blob)
    assert st == bf.BF_OK
    f = bf.ParquetFilter(num_bytes)
    try:
        log(f"parquet vs arrow: {n} values into {num_bytes} B (strategy {f.add_strategy(n)})")
        f.add(to_device(values.view(np.uint64)))
        got = f.to_parquet_blob()
    finally:
        f.close()
    # compared as arrays: a failed `==` on megabyte bytes objects makes pytest
    # build a diff of them for minutes
    g, w = np.frombuffer(got, dtype=np.uint8), np.frombuffer(blob, dtype=np.uint8)
    assert g.size == w.size, (g.size, w.size)
    bad = np.flatnonzero(g != w)
    assert bad.size == 0, f"{bad.size} bytes differ from Arrow's (first at {bad[:4]})"


def test_gpu_lookups_in_an_arrow_filter():
    pa = pytest.importorskip("pyarrow")
    bf = _bf()
    rng = workloads.rng(11)
    values = rng.standard_normal(200_000)             # a DOUBLE column: keys are the bits
    blob = _arrow_blob(pa.array(values, type=pa.float64()), 200_000, 0.01)
    queries = np.concatenate([values[:50_000], rng.standard_normal(150_000)]).view(np.uint64)
    f = bf.ParquetFilter.from_parquet_blob(blob)
    try:
        out = f.contains(to_device(queries)).cpu().numpy()
        torch.cuda.synchronize()
    finally:
        f.close()
    st, num_bytes, header_len = bf.bf_parquet_parse_header(blob)
    ref = oracle.ParquetOracle(num_bytes)
    ref.bytes = np.frombuffer(blob[header_len:], dtype=np.uint8).copy()
    want = ref.contains(queries)
    assert np.array_equal(out, want)
    assert out[:50_000].all()
    # the same bitset adopted in place (bf_create_parquet_in)
    words = torch.from_numpy(ref.bytes.copy()).to("cuda")
    st, h = bf.bf_create_parquet_in(words.data_ptr(), num_bytes)
    assert st == bf.BF_OK
    try:
        d_q = to_device(queries)
        d_out = torch.empty(queries.size, dtype=torch.uint8, device="cuda")
        assert bf.bf_contains(h, d_q.data_ptr(), queries.size, d_out.data_ptr(),
                              torch.cuda.current_stream().cuda_stream) == bf.BF_OK
        assert np.array_equal(d_out.cpu().numpy(), want)
    finally:
        assert bf.bf_destroy(h) == bf.BF_OK
