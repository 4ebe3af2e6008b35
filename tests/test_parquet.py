"""The Parquet split-block Bloom filter (the Arrow / Parquet-compatible
configuration of the paper's Sec. I and Sec. VI) on the CPU: the oracle's
bitset is pinned to the bitsets Apache Arrow (pyarrow, an independent
implementation of the format) writes into Parquet files, and the library's
host-only header functions to the headers it writes.  No GPU needed.
"""
from __future__ import annotations

import io

import numpy as np
import pytest

import oracle
from oracle import parallel as oracle_par

pa = pytest.importorskip("pyarrow")
pq = pytest.importorskip("pyarrow.parquet")


def arrow_blobs(column, ndv: int, fpp: float, row_group_size: int | None = None):
    """The serialized bloom filters (header + bitset) pyarrow writes for one
    column, one per row group."""
    buf = io.BytesIO()
    pq.write_table(pa.table({"x": column}), buf, row_group_size=row_group_size,
                   bloom_filter_options={"x": {"ndv": ndv, "fpp": fpp}})
    data = buf.getvalue()
    md = pq.ParquetFile(io.BytesIO(data)).metadata
    out = []
    for g in range(md.num_row_groups):
        c = md.row_group(g).column(0)
        assert c.bloom_filter_offset is not None, "pyarrow wrote no bloom filter"
        out.append(data[c.bloom_filter_offset:c.bloom_filter_offset + c.bloom_filter_length])
    return out


def split(blob: bytes):
    """(num_bytes, bitset) of a serialized filter: the header's first field is
    numBytes (Thrift compact i32: field header 0x15, zigzag varint)."""
    assert blob[0] == 0x15
    i, shift, z = 1, 0, 0
    while True:
        b = blob[i]
        z |= (b & 0x7F) << shift
        i += 1
        shift += 7
        if not b & 0x80:
            break
    num_bytes = (z >> 1) ^ -(z & 1)
    return num_bytes, np.frombuffer(blob[len(blob) - num_bytes:], dtype=np.uint8)


CASES = [  # (values, ndv, fpp, seed)
    (1000, 1000, 0.01, 1),
    (300, 50, 0.2, 2),          # more values than ndv: a dense 32-byte-per-block filter
    (20_000, 100_000, 0.001, 3),
    (200_000, 200_000, 0.05, 4),
    (5, 1, 0.5, 5),             # the format's smallest filter (32 bytes)
]


@pytest.mark.parametrize("n,ndv,fpp,seed", CASES)
def test_oracle_bitset_equals_arrow(n, ndv, fpp, seed):
    rng = np.random.default_rng(seed)
    values = rng.integers(-(2**63), 2**63 - 1, size=n, dtype=np.int64)
    (blob,) = arrow_blobs(pa.array(values), ndv, fpp)
    num_bytes, bits = split(blob)
    ref = oracle.ParquetOracle(num_bytes)
    ref.add(values.view(np.uint64))
    assert np.array_equal(ref.bytes, bits)
    # every value is found in Arrow's bitset
    assert ref.contains(values.view(np.uint64)).all()
    view = oracle.ParquetOracle(num_bytes)
    view.bytes = bits.copy()
    assert view.contains(values.view(np.uint64)).all()


def test_oracle_equals_arrow_on_edge_values_and_duplicates():
    values = np.array([0, -1, 1, 2**63 - 1, -(2**63), 42, 42, 42, -42] * 3, dtype=np.int64)
    (blob,) = arrow_blobs(pa.array(values), 64, 0.01)
    num_bytes, bits = split(blob)
    ref = oracle.ParquetOracle(num_bytes)
    ref.add(values.view(np.uint64))
    assert np.array_equal(ref.bytes, bits)


def test_oracle_equals_arrow_for_double_columns():
    """DOUBLE values hash their IEEE-754 bits: the key is the value's bits."""
    rng = np.random.default_rng(7)
    values = np.concatenate([rng.standard_normal(3000), [0.0, 1.5, -2.25, 1e300]])
    (blob,) = arrow_blobs(pa.array(values, type=pa.float64()), 4000, 0.01)
    num_bytes, bits = split(blob)
    ref = oracle.ParquetOracle(num_bytes)
    ref.add(values.view(np.uint64))
    assert np.array_equal(ref.bytes, bits)


def test_oracle_equals_arrow_per_row_group():
    rng = np.random.default_rng(8)
    values = rng.integers(0, 10**12, size=9000, dtype=np.int64)
    blobs = arrow_blobs(pa.array(values), 3000, 0.01, row_group_size=3000)
    assert len(blobs) == 3
    for g, blob in enumerate(blobs):
        num_bytes, bits = split(blob)
        ref = oracle.ParquetOracle(num_bytes)
        ref.add(values[g * 3000:(g + 1) * 3000].view(np.uint64))
        assert np.array_equal(ref.bytes, bits), f"row group {g}"


def test_oracle_false_positive_rate_matches_the_block_model():
    """Lookups of absent values against Arrow's filter: the split-block FPR
    (each value's 8 bits in one 256-bit block: Poisson mixture over block
    loads) within a 5-sigma band."""
    from math import exp, factorial

    rng = np.random.default_rng(9)
    values = rng.integers(0, 2**62, size=50_000, dtype=np.int64)
    (blob,) = arrow_blobs(pa.array(values), 50_000, 0.01)
    num_bytes, bits = split(blob)
    view = oracle.ParquetOracle(num_bytes)
    view.bytes = bits.copy()
    queries = rng.integers(2**62, 2**63 - 1, size=400_000, dtype=np.int64)
    got = float(view.contains(queries.view(np.uint64)).mean())
    lam = values.size / (num_bytes // 32)
    want = sum(exp(-lam) * lam**i / factorial(i) * (1 - (1 - 1 / 32) ** i) ** 8 for i in range(80))
    sigma = (want * (1 - want) / queries.size) ** 0.5
    assert abs(got - want) < 5 * sigma + 1e-6, (got, want)


def test_parallel_oracle_equals_single_call():
    rng = np.random.default_rng(10)
    values = rng.integers(0, 2**64 - 1, size=40_000, dtype=np.uint64)
    num_bytes = 1 << 16
    ref = oracle.ParquetOracle(num_bytes)
    ref.add(values)
    words = oracle_par.parquet_filter_words(num_bytes, values, threads=4, parts=13)
    assert np.array_equal(words, ref.bytes)
    queries = rng.integers(0, 2**64 - 1, size=10_000, dtype=np.uint64)
    assert np.array_equal(oracle_par.parquet_contains(words, num_bytes, queries, threads=4),
                          ref.contains(queries))


def test_oracle_rejects_bad_sizes():
    for nb in (0, 16, 33, 48 + 1):
        with pytest.raises(ValueError):
            oracle.ParquetOracle(nb)


# ---- the library's host-only header functions (no GPU call) -------------------

def _bf():
    from paper_2512_15595_amd import bf

    return bf


@pytest.mark.parametrize("n,ndv,fpp,seed", CASES)
def test_library_header_equals_arrow(n, ndv, fpp, seed):
    bf = _bf()
    rng = np.random.default_rng(seed)
    (blob,) = arrow_blobs(pa.array(rng.integers(0, 2**40, size=n, dtype=np.int64)), ndv, fpp)
    num_bytes, _ = split(blob)
    st, got_nb, header_len = bf.bf_parquet_parse_header(blob)
    assert st == bf.BF_OK
    assert got_nb == num_bytes and header_len + num_bytes == len(blob)
    st, header = bf.bf_parquet_header(num_bytes)
    assert st == bf.BF_OK and header == blob[:header_len]


def test_library_header_round_trip_and_errors():
    bf = _bf()
    for nb in (32, 96, 1 << 20, 128 << 20, (1 << 31) - 32):
        st, h = bf.bf_parquet_header(nb)
        assert st == bf.BF_OK and len(h) <= 20
        assert bf.bf_parquet_parse_header(h + b"\x00" * 8) == (bf.BF_OK, nb, len(h))
    for nb in (0, 16, 33, 1 << 31):
        assert bf.bf_parquet_header(nb)[0] == bf.BF_EINVAL
    st, h = bf.bf_parquet_header(2048)
    for cut in range(len(h)):  # every truncation is malformed
        assert bf.bf_parquet_parse_header(h[:cut])[0] == bf.BF_EINVAL
    # another algorithm / hash / compression (field 2 of the union) is not this format
    other = bytearray(h)
    other[h.index(0x1C) + 1] = 0x2C
    assert bf.bf_parquet_parse_header(bytes(other))[0] == bf.BF_EUNSUPPORTED
    # a field the format might add later (id 5, binary) is skipped
    extended = h[:-1] + bytes([0x18, 3]) + b"abc" + b"\x00"
    assert bf.bf_parquet_parse_header(extended) == (bf.BF_OK, 2048, len(extended))
    # numBytes not a multiple of 32
    assert bf.bf_parquet_parse_header(bytes([0x15, 2 * 40]) + h[2:])[0] == bf.BF_EINVAL


def test_library_rejects_bad_parquet_sizes_without_gpu():
    bf = _bf()
    for nb in (0, 16, 33, (1 << 37) + 32):
        st, _ = bf.bf_create_parquet(nb)
        assert st == bf.BF_EINVAL
        st, _ = bf.bf_create_parquet_in(256, nb)
        assert st == bf.BF_EINVAL


def test_header_parser_survives_arbitrary_bytes():
    """Random and mutated headers: every call returns a status (no crash, no
    hang), and an OK parse stays inside the bytes it was given."""
    bf = _bf()
    rng = np.random.default_rng(12)
    st, good = bf.bf_parquet_header(1 << 20)
    cases = [bytes(rng.integers(0, 256, size=int(n), dtype=np.uint8)) for n in rng.integers(0, 64, size=2000)]
    for _ in range(2000):
        m = bytearray(good + bytes(rng.integers(0, 256, size=8, dtype=np.uint8)))
        for _ in range(int(rng.integers(1, 4))):
            m[int(rng.integers(0, len(m)))] = int(rng.integers(0, 256))
        cases.append(bytes(m))
    for blob in cases:
        st, nb, hl = bf.bf_parquet_parse_header(blob)
        assert st in (bf.BF_OK, bf.BF_EINVAL, bf.BF_EUNSUPPORTED)
        if st == bf.BF_OK:
            assert 0 < hl <= len(blob) and nb > 0 and nb % 32 == 0
