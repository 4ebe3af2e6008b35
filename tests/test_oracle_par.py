"""The threaded driver of the unchanged oracle (oracle/parallel.py) used by
the full-size parity tests gives exactly what one single-threaded oracle call
gives, for ragged block ranges and query slices."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle import parallel as oracle_par
from paper_2512_15595_amd import workloads


@pytest.mark.parametrize("nb,s,S,k,parts", [(1, 8, 32, 8, 3), (1000, 8, 32, 8, 7),
                                            (4099, 4, 64, 9, 16), (257, 16, 32, 16, 5),
                                            (12345, 1, 64, 8, 13)])
def test_parallel_oracle_equals_single_call(nb, s, S, k, parts):
    keys = workloads.uniform_keys(20_000, nb)
    queries = np.concatenate([keys[::3], workloads.uniform_keys(9_999, nb + 1)])
    ref = oracle.OracleFilter(nb, s, S, k, 77)
    ref.add(keys)
    got = oracle_par.filter_words(nb, s, S, k, 77, keys, threads=4, parts=parts)
    assert np.array_equal(got, ref.bytes)
    out = oracle_par.contains(got, nb, s, S, k, 77, queries, threads=3)
    assert np.array_equal(out, ref.contains(queries))


def test_per_filter_keeps_job_order():
    assert oracle_par.per_filter(list(range(50)), lambda i: i * i, threads=7) == [i * i for i in range(50)]
    assert 1 <= oracle_par.workers() <= 16


@pytest.mark.parametrize("s,S,z,k,parts", [(8, 32, 2, 4, 5), (16, 64, 4, 8, 3), (4, 32, 4, 12, 7)])
def test_parallel_csbf_oracle_equals_single_call(s, S, z, k, parts):
    nb = 3001
    keys = workloads.uniform_keys(15_000, s + z)
    queries = np.concatenate([keys[::5], workloads.uniform_keys(7_001, 3)])
    ref = oracle.CsbfOracle(nb, s, S, z, k, 5)
    ref.add(keys)
    got = oracle_par.csbf_filter_words(nb, s, S, z, k, 5, keys, threads=4, parts=parts)
    assert np.array_equal(got, ref.bytes)
    out = oracle_par.csbf_contains(got, nb, s, S, z, k, 5, queries, threads=3)
    assert np.array_equal(out, ref.contains(queries))


@pytest.mark.parametrize("m,k,parts", [(64 * 1001, 8, 6), (1 << 16, 16, 4), (64 * 37, 4, 9)])
def test_parallel_classic_oracle_equals_single_call(m, k, parts):
    keys = workloads.uniform_keys(3_000, m)
    queries = np.concatenate([keys[::4], workloads.uniform_keys(5_003, 7)])
    ref = oracle.ClassicOracle(m, k, 11)
    ref.add(keys)
    got = oracle_par.classic_filter_words(m, k, 11, keys, threads=4, parts=parts)
    assert np.array_equal(got, ref.bytes)
    out = oracle_par.classic_contains(got, m, k, 11, queries, threads=3)
    assert np.array_equal(out, ref.contains(queries))
