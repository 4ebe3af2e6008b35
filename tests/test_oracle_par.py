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
