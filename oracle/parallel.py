"""Runs the unchanged single-threaded CPU oracle over many host threads --
TEST INFRASTRUCTURE, like the rest of this package: for parity checks at
full size and for the all-core timing of the oracle beside the benchmark.

Nothing here computes a hash, a block or a pattern: every filter byte and
every lookup result comes from one call of the oracle's own C functions.
The work is split so that the calls touch disjoint outputs:

* the words of a filter are built block range by block range
  (``oracle.block_words`` -- or ``csbf_block_words``, or ``classic_words``
  over ranges of 64-bit words -- over a contiguous range, which applies
  exactly the keys that reach the range), and the ranges are concatenated;
* lookups are split into query slices, each answered by
  ``OracleFilter.contains`` semantics over the complete oracle words.

ctypes releases the GIL for the duration of each C call, so the threads run
in parallel.  OR is commutative and idempotent, so the merged result is the
one a single call over all keys gives (tests/test_oracle.py pins the
block-range form against the whole-filter form on small filters).
"""
from __future__ import annotations

import concurrent.futures
import os

import numpy as np

from . import (ClassicOracle, CsbfOracle, OracleFilter, ParquetOracle, block_words,
               classic_words, csbf_block_words, parquet_block_words)


def workers(limit: int = 16) -> int:
    """Threads to use: the CPUs this process may run on, at most `limit`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 4
    return max(1, min(n, limit))


def _ranges(total: int, parts: int):
    parts = max(1, min(parts, total)) if total > 0 else 1
    step = -(-total // parts)
    return [(lo, min(total, lo + step)) for lo in range(0, total, step)] or [(0, 0)]


def _by_ranges(units: int, unit_bytes: int, rows_of, threads: int | None, parts: int | None):
    """Filter bytes assembled from rows_of(sel) -- the oracle's bytes of the
    units (blocks or words) sel -- over contiguous unit ranges."""
    out = np.zeros(units * unit_bytes, dtype=np.uint8)
    threads = threads or workers()

    def one(r):
        lo, hi = r
        if hi > lo:
            rows = rows_of(np.arange(lo, hi, dtype=np.uint64))
            out[lo * unit_bytes:hi * unit_bytes] = np.ascontiguousarray(rows).view(np.uint8).reshape(-1)

    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, _ranges(units, parts or threads)))
    return out


def filter_words(num_blocks: int, words_per_block: int, word_bits: int, k: int, seed: int,
                 keys: np.ndarray, threads: int | None = None, parts: int | None = None) -> np.ndarray:
    """The oracle's filter bytes after adding `keys`, built by block ranges."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    return _by_ranges(num_blocks, words_per_block * word_bits // 8,
                      lambda sel: block_words(num_blocks, words_per_block, word_bits, k, seed, keys, sel),
                      threads, parts)


def csbf_filter_words(num_blocks: int, words_per_block: int, word_bits: int, groups: int, k: int,
                      seed: int, keys: np.ndarray, threads: int | None = None,
                      parts: int | None = None) -> np.ndarray:
    """The cache-sectorized oracle's filter bytes after adding `keys`, by block ranges."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    return _by_ranges(num_blocks, words_per_block * word_bits // 8,
                      lambda sel: csbf_block_words(num_blocks, words_per_block, word_bits, groups, k,
                                                   seed, keys, sel),
                      threads, parts)


def classic_filter_words(num_bits: int, k: int, seed: int, keys: np.ndarray,
                         threads: int | None = None, parts: int | None = None) -> np.ndarray:
    """The classic oracle's filter bytes after adding `keys`, by ranges of
    64-bit words."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    return _by_ranges(num_bits // 64, 8, lambda sel: classic_words(num_bits, k, seed, keys, sel),
                      threads, parts)


def parquet_filter_words(num_bytes: int, values: np.ndarray, threads: int | None = None,
                         parts: int | None = None) -> np.ndarray:
    """The Parquet split-block oracle's bitset after adding `values`, by block ranges."""
    values = np.ascontiguousarray(values, dtype=np.uint64)
    return _by_ranges(num_bytes // 32, 32, lambda sel: parquet_block_words(num_bytes, values, sel),
                      threads, parts)


def lookups(view, queries: np.ndarray, threads: int | None = None) -> np.ndarray:
    """view.contains(q) of every query, by query slices; `view` is an oracle
    filter object (any layout) holding the state to look up in."""
    queries = np.ascontiguousarray(queries, dtype=np.uint64)
    out = np.zeros(queries.size, dtype=np.uint8)
    threads = threads or workers()

    def one(r):
        lo, hi = r
        if hi > lo:
            out[lo:hi] = view.contains(queries[lo:hi])

    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(one, _ranges(queries.size, 4 * threads)))
    return out


def _holding(view, filter_bytes: np.ndarray):
    assert filter_bytes.size == view.nbytes
    view.bytes = filter_bytes  # the zero state it allocated is never touched
    return view


def contains(filter_bytes: np.ndarray, num_blocks: int, words_per_block: int, word_bits: int,
             k: int, seed: int, queries: np.ndarray, threads: int | None = None) -> np.ndarray:
    """The oracle's lookup result of every query against `filter_bytes`
    (oracle words), by query slices."""
    view = _holding(OracleFilter(num_blocks, words_per_block, word_bits, k, seed), filter_bytes)
    return lookups(view, queries, threads)


def csbf_contains(filter_bytes: np.ndarray, num_blocks: int, words_per_block: int, word_bits: int,
                  groups: int, k: int, seed: int, queries: np.ndarray,
                  threads: int | None = None) -> np.ndarray:
    """Cache-sectorized oracle lookups against `filter_bytes`, by query slices."""
    view = _holding(CsbfOracle(num_blocks, words_per_block, word_bits, groups, k, seed), filter_bytes)
    return lookups(view, queries, threads)


def classic_contains(filter_bytes: np.ndarray, num_bits: int, k: int, seed: int,
                     queries: np.ndarray, threads: int | None = None) -> np.ndarray:
    """Classic oracle lookups against `filter_bytes`, by query slices."""
    view = _holding(ClassicOracle(num_bits, k, seed), filter_bytes)
    return lookups(view, queries, threads)


def parquet_contains(filter_bytes: np.ndarray, num_bytes: int, queries: np.ndarray,
                     threads: int | None = None) -> np.ndarray:
    """Parquet split-block oracle lookups against `filter_bytes`, by query slices."""
    view = _holding(ParquetOracle(num_bytes), filter_bytes)
    return lookups(view, queries, threads)


def per_filter(jobs, fn, threads: int | None = None):
    """fn(job) for every job on a thread pool, results in job order (used to
    run one independent oracle filter per job)."""
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads or workers()) as ex:
        return list(ex.map(fn, jobs))
