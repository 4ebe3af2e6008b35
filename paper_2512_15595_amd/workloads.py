"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module holds no filter arithmetic (no hashing, no block or pattern
rule); it only draws keys.  The paper's workloads are themselves synthetic:
unique uniform random 64-bit keys, lookups either all present or all absent
(Sec. V-A).  All draws use numpy's PCG64 with explicit seeds.
"""
from __future__ import annotations

import math

import numpy as np

U64_MAX = 2**64


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_keys(n: int, seed: int) -> np.ndarray:
    """n uniform uint64 keys from PCG64(seed)."""
    return rng(seed).integers(0, U64_MAX, size=n, dtype=np.uint64)


def affine_permutation(n: int, seed: int) -> np.ndarray:
    """A seeded bijection of range(n): i -> (a*i + c) mod n with gcd(a, n) = 1.

    Used in place of a full random permutation at 2^28 elements, where
    numpy's shuffle alone costs ~10 s; the order of already random keys only
    has to differ from insertion order.
    """
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    g = rng(seed)
    while True:
        a = int(g.integers(1, max(n, 2)))
        if math.gcd(a, n) == 1:
            break
    c = int(g.integers(0, n))
    i = np.arange(n, dtype=np.uint64)
    return ((np.uint64(a) * i + np.uint64(c)) % np.uint64(n)).astype(np.int64)


def mix(hits: np.ndarray, misses: np.ndarray, hit_fraction: float, seed: int) -> np.ndarray:
    """Per position, take the hit with probability hit_fraction, else the miss."""
    assert hits.shape == misses.shape
    if hit_fraction <= 0.0:
        return misses.copy()
    if hit_fraction >= 1.0:
        return hits.copy()
    take = rng(seed).random(hits.size) < hit_fraction
    return np.where(take, hits, misses)


def correctness_workload():
    """The small parity workload: 2^20-bit filter, 4096 blocks x 8 x 32-bit
    words, k = 8, seed 0; 20,000 inserted keys from PCG64(1); 1,000,000
    queries from the same generator: 500,000 drawn with replacement from the
    inserted keys and 500,000 fresh, concatenated and shuffled."""
    g = rng(1)
    adds = g.integers(0, U64_MAX, size=20_000, dtype=np.uint64)
    hits = adds[g.integers(0, adds.size, size=500_000)]
    fresh = g.integers(0, U64_MAX, size=500_000, dtype=np.uint64)
    queries = np.concatenate([hits, fresh])
    queries = queries[g.permutation(queries.size)]
    params = dict(num_blocks=4096, words_per_block=8, word_bits=32, k=8, seed=0)
    return params, adds, queries


def dram_workload(n: int = 2**28, add_seed: int = 1, miss_seed: int = 2,
                  perm_seed: int = 3):
    """The DRAM-resident workload's keys: n inserted keys from PCG64(1); the
    0 % hit queries are n fresh keys from PCG64(2); the 100 % hit queries are
    the inserted keys in a PCG64(3)-seeded order; the 50 % queries mix the
    two position by position."""
    adds = uniform_keys(n, add_seed)
    q0 = uniform_keys(n, miss_seed)
    q100 = adds[affine_permutation(n, perm_seed)]
    q50 = mix(q100, q0, 0.5, perm_seed + 1)
    return adds, {0: q0, 50: q50, 100: q100}


def kmer_keys(n_bases: int, seed: int, k: int = 31, segment: int = 1000,
              repeat_p: float = 0.1) -> np.ndarray:
    """2-bit packed forward k-mers (A=0 C=1 G=2 T=3, first base most
    significant) of a seeded random sequence built in segments, each of which
    is, with probability repeat_p, a copy of an earlier segment."""
    g = rng(seed)
    nseg = max(1, math.ceil(n_bases / segment))
    seq = np.empty(nseg * segment, dtype=np.uint8)
    for i in range(nseg):
        if i > 0 and g.random() < repeat_p:
            j = int(g.integers(0, i))
            seq[i * segment:(i + 1) * segment] = seq[j * segment:(j + 1) * segment]
        else:
            seq[i * segment:(i + 1) * segment] = g.integers(0, 4, size=segment, dtype=np.uint8)
    seq = seq[:n_bases]
    if seq.size < k:
        return np.zeros(0, dtype=np.uint64)
    nk = seq.size - k + 1
    out = np.zeros(nk, dtype=np.uint64)
    for i in range(k):
        out = (out << np.uint64(2)) | seq[i:i + nk].astype(np.uint64)
    return out
