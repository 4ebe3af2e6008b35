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


def zipf_counts(nitems: int, total: int, exponent: float = 1.1, lo: int = 100,
                hi: int = 10_000_000, seed: int = 4) -> np.ndarray:
    """Per-item counts c_r = clip(a * r^-exponent, lo, hi) for ranks r = 1..n,
    with a chosen so the counts sum to `total` (bisection on a, then
    largest-remainder rounding); ranks are given to items by a seeded
    permutation."""
    r = np.arange(1, nitems + 1, dtype=np.float64) ** (-exponent)

    def total_for(a):
        return np.clip(a * r, lo, hi).sum()

    a_lo, a_hi = 0.0, float(hi) * 2
    while total_for(a_hi) < total and a_hi < 1e30:
        a_hi *= 2
    for _ in range(200):
        mid = 0.5 * (a_lo + a_hi)
        if total_for(mid) < total:
            a_lo = mid
        else:
            a_hi = mid
    c = np.clip(a_hi * r, lo, hi)
    c = c * (total / c.sum())
    base = np.floor(c).astype(np.int64)
    short = int(total - base.sum())
    if short > 0:
        base[np.argsort(-(c - base))[:short]] += 1
    return base[rng(seed).permutation(nitems)]


def log_uniform_sizes(nitems: int, lo_bytes: int, hi_bytes: int, align: int, seed: int) -> np.ndarray:
    """Sizes log-uniform on [lo, hi], rounded to a multiple of `align`."""
    u = rng(seed).random(nitems)
    sizes = np.exp(np.log(lo_bytes) + u * (np.log(hi_bytes) - np.log(lo_bytes)))
    return np.maximum(align, np.round(sizes / align).astype(np.int64) * align)


def batched_workload(nfilters: int = 4096, total_keys: int = 2**28, lo_bytes: int = 4 << 10,
                     hi_bytes: int = 16 << 20, block_bytes: int = 32, seed: int = 4,
                     max_count: int = 10_000_000, min_count: int = 100):
    """Many independent filters: sizes log-uniform on [4 KiB, 16 MiB] (rounded
    to whole blocks), key counts Zipf(1.1) clipped to [1e2, 1e7] summing to
    total_keys.  Returns (sizes_bytes, offsets, keys, queries) where filter i
    owns keys[offsets[i]:offsets[i+1]] and the same range of queries; half
    of each filter's queries are its own inserted keys, half fresh keys."""
    sizes = log_uniform_sizes(nfilters, lo_bytes, hi_bytes, block_bytes, seed)
    counts = zipf_counts(nfilters, total_keys, 1.1, min_count, max_count, seed + 1)
    offsets = np.zeros(nfilters + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    keys = uniform_keys(int(offsets[-1]), seed + 2)
    fresh = uniform_keys(int(offsets[-1]), seed + 3)
    g = rng(seed + 4)
    # per position: hit (a key of the same filter, chosen by an in-filter
    # offset) or miss, each with probability 1/2
    owner = np.repeat(np.arange(nfilters), counts)
    start = offsets[:-1][owner]
    pick = start + (g.random(owner.size) * counts[owner]).astype(np.int64)
    hits = keys[pick]
    take = g.random(owner.size) < 0.5
    queries = np.where(take, hits, fresh)
    return sizes, offsets, keys, queries


SPLITMIX_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, first: int, n: int) -> np.ndarray:
    """Elements first..first+n-1 of the SplitMix64 stream `seed` (Steele,
    Lea, Flood 2014): the output function of seed + (i + 1) * gamma.  The
    same definition runs on the device for workloads too large for the host
    (bfb_fill_splitmix64)."""
    with np.errstate(over="ignore"):
        i = np.arange(first, first + n, dtype=np.uint64)
        z = np.uint64(seed) + (i + np.uint64(1)) * SPLITMIX_GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def mixed_queries(n: int, src_seed: int, src_first: int, src_count: int, fresh_seed: int,
                  fresh_first: int, hit_fraction: float, mix_seed: int) -> np.ndarray:
    """Host twin of bfb_fill_mixed_queries."""
    hit_q32 = np.uint64(min(int(hit_fraction * 2**32), 2**32 - 1))
    r = splitmix64(mix_seed, 0, n)
    choose = r >> np.uint64(32)
    pick = ((r & np.uint64(0xFFFFFFFF)) * np.uint64(src_count)) >> np.uint64(32)
    with np.errstate(over="ignore"):
        src = np.uint64(src_seed) + (np.uint64(src_first) + pick + np.uint64(1)) * SPLITMIX_GAMMA
        z = (src ^ (src >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        hits = z ^ (z >> np.uint64(31))
    fresh = splitmix64(fresh_seed, fresh_first, n)
    return np.where(choose < hit_q32, hits, fresh)
