"""Parity over the cache-resident regime sweep at full size: the four layouts
of the sweep -- register-blocked 1 x 64-bit and 1 x 32-bit words, sectorized
8 x 32-bit (cache-sectorized 8 x 32 with z = 4 / 2 groups for k = 4 / 6,
where a sectorized block needs k >= 8), classic -- at every k of the sweep
(4, 6, 8, 12, 16) on the largest filter (256 MiB) at 16 bits per key
(2^27 uniform keys), and at 1 MiB and 16 MiB at 8 bits per key; plus 2-bit
packed 31-mer keys of a seeded sequence with repeated segments.

Each filter is built with the library's default construction (partitioned at
these densities) and with the direct one; every filter byte, and every
lookup byte of 2^25 queries (half of them inserted keys), is compared with
the CPU oracle (the unchanged single-threaded C on host threads:
oracle/parallel.py).
"""
from __future__ import annotations

import time

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import log
from oracle import parallel as oracle_par
from paper_2512_15595_amd import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

LAYOUTS = ("rbbf_1x64", "rbbf_1x32", "sbf_8x32", "classic")
KS = (4, 6, 8, 12, 16)


def _make(bf, layout, nbytes, k, seed):
    """(GPU filter, a description for the oracle) of one sweep layout."""
    if layout == "rbbf_1x64":
        return bf.BloomFilter(nbytes // 8, 1, 64, k, seed), ("sbf", nbytes // 8, 1, 64, 0)
    if layout == "rbbf_1x32":
        return bf.BloomFilter(nbytes // 4, 1, 32, k, seed), ("sbf", nbytes // 4, 1, 32, 0)
    if layout == "sbf_8x32":
        if k >= 8:
            return bf.BloomFilter(nbytes // 32, 8, 32, k, seed), ("sbf", nbytes // 32, 8, 32, 0)
        z = 4 if k % 4 == 0 else 2
        return (bf.CacheSectorizedFilter(nbytes // 32, 8, 32, z, k, seed),
                ("csbf", nbytes // 32, 8, 32, z))
    return bf.ClassicFilter(nbytes * 8, k, seed), ("classic", nbytes * 8, 0, 0, 0)


def _oracle(desc, k, seed, adds, queries):
    kind, a, s, S, z = desc
    if kind == "sbf":
        w = oracle_par.filter_words(a, s, S, k, seed, adds)
        return w, oracle_par.contains(w, a, s, S, k, seed, queries)
    if kind == "csbf":
        w = oracle_par.csbf_filter_words(a, s, S, z, k, seed, adds)
        return w, oracle_par.csbf_contains(w, a, s, S, z, k, seed, queries)
    w = oracle_par.classic_filter_words(a, k, seed, adds)
    return w, oracle_par.classic_contains(w, a, k, seed, queries)


def _check(layout, nbytes, k, adds, queries, seed):
    from paper_2512_15595_amd import bf

    f, desc = _make(bf, layout, nbytes, k, seed)
    g, _ = _make(bf, layout, nbytes, k, seed)
    d_adds = torch.from_numpy(np.ascontiguousarray(adds).view(np.int64)).to("cuda")
    d_q = torch.from_numpy(np.ascontiguousarray(queries).view(np.int64)).to("cuda")
    try:
        log(f"cache regime {layout} {nbytes >> 20} MiB k={k}: {adds.size} adds "
            f"(default strategy {f.add_strategy(adds.size)}), {queries.size} lookups")
        f.add(d_adds)
        g.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_DIRECT)
        g.add(d_adds)
        direct_equal = bool(torch.equal(f.words(), g.words()))
        out = f.contains(d_q).cpu().numpy()
        words = f.words().cpu().numpy()
        torch.cuda.synchronize()
    finally:
        f.close()
        g.close()
    assert direct_equal, "direct and default construction differ"
    t0 = time.perf_counter()
    want_words, want = _oracle(desc, k, seed, adds, queries)
    log(f"cache regime {layout} {nbytes >> 20} MiB k={k}: oracle in {time.perf_counter() - t0:.1f}s")
    if not np.array_equal(words, want_words):
        bad = np.flatnonzero(words != want_words)
        pytest.fail(f"{bad.size} filter bytes differ from the oracle (first {bad[:8]})")
    if not np.array_equal(out, want):
        bad = np.flatnonzero(out != want)
        pytest.fail(f"{bad.size} lookups differ from the oracle (first {bad[:8]})")


@pytest.fixture(scope="module")
def keys_256mib():
    n = (256 << 20) * 8 // 16                         # 16 bits per key: 2^27 keys
    adds = workloads.uniform_keys(n, 41)
    queries = workloads.mix(adds[: 1 << 25], workloads.uniform_keys(1 << 25, 42), 0.5, 43)
    return adds, queries


@pytest.mark.parametrize("k", KS)
@pytest.mark.parametrize("layout", LAYOUTS)
def test_256mib_every_k_equals_oracle(keys_256mib, layout, k):
    adds, queries = keys_256mib
    _check(layout, 256 << 20, k, adds, queries, seed=1000 + k)


@pytest.mark.parametrize("nbytes", [1 << 20, 16 << 20], ids=["1MiB", "16MiB"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_small_filters_at_8_bits_per_key(layout, nbytes):
    n = nbytes * 8 // 8
    adds = workloads.uniform_keys(n, 51)
    queries = workloads.mix(adds, workloads.uniform_keys(n, 52), 0.5, 53)
    _check(layout, nbytes, 8, adds, queries, seed=7)


@pytest.mark.parametrize("layout", ["sbf_8x32", "classic"])
def test_kmer_keys(layout):
    adds = workloads.kmer_keys((1 << 25) + 30, 61)    # 2^25 31-mers, 10 % repeated segments
    fresh = workloads.kmer_keys((1 << 24) + 30, 62)
    queries = workloads.mix(adds[: fresh.size], fresh, 0.5, 63)
    _check(layout, 64 << 20, 8, adds, queries, seed=9)
