"""Seeded random configurations across every layout, mapping and strategy,
each checked bit-exact against the oracle (filter bytes and every lookup).

Parameters are drawn from the accepted ranges: block counts from 1 to a few
thousand (including non-powers of two), every (s, S), k from its lower bound
to 32 (compiled and runtime values), cache-sectorized group counts, classic
sizes, key counts from 0 to ~70k (ragged tails) at aligned and misaligned
addresses, and every valid execution mapping and construction strategy.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_helpers import log, to_device
from paper_2512_15595_amd import workloads

pytestmark = pytest.mark.gpu


def _bf():
    from paper_2512_15595_amd import bf

    return bf


def _pow2_upto(g, hi):
    return int(2 ** g.integers(0, int(np.log2(hi)) + 1))


def _config(seed):
    g = workloads.rng(10_000 + seed)
    layout = ["sbf", "sbf", "csbf", "classic", "chained"][int(g.integers(0, 5))]
    S = int(g.choice([32, 64]))
    s = _pow2_upto(g, 16)
    cfg = {"layout": layout, "seed": int(g.integers(0, 2**63))}
    if layout == "classic":
        cfg["m"] = 64 * int(g.integers(1, 60_000))
        if g.random() < 0.3:
            cfg["m"] = 1 << int(g.integers(6, 24))
        cfg["k"] = int(g.choice([1, 3, 4, 6, 8, 12, 16, 23, 32]))
    else:
        cfg["b"] = int(g.integers(1, 5000))
        cfg["s"], cfg["S"] = s, S
        if layout == "csbf":
            z = _pow2_upto(g, s)
            cfg["z"] = z
            cfg["k"] = z * int(g.integers(1, 32 // z + 1))
        else:
            cfg["k"] = int(g.integers(s, 33))
    n = int(g.integers(0, 70_000))
    cfg["n"] = n
    cfg["offset"] = int(g.integers(0, 2))
    cfg["g"] = g
    return cfg


def _mapping(bf, cfg, g):
    """A random valid (op, lanes, phi, kt, atomic, strategy) choice per op."""
    lay = cfg["layout"]
    if lay == "classic":
        add = (1, 1, int(g.choice([1, 2, 4])), 0)
        con = (1, 1, int(g.choice([1, 2, 4])), 0)
    elif lay == "chained":
        add = con = (1, cfg["s"], 1, 0)
    elif lay == "csbf":
        def one():
            theta = _pow2_upto(g, cfg["z"])
            kt = int(g.choice([1, 2])) if theta == 1 else 1
            return (theta, cfg["s"] // theta, kt, 0)
        add, con = one(), one()
    else:
        def one(op):
            theta = _pow2_upto(g, cfg["s"])
            phi = _pow2_upto(g, cfg["s"] // theta)
            kt = int(g.choice([1, 2, 4]))
            atomic = 64 if (op == "add" and cfg["S"] == 32 and phi >= 2 and g.random() < 0.5) else 0
            return (theta, phi, kt, atomic)
        add, con = one("add"), one("contains")
    strategies = [bf.BF_STRATEGY_AUTO, bf.BF_STRATEGY_DIRECT]
    partitionable = lay in ("sbf", "csbf") or (lay == "classic" and cfg["k"] in (4, 6, 8, 12, 16))
    if partitionable:
        strategies.append(bf.BF_STRATEGY_PARTITIONED)
    return add, con, int(g.choice(strategies))


def _make(bf, cfg):
    lay = cfg["layout"]
    if lay == "classic":
        return (bf.ClassicFilter(cfg["m"], cfg["k"], cfg["seed"]),
                oracle.ClassicOracle(cfg["m"], cfg["k"], cfg["seed"]))
    if lay == "csbf":
        p = (cfg["b"], cfg["s"], cfg["S"], cfg["z"], cfg["k"], cfg["seed"])
        return bf.CacheSectorizedFilter(*p), oracle.CsbfOracle(*p)
    p = (cfg["b"], cfg["s"], cfg["S"], cfg["k"], cfg["seed"])
    if lay == "chained":
        return bf.ChainedHashFilter(*p), oracle.ChainedOracle(*p)
    return bf.BloomFilter(*p), oracle.OracleFilter(*p)


@pytest.mark.parametrize("seed", range(160))
def test_random_configuration(seed):
    bf = _bf()
    cfg = _config(seed)
    g = cfg.pop("g")
    add_map, con_map, strategy = _mapping(bf, cfg, g)
    log(f"random config {seed}: {cfg} add={add_map} contains={con_map} strategy={strategy}")
    keys = g.integers(0, 2**64, size=cfg["n"], dtype=np.uint64)
    if cfg["n"] > 10 and g.random() < 0.3:
        keys[: cfg["n"] // 3] = keys[0]                 # repeated keys
    queries = np.concatenate([keys[::3], g.integers(0, 2**64, size=3000, dtype=np.uint64)])
    f, ref = _make(bf, cfg)
    try:
        f.set_mapping(bf.BF_OP_ADD, *add_map, strategy=strategy)
        f.set_mapping(bf.BF_OP_CONTAINS, *con_map)
        if keys.size:
            f.add(to_device(keys, cfg["offset"]))
        out = f.contains(to_device(queries, cfg["offset"])).cpu().numpy()
        words = f.words().cpu().numpy()
    finally:
        f.close()
    ref.add(keys)
    assert np.array_equal(words, ref.bytes)
    assert np.array_equal(out, ref.contains(queries))
    assert np.all(out[: keys[::3].size] == 1)
