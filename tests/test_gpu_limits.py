"""GPU parity at the largest accepted sizes: 2^32 blocks (the block rule's
upper half-word path, 16-32 GiB filters) and classic filters of 2^38 and
2^39 + 320 bits (positions beyond 2^32 words, both reduction paths).

The oracle computes each key's block and pattern one by one (for the
cache-sectorized layout, as the words of a one-block oracle filter holding
that key, since a block's contents do not depend on its index); the test
reads every touched block back from the device, checks untouched sampled
blocks are zero, and checks lookups of the inserted keys and of fresh keys
against the expected state.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_helpers import log, read_device_bytes, to_device
from paper_2512_15595_amd import workloads

pytestmark = pytest.mark.gpu


def _bf():
    from paper_2512_15595_amd import bf

    return bf


def _keys(n, seed):
    return workloads.rng(seed).integers(0, 2**64, size=n, dtype=np.uint64)


def _expected_blocks(keys, b, s, S, k, seed, groups=None):
    """block index -> block bytes after adding keys (touched blocks only)."""
    block_bytes = s * S // 8
    out = {}
    for x in keys:
        h = oracle.hash_key(int(x), seed)
        blk = oracle.block_index(h, b)
        if groups is None:
            words = np.array(oracle.pattern(h, s, S, k), dtype=np.uint64)
            pat = words.astype(np.uint32 if S == 32 else np.uint64).view(np.uint8)
        else:
            one = oracle.CsbfOracle(1, s, S, groups, k, seed)
            one.add([x])
            pat = one.bytes
        cur = out.get(blk)
        out[blk] = pat.copy() if cur is None else (cur | pat)
    assert all(v.size == block_bytes for v in out.values())
    return out


def _check_blocks(f, expected, b, block_bytes, seed):
    base = int(f.info().d_words)
    for blk, want in expected.items():
        got = read_device_bytes(base, blk * block_bytes, block_bytes)
        assert np.array_equal(got, want), f"block {blk}"
    g = workloads.rng(seed)
    for blk in g.integers(0, b, size=512, dtype=np.uint64):
        blk = int(blk)
        if blk not in expected:
            assert not read_device_bytes(base, blk * block_bytes, block_bytes).any(), f"block {blk}"


def _lookup_expected(keys, expected, b, s, S, k, seed, groups=None):
    want = np.zeros(keys.size, dtype=np.uint8)
    for i, x in enumerate(keys):
        h = oracle.hash_key(int(x), seed)
        blk = oracle.block_index(h, b)
        if groups is None:
            words = np.array(oracle.pattern(h, s, S, k), dtype=np.uint64)
            pat = words.astype(np.uint32 if S == 32 else np.uint64).view(np.uint8)
        else:
            one = oracle.CsbfOracle(1, s, S, groups, k, seed)
            one.add([x])
            pat = one.bytes
        state = expected.get(blk)
        want[i] = 1 if state is not None and np.array_equal(state & pat, pat) else 0
    return want


@pytest.mark.parametrize("layout", ["sbf_1x32", "csbf_2x32_z2"])
def test_max_block_count(layout):
    bf = _bf()
    b = 1 << 32
    if layout == "sbf_1x32":
        s, S, k, z = 1, 32, 8, None
    else:
        s, S, k, z = 2, 32, 4, 2
    seed = 0xFACE
    adds = _keys(1 << 15, 71)
    fresh = _keys(1 << 14, 72)
    expected = _expected_blocks(adds, b, s, S, k, seed, z)
    queries = np.concatenate([adds[: 1 << 13], fresh])
    want = _lookup_expected(queries, expected, b, s, S, k, seed, z)
    assert want[: 1 << 13].all()
    for strategy in ("DIRECT", "PARTITIONED"):
        log(f"max blocks {layout} strategy={strategy}")
        f = (bf.BloomFilter(b, s, S, k, seed) if z is None
             else bf.CacheSectorizedFilter(b, s, S, z, k, seed))
        try:
            assert f.info().num_blocks == b
            f.set_mapping(bf.BF_OP_ADD, strategy=getattr(bf, "BF_STRATEGY_" + strategy))
            f.add(to_device(adds))
            out = f.contains(to_device(queries)).cpu().numpy()
            _check_blocks(f, expected, b, s * S // 8, 73)
        finally:
            f.close()
        assert np.array_equal(out, want)


@pytest.mark.parametrize("m", [1 << 38, (1 << 39) + 320])
def test_classic_large(m):
    bf = _bf()
    k, seed = 8, 0xBEEF
    adds = _keys(1 << 13, 81)
    fresh = _keys(1 << 13, 82)
    touched = {}
    for x in adds:
        h = oracle.hash_key(int(x), seed)
        for j in range(k):
            p = oracle.classic_position(h, m, j)
            touched[p // 64] = touched.get(p // 64, 0) | (1 << (p % 64))
    queries = np.concatenate([adds, fresh])
    want = np.zeros(queries.size, dtype=np.uint8)
    for i, x in enumerate(queries):
        h = oracle.hash_key(int(x), seed)
        ok = True
        for j in range(k):
            p = oracle.classic_position(h, m, j)
            ok = ok and (touched.get(p // 64, 0) >> (p % 64)) & 1 == 1
        want[i] = 1 if ok else 0
    log(f"classic m={m}")
    f = bf.ClassicFilter(m, k, seed)
    try:
        f.add(to_device(adds))
        out = f.contains(to_device(queries)).cpu().numpy()
        base = int(f.info().d_words)
        for w, v in touched.items():
            got = read_device_bytes(base, w * 8, 8).view("<u8")[0]
            assert int(got) == v, f"word {w}"
        g = workloads.rng(83)
        for w in g.integers(0, m // 64, size=512, dtype=np.uint64):
            if int(w) not in touched:
                assert not read_device_bytes(base, int(w) * 8, 8).any()
        assert any(w >= (1 << 32) // 2 for w in touched)  # 32-bit words beyond 2^32
    finally:
        f.close()
    assert np.array_equal(out, want)
