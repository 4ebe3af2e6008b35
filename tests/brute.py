"""Brute-force model of the filter, for tiny inputs only.

Pure Python on top of the independent ``xxhash`` package: a filter is the
set of (block, word, bit) triples its keys set.  It shares no code with the
C oracle or the HIP library and exists to pin the oracle's bit layout,
block rule and pattern rule (paper Sec. II-A-2/4 and Sec. IV-B; the readings
for what the paper leaves open are the same ones the oracle documents).
"""
from __future__ import annotations

import xxhash

SALT_SEED = int.from_bytes(b"bf-salts", "little")
M64 = 2**64 - 1
M32 = 2**32 - 1


def base_hash(key: int, seed: int) -> int:
    return xxhash.xxh64_intdigest((key & M64).to_bytes(8, "little"), seed & M64)


def salts() -> list[int]:
    return [(base_hash(j, SALT_SEED) & M32) | 1 for j in range(32)]


_SALTS = salts()


def triples_of_key(key: int, b: int, s: int, S: int, k: int, seed: int) -> set:
    h = base_hash(key, seed)
    hi, lo = h >> 32, h & M32
    blk = hi * b // 2**32
    L = S.bit_length() - 1
    out = set()
    for j in range(k):
        p = ((lo * _SALTS[j]) & M32) >> (32 - L)
        out.add((blk, j % s, p))
    return out


def build(keys, b: int, s: int, S: int, k: int, seed: int) -> set:
    bits = set()
    for x in keys:
        bits |= triples_of_key(int(x), b, s, S, k, seed)
    return bits


def contains(bits: set, key: int, b: int, s: int, S: int, k: int, seed: int) -> bool:
    return triples_of_key(int(key), b, s, S, k, seed) <= bits


def triples_of_bytes(filter_bytes, s: int, S: int) -> set:
    """Decode a little-endian word array (as bytes) into (block, word, bit)."""
    out = set()
    data = bytes(filter_bytes)
    wbytes = S // 8
    for byte_index, value in enumerate(data):
        if not value:
            continue
        for bit in range(8):
            if (value >> bit) & 1:
                word_index = byte_index // wbytes
                p = (byte_index % wbytes) * 8 + bit
                out.add((word_index // s, word_index % s, p))
    return out


# -- classic filter (Sec. II-A-1): positions anywhere in m bits -------------

def salts64() -> list[int]:
    return [base_hash(j, SALT_SEED) | 1 for j in range(32)]


_SALTS64 = salts64()


def classic_positions(key: int, m: int, k: int, seed: int) -> set:
    h = base_hash(key, seed)
    return {(((h * _SALTS64[j]) & M64) * m) >> 64 for j in range(k)}


def classic_build(keys, m: int, k: int, seed: int) -> set:
    bits = set()
    for x in keys:
        bits |= classic_positions(int(x), m, k, seed)
    return bits


def positions_of_bytes(filter_bytes) -> set:
    """Bit p is bit p % 8 of byte p // 8."""
    out = set()
    for byte_index, value in enumerate(bytes(filter_bytes)):
        for bit in range(8):
            if (value >> bit) & 1:
                out.add(byte_index * 8 + bit)
    return out


# -- cache-sectorized filter (Sec. II-A-5): one word per group --------------

def group_salts() -> list[int]:
    return [(base_hash(32 + g, SALT_SEED) & M32) | 1 for g in range(16)]


_GSALTS = group_salts()


def csbf_triples_of_key(key: int, b: int, s: int, S: int, z: int, k: int, seed: int) -> set:
    h = base_hash(key, seed)
    hi, lo = h >> 32, h & M32
    blk = hi * b // 2**32
    L = S.bit_length() - 1
    width = s // z
    wl = width.bit_length() - 1
    chosen = []
    for g in range(z):
        sel = (((lo * _GSALTS[g]) & M32) >> (32 - wl)) if wl else 0
        chosen.append(g * width + sel)
    out = set()
    for j in range(k):
        p = ((lo * _SALTS[j]) & M32) >> (32 - L)
        out.add((blk, chosen[j % z], p))
    return out


def csbf_build(keys, b: int, s: int, S: int, z: int, k: int, seed: int) -> set:
    bits = set()
    for x in keys:
        bits |= csbf_triples_of_key(int(x), b, s, S, z, k, seed)
    return bits


# -- chained pattern hashing (prior-art rule of Sec. IV-B) -------------------

def chained_triples_of_key(key: int, b: int, s: int, S: int, k: int, seed: int) -> set:
    h = base_hash(key, seed)
    blk = (h >> 32) * b // 2**32
    L = S.bit_length() - 1
    out = set()
    for j in range(k):
        h = base_hash(key, h)
        out.add((blk, j % s, (h & M32) >> (32 - L)))
    return out


def chained_build(keys, b: int, s: int, S: int, k: int, seed: int) -> set:
    bits = set()
    for x in keys:
        bits |= chained_triples_of_key(int(x), b, s, S, k, seed)
    return bits
