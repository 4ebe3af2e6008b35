"""CPU oracle for the blocked / sectorized Bloom filter -- TEST INFRASTRUCTURE.

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this module.  It wraps ``bf_oracle.c`` (plain
single-threaded C, the definition of what the GPU path computes) through
ctypes and shares nothing with the HIP library.

The filter definition follows "Optimizing Bloom Filters on Modern GPUs"
(arXiv 2512.15595): Sec. II-A-2/3/4 for the blocked, register-blocked and
sectorized layouts, Sec. IV-B for one xxHash64 base hash per key and salted
multiplicative bit positions; Sec. II-A-1 for the classic (unblocked) filter
and Sec. II-A-5 with Sec. V-A for the cache-sectorized filter; the chained
pattern hashing of prior GPU filters (Sec. IV-B) for the optimization
breakdown of Sec. V-E.  ``bf_oracle.h`` lists the readings taken where
the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

SALT_SEED = 0x73746C61732D6662
MAX_K = 32


def build(force: bool = False) -> str:
    """Compile bf_oracle.c into liboracle.so with gcc (host code only)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
             "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        vp = ctypes.c_void_p
        lib.oracle_xxh64.argtypes = [vp, ctypes.c_size_t, u64]
        lib.oracle_xxh64.restype = u64
        lib.oracle_hash_key.argtypes = [u64, u64]
        lib.oracle_hash_key.restype = u64
        lib.oracle_salts.argtypes = [vp]
        lib.oracle_salts.restype = None
        lib.oracle_check_params.argtypes = [u64, u32, u32, u32]
        lib.oracle_check_params.restype = i32
        lib.oracle_block_index.argtypes = [u64, u64]
        lib.oracle_block_index.restype = u64
        lib.oracle_pattern.argtypes = [u64, u32, u32, u32, vp]
        lib.oracle_pattern.restype = i32
        lib.oracle_add.argtypes = [vp, u64, u32, u32, u32, u64, vp, u64]
        lib.oracle_add.restype = i32
        lib.oracle_contains.argtypes = [vp, u64, u32, u32, u32, u64, vp, u64, vp]
        lib.oracle_contains.restype = i32
        lib.oracle_clear.argtypes = [vp, u64]
        lib.oracle_clear.restype = None
        lib.oracle_block_words.argtypes = [u64, u32, u32, u32, u64, vp, u64, vp, u64, vp]
        lib.oracle_block_words.restype = i32
        lib.oracle_salts64.argtypes = [vp]
        lib.oracle_salts64.restype = None
        lib.oracle_classic_position.argtypes = [u64, u64, u32]
        lib.oracle_classic_position.restype = u64
        lib.oracle_classic_add.argtypes = [vp, u64, u32, u64, vp, u64]
        lib.oracle_classic_add.restype = i32
        lib.oracle_classic_contains.argtypes = [vp, u64, u32, u64, vp, u64, vp]
        lib.oracle_classic_contains.restype = i32
        lib.oracle_classic_words.argtypes = [u64, u32, u64, vp, u64, vp, u64, vp]
        lib.oracle_classic_words.restype = i32
        lib.oracle_check_csbf_params.argtypes = [u64, u32, u32, u32, u32]
        lib.oracle_check_csbf_params.restype = i32
        lib.oracle_group_salts.argtypes = [vp]
        lib.oracle_group_salts.restype = None
        lib.oracle_csbf_add.argtypes = [vp, u64, u32, u32, u32, u32, u64, vp, u64]
        lib.oracle_csbf_add.restype = i32
        lib.oracle_csbf_contains.argtypes = [vp, u64, u32, u32, u32, u32, u64, vp, u64, vp]
        lib.oracle_csbf_contains.restype = i32
        lib.oracle_csbf_block_words.argtypes = [u64, u32, u32, u32, u32, u64, vp, u64, vp,
                                                u64, vp]
        lib.oracle_csbf_block_words.restype = i32
        lib.oracle_chained_add.argtypes = [vp, u64, u32, u32, u32, u64, vp, u64]
        lib.oracle_chained_add.restype = i32
        lib.oracle_chained_contains.argtypes = [vp, u64, u32, u32, u32, u64, vp, u64, vp]
        lib.oracle_chained_contains.restype = i32
        lib.oracle_parquet_add.argtypes = [vp, u64, vp, u64]
        lib.oracle_parquet_add.restype = i32
        lib.oracle_parquet_contains.argtypes = [vp, u64, vp, u64, vp]
        lib.oracle_parquet_contains.restype = i32
        lib.oracle_parquet_block_words.argtypes = [u64, vp, u64, vp, u64, vp]
        lib.oracle_parquet_block_words.restype = i32
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _keys(keys) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))


def xxh64(data: bytes, seed: int = 0) -> int:
    buf = np.frombuffer(bytes(data) + b"\0", dtype=np.uint8)
    return int(_load().oracle_xxh64(_ptr(buf), len(data), seed & (2**64 - 1)))


def hash_key(key: int, seed: int = 0) -> int:
    return int(_load().oracle_hash_key(key & (2**64 - 1), seed & (2**64 - 1)))


def salts() -> list[int]:
    out = np.zeros(MAX_K, dtype=np.uint32)
    _load().oracle_salts(_ptr(out))
    return [int(v) for v in out]


def check_params(num_blocks: int, words_per_block: int, word_bits: int, k: int) -> bool:
    if not (0 <= num_blocks < 2**64):
        return False
    return _load().oracle_check_params(num_blocks, words_per_block, word_bits, k) == 0


def block_index(h: int, num_blocks: int) -> int:
    return int(_load().oracle_block_index(h, num_blocks))


def pattern(h: int, words_per_block: int, word_bits: int, k: int) -> list[int]:
    out = np.zeros(16, dtype=np.uint64)
    rc = _load().oracle_pattern(h, words_per_block, word_bits, k, _ptr(out))
    if rc != 0:
        raise ValueError("bad filter parameters")
    return [int(v) for v in out[:words_per_block]]


class OracleFilter:
    """Host-memory filter state driven by the C oracle."""

    def __init__(self, num_blocks: int, words_per_block: int, word_bits: int,
                 k: int, seed: int = 0):
        if not check_params(num_blocks, words_per_block, word_bits, k):
            raise ValueError("bad filter parameters")
        self.num_blocks = num_blocks
        self.words_per_block = words_per_block
        self.word_bits = word_bits
        self.k = k
        self.seed = seed & (2**64 - 1)
        self.nbytes = num_blocks * words_per_block * word_bits // 8
        self.bytes = np.zeros(self.nbytes, dtype=np.uint8)

    def _args(self):
        return (self.num_blocks, self.words_per_block, self.word_bits, self.k, self.seed)

    def add(self, keys) -> None:
        keys = _keys(keys)
        rc = _load().oracle_add(_ptr(self.bytes), *self._args(), _ptr(keys), keys.size)
        assert rc == 0

    def contains(self, keys) -> np.ndarray:
        keys = _keys(keys)
        out = np.zeros(max(keys.size, 1), dtype=np.uint8)
        rc = _load().oracle_contains(_ptr(self.bytes), *self._args(), _ptr(keys),
                                     keys.size, _ptr(out))
        assert rc == 0
        return out[: keys.size]

    def clear(self) -> None:
        _load().oracle_clear(_ptr(self.bytes), self.nbytes)

    def words(self) -> np.ndarray:
        """The state as little-endian words of ``word_bits`` bits."""
        dt = np.dtype("<u4") if self.word_bits == 32 else np.dtype("<u8")
        return self.bytes.view(dt)


def block_words(num_blocks: int, words_per_block: int, word_bits: int, k: int,
                seed: int, keys, blocks) -> np.ndarray:
    """Bytes of the selected blocks after adding ``keys`` (one row per block)."""
    keys = _keys(keys)
    sel = np.ascontiguousarray(np.asarray(blocks, dtype=np.uint64))
    block_bytes = words_per_block * word_bits // 8
    out = np.zeros((max(sel.size, 1), block_bytes), dtype=np.uint8)
    rc = _load().oracle_block_words(num_blocks, words_per_block, word_bits, k,
                                    seed & (2**64 - 1), _ptr(keys), keys.size,
                                    _ptr(sel), sel.size, _ptr(out))
    if rc != 0:
        raise ValueError("bad parameters or block selection")
    return out[: sel.size]


def salts64() -> list[int]:
    out = np.zeros(MAX_K, dtype=np.uint64)
    _load().oracle_salts64(_ptr(out))
    return [int(v) for v in out]


def group_salts() -> list[int]:
    out = np.zeros(16, dtype=np.uint32)
    _load().oracle_group_salts(_ptr(out))
    return [int(v) for v in out]


def classic_position(h: int, num_bits: int, j: int) -> int:
    return int(_load().oracle_classic_position(h & (2**64 - 1), num_bits, j))


def check_classic_params(num_bits: int, k: int) -> bool:
    return num_bits >= 64 and num_bits % 64 == 0 and 1 <= k <= MAX_K


def check_csbf_params(num_blocks: int, words_per_block: int, word_bits: int,
                      groups: int, k: int) -> bool:
    if not (0 <= num_blocks < 2**64):
        return False
    return _load().oracle_check_csbf_params(num_blocks, words_per_block, word_bits,
                                            groups, k) == 0


class ClassicOracle:
    """Classic filter of ``num_bits`` bits (Sec. II-A-1) in host memory."""

    def __init__(self, num_bits: int, k: int, seed: int = 0):
        if not check_classic_params(num_bits, k):
            raise ValueError("bad filter parameters")
        self.num_bits, self.k, self.seed = num_bits, k, seed & (2**64 - 1)
        self.nbytes = num_bits // 8
        self.bytes = np.zeros(self.nbytes, dtype=np.uint8)

    def add(self, keys) -> None:
        keys = _keys(keys)
        rc = _load().oracle_classic_add(_ptr(self.bytes), self.num_bits, self.k, self.seed,
                                        _ptr(keys), keys.size)
        assert rc == 0

    def contains(self, keys) -> np.ndarray:
        keys = _keys(keys)
        out = np.zeros(max(keys.size, 1), dtype=np.uint8)
        rc = _load().oracle_classic_contains(_ptr(self.bytes), self.num_bits, self.k,
                                             self.seed, _ptr(keys), keys.size, _ptr(out))
        assert rc == 0
        return out[: keys.size]

    def clear(self) -> None:
        _load().oracle_clear(_ptr(self.bytes), self.nbytes)


def classic_words(num_bits: int, k: int, seed: int, keys, words) -> np.ndarray:
    """Selected 64-bit words of a classic filter after adding ``keys``."""
    keys = _keys(keys)
    sel = np.ascontiguousarray(np.asarray(words, dtype=np.uint64))
    out = np.zeros(max(sel.size, 1), dtype=np.uint64)
    rc = _load().oracle_classic_words(num_bits, k, seed & (2**64 - 1), _ptr(keys), keys.size,
                                      _ptr(sel), sel.size, _ptr(out))
    if rc != 0:
        raise ValueError("bad parameters or word selection")
    return out[: sel.size]


class CsbfOracle:
    """Cache-sectorized filter (Sec. II-A-5) in host memory."""

    def __init__(self, num_blocks: int, words_per_block: int, word_bits: int,
                 groups: int, k: int, seed: int = 0):
        if not check_csbf_params(num_blocks, words_per_block, word_bits, groups, k):
            raise ValueError("bad filter parameters")
        self.num_blocks = num_blocks
        self.words_per_block = words_per_block
        self.word_bits = word_bits
        self.groups = groups
        self.k = k
        self.seed = seed & (2**64 - 1)
        self.nbytes = num_blocks * words_per_block * word_bits // 8
        self.bytes = np.zeros(self.nbytes, dtype=np.uint8)

    def _args(self):
        return (self.num_blocks, self.words_per_block, self.word_bits, self.groups, self.k,
                self.seed)

    def add(self, keys) -> None:
        keys = _keys(keys)
        rc = _load().oracle_csbf_add(_ptr(self.bytes), *self._args(), _ptr(keys), keys.size)
        assert rc == 0

    def contains(self, keys) -> np.ndarray:
        keys = _keys(keys)
        out = np.zeros(max(keys.size, 1), dtype=np.uint8)
        rc = _load().oracle_csbf_contains(_ptr(self.bytes), *self._args(), _ptr(keys),
                                          keys.size, _ptr(out))
        assert rc == 0
        return out[: keys.size]

    def clear(self) -> None:
        _load().oracle_clear(_ptr(self.bytes), self.nbytes)

    def words(self) -> np.ndarray:
        dt = np.dtype("<u4") if self.word_bits == 32 else np.dtype("<u8")
        return self.bytes.view(dt)


def csbf_block_words(num_blocks: int, words_per_block: int, word_bits: int, groups: int,
                     k: int, seed: int, keys, blocks) -> np.ndarray:
    """Bytes of the selected blocks of a cache-sectorized filter after ``keys``."""
    keys = _keys(keys)
    sel = np.ascontiguousarray(np.asarray(blocks, dtype=np.uint64))
    block_bytes = words_per_block * word_bits // 8
    out = np.zeros((max(sel.size, 1), block_bytes), dtype=np.uint8)
    rc = _load().oracle_csbf_block_words(num_blocks, words_per_block, word_bits, groups, k,
                                         seed & (2**64 - 1), _ptr(keys), keys.size,
                                         _ptr(sel), sel.size, _ptr(out))
    if rc != 0:
        raise ValueError("bad parameters or block selection")
    return out[: sel.size]


class ChainedOracle(OracleFilter):
    """Sectorized filter with chained pattern hashing (prior-art rule, Sec. IV-B)."""

    def add(self, keys) -> None:
        keys = _keys(keys)
        rc = _load().oracle_chained_add(_ptr(self.bytes), *self._args(), _ptr(keys), keys.size)
        assert rc == 0

    def contains(self, keys) -> np.ndarray:
        keys = _keys(keys)
        out = np.zeros(max(keys.size, 1), dtype=np.uint8)
        rc = _load().oracle_chained_contains(_ptr(self.bytes), *self._args(), _ptr(keys),
                                             keys.size, _ptr(out))
        assert rc == 0
        return out[: keys.size]


class ParquetOracle:
    """Parquet split-block filter of num_bytes bytes (the format's bitset)."""

    def __init__(self, num_bytes: int):
        if num_bytes < 32 or num_bytes % 32 or num_bytes // 32 > 2**32:
            raise ValueError("num_bytes must be a multiple of 32 in [32, 2^37]")
        self.nbytes = num_bytes
        self.bytes = np.zeros(num_bytes, dtype=np.uint8)

    def add(self, values) -> None:
        values = _keys(values)
        assert _load().oracle_parquet_add(_ptr(self.bytes), self.nbytes, _ptr(values), values.size) == 0

    def contains(self, values) -> np.ndarray:
        values = _keys(values)
        out = np.zeros(max(values.size, 1), dtype=np.uint8)
        assert _load().oracle_parquet_contains(_ptr(self.bytes), self.nbytes, _ptr(values),
                                               values.size, _ptr(out)) == 0
        return out[: values.size]

    def clear(self) -> None:
        _load().oracle_clear(_ptr(self.bytes), self.nbytes)


def parquet_block_words(num_bytes: int, values, blocks) -> np.ndarray:
    """Bytes of the selected blocks of a Parquet split-block filter after
    adding ``values`` (one 32-byte row per block)."""
    values = _keys(values)
    sel = np.ascontiguousarray(np.asarray(blocks, dtype=np.uint64))
    out = np.zeros((max(sel.size, 1), 32), dtype=np.uint8)
    rc = _load().oracle_parquet_block_words(num_bytes, _ptr(values), values.size, _ptr(sel),
                                            sel.size, _ptr(out))
    if rc != 0:
        raise ValueError("bad parameters or block selection")
    return out[: sel.size]
