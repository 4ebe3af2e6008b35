"""Thin Python binding of the C ABI in include/bf.h (argument marshalling only).

Low-level functions carry the C names and take plain integers for device
pointers and streams; every step of add / contains / clear runs in the HIP
kernels of libbf.so.  ``BloomFilter`` wraps them for torch tensors, taking
device memory and the current stream from torch and nothing else.

Importing this module loads libbf.so and raises ImportError if it has not
been built (``python -m paper_2512_15595_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbf.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -m paper_2512_15595_amd.build)"
    )

_lib = ctypes.CDLL(LIB_PATH)

BF_OK = 0
BF_EINVAL = -1
BF_ENOMEM = -2
BF_EDEVICE = -3
BF_EUNSUPPORTED = -4
BF_ESCRATCH = -5
BF_NOALLOC_SCRATCH_BYTES = 256 << 20
BF_OP_ADD = 0
BF_OP_CONTAINS = 1
BF_STRATEGY_AUTO = 0
BF_STRATEGY_DIRECT = 1
BF_STRATEGY_PARTITIONED = 2
BF_LAYOUT_SECTORIZED = 0
BF_LAYOUT_CLASSIC = 1
BF_LAYOUT_CACHE_SECTORIZED = 2
BF_LAYOUT_SECTORIZED_CHAINED = 3
BF_LAYOUT_PARQUET = 4


class bf_mapping_t(ctypes.Structure):
    _fields_ = [
        ("lanes_per_key", ctypes.c_uint32),
        ("words_per_lane", ctypes.c_uint32),
        ("keys_per_lane", ctypes.c_uint32),
        ("atomic_bits", ctypes.c_uint32),
        ("max_workgroups", ctypes.c_uint32),
        ("strategy", ctypes.c_uint32),
        ("workgroup_threads", ctypes.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class bf_info_t(ctypes.Structure):
    _fields_ = [
        ("num_blocks", ctypes.c_uint64),
        ("words_per_block", ctypes.c_uint32),
        ("word_bits", ctypes.c_uint32),
        ("k", ctypes.c_uint32),
        ("device", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("size_bytes", ctypes.c_uint64),
        ("d_words", ctypes.c_void_p),
        ("mapping", bf_mapping_t * 2),
        ("layout", ctypes.c_uint32),
        ("groups", ctypes.c_uint32),
        ("num_bits", ctypes.c_uint64),
    ]


_u64, _u32, _i32, _vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_void_p
_lib.bf_create.argtypes = [_u64, _u32, _u32, _u32, _u64, ctypes.POINTER(_vp)]
_lib.bf_create.restype = _i32
_lib.bf_create_in.argtypes = [_u64, _u32, _u32, _u32, _u64, _vp, _u64, ctypes.POINTER(_vp)]
_lib.bf_create_in.restype = _i32
_lib.bf_create_classic.argtypes = [_u64, _u32, _u64, ctypes.POINTER(_vp)]
_lib.bf_create_classic.restype = _i32
_lib.bf_create_csbf.argtypes = [_u64, _u32, _u32, _u32, _u32, _u64, ctypes.POINTER(_vp)]
_lib.bf_create_csbf.restype = _i32
_lib.bf_create_chained.argtypes = [_u64, _u32, _u32, _u32, _u64, ctypes.POINTER(_vp)]
_lib.bf_create_chained.restype = _i32
_lib.bf_create_parquet.argtypes = [_u64, ctypes.POINTER(_vp)]
_lib.bf_create_parquet.restype = _i32
_lib.bf_create_parquet_in.argtypes = [_vp, _u64, ctypes.POINTER(_vp)]
_lib.bf_create_parquet_in.restype = _i32
_lib.bf_parquet_header.argtypes = [_u64, _vp, _u64, ctypes.POINTER(_u64)]
_lib.bf_parquet_header.restype = _i32
_lib.bf_parquet_parse_header.argtypes = [_vp, _u64, ctypes.POINTER(_u64), ctypes.POINTER(_u64)]
_lib.bf_parquet_parse_header.restype = _i32
_lib.bf_destroy.argtypes = [_vp]
_lib.bf_destroy.restype = _i32
_lib.bf_add.argtypes = [_vp, _vp, _u64, _vp]
_lib.bf_add.restype = _i32
_lib.bf_contains.argtypes = [_vp, _vp, _u64, _vp, _vp]
_lib.bf_contains.restype = _i32
_lib.bf_clear.argtypes = [_vp, _vp]
_lib.bf_clear.restype = _i32
_lib.bf_info.argtypes = [_vp, ctypes.POINTER(bf_info_t)]
_lib.bf_info.restype = _i32
_lib.bf_tuned_mapping.argtypes = [ctypes.c_int, _u64, _u32, _u32, _u32, _u64,
                                  ctypes.POINTER(bf_mapping_t)]
_lib.bf_tuned_mapping.restype = _i32
_lib.bf_add_noalloc.argtypes = [_vp, _vp, _u64, _vp]
_lib.bf_add_noalloc.restype = _i32
_lib.bf_add_strategy.argtypes = [_vp, _u64, ctypes.POINTER(_u32)]
_lib.bf_add_strategy.restype = _i32
_lib.bf_set_mapping.argtypes = [_vp, ctypes.c_int, _u32, _u32, _u32]
_lib.bf_set_mapping.restype = _i32
_lib.bf_set_mapping_ex.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(bf_mapping_t)]
_lib.bf_set_mapping_ex.restype = _i32
_lib.bf_export_words.argtypes = [_vp, _vp, _u64, _vp]
_lib.bf_export_words.restype = _i32
_lib.bf_import_words.argtypes = [_vp, _vp, _u64, _vp]
_lib.bf_import_words.restype = _i32
class bf_batch_info_t(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_uint32),
        ("nfilters", ctypes.c_uint32),
        ("nkeys", ctypes.c_uint64),
        ("ntiles", ctypes.c_uint64),
        ("grid", ctypes.c_uint32),
        ("tiles_per_class", ctypes.c_uint32 * 3),
        ("mapping", bf_mapping_t * 3),
        ("strategy", ctypes.c_uint32),
    ]


_lib.bf_batch_plan.argtypes = [ctypes.c_int, ctypes.POINTER(_vp), _u32, _vp,
                               ctypes.POINTER(_u64), _vp, ctypes.POINTER(_vp)]
_lib.bf_batch_plan.restype = _i32
for _name in ("bf_batch_launch", "bf_batch_launch_direct", "bf_batch_launch_per_filter"):
    getattr(_lib, _name).argtypes = [_vp, _vp]
    getattr(_lib, _name).restype = _i32
_lib.bf_batch_info.argtypes = [_vp, ctypes.POINTER(bf_batch_info_t)]
_lib.bf_batch_info.restype = _i32
_lib.bf_batch_destroy.argtypes = [_vp]
_lib.bf_batch_destroy.restype = _i32
class bf_server_config_t(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("max_inflight", ctypes.c_uint32),
        ("nstreams", ctypes.c_uint32),
        ("coalesce_max_keys", ctypes.c_uint64),
        ("coalesce_max_requests", ctypes.c_uint32),
        ("coalesce_max_tiles", ctypes.c_uint32),
    ]


class bf_request_t(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_uint32),
        ("filter", ctypes.c_uint32),
        ("d_keys", ctypes.c_void_p),
        ("n", ctypes.c_uint64),
        ("d_out", ctypes.c_void_p),
        ("arrival_ns", ctypes.c_uint64),
    ]


class bf_request_result_t(ctypes.Structure):
    _fields_ = [
        ("arrival_ns", ctypes.c_uint64),
        ("admit_ns", ctypes.c_uint64),
        ("complete_ns", ctypes.c_uint64),
        ("launch", ctypes.c_uint32),
        ("status", ctypes.c_int32),
    ]


class bf_server_stats_t(ctypes.Structure):
    _fields_ = [
        ("requests", ctypes.c_uint64),
        ("launches", ctypes.c_uint64),
        ("coalesced_launches", ctypes.c_uint64),
        ("peak_inflight_bytes", ctypes.c_uint64),
        ("peak_inflight_launches", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


_lib.bf_server_create.argtypes = [ctypes.POINTER(_vp), _u32, ctypes.POINTER(bf_server_config_t),
                                  ctypes.POINTER(_vp)]
_lib.bf_server_create.restype = _i32
_lib.bf_server_submit.argtypes = [_vp, ctypes.POINTER(bf_request_t), ctypes.POINTER(_u64)]
_lib.bf_server_submit.restype = _i32
_lib.bf_server_wait.argtypes = [_vp, ctypes.POINTER(_u64), _u64, ctypes.POINTER(bf_request_result_t)]
_lib.bf_server_wait.restype = _i32
for _name in ("bf_server_replay", "bf_server_replay_serial"):
    getattr(_lib, _name).argtypes = [_vp, ctypes.POINTER(bf_request_t), _u64,
                                     ctypes.POINTER(bf_request_result_t)]
    getattr(_lib, _name).restype = _i32
_lib.bf_server_stats.argtypes = [_vp, ctypes.POINTER(bf_server_stats_t)]
_lib.bf_server_stats.restype = _i32
_lib.bf_server_destroy.argtypes = [_vp]
_lib.bf_server_destroy.restype = _i32
_lib.bf_strerror.argtypes = [_i32]
_lib.bf_strerror.restype = ctypes.c_char_p


class BfError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {bf_strerror(status)} ({status})" if what else bf_strerror(status))


def _check(status: int, what: str) -> None:
    if status != BF_OK:
        raise BfError(status, what)


# ---- C names, plain integers -------------------------------------------------

def bf_create(num_blocks: int, words_per_block: int, word_bits: int, k: int, seed: int):
    """Returns (status, handle)."""
    h = _vp()
    st = _lib.bf_create(num_blocks, words_per_block, word_bits, k, seed & (2**64 - 1),
                        ctypes.byref(h))
    return st, h


def bf_create_in(num_blocks: int, words_per_block: int, word_bits: int, k: int, seed: int,
                 d_words: int, nbytes: int):
    """Returns (status, handle) of a filter over caller-owned device words."""
    h = _vp()
    st = _lib.bf_create_in(num_blocks, words_per_block, word_bits, k, seed & (2**64 - 1), d_words,
                           nbytes, ctypes.byref(h))
    return st, h


def bf_create_classic(num_bits: int, k: int, seed: int):
    """Returns (status, handle)."""
    h = _vp()
    st = _lib.bf_create_classic(num_bits, k, seed & (2**64 - 1), ctypes.byref(h))
    return st, h


def bf_create_csbf(num_blocks: int, words_per_block: int, word_bits: int, groups: int, k: int,
                   seed: int):
    """Returns (status, handle)."""
    h = _vp()
    st = _lib.bf_create_csbf(num_blocks, words_per_block, word_bits, groups, k,
                             seed & (2**64 - 1), ctypes.byref(h))
    return st, h


def bf_create_chained(num_blocks: int, words_per_block: int, word_bits: int, k: int, seed: int):
    """Returns (status, handle)."""
    h = _vp()
    st = _lib.bf_create_chained(num_blocks, words_per_block, word_bits, k, seed & (2**64 - 1),
                                ctypes.byref(h))
    return st, h


def bf_create_parquet(num_bytes: int):
    """Returns (status, handle) of a Parquet split-block filter (bf_parquet.h)."""
    h = _vp()
    st = _lib.bf_create_parquet(num_bytes, ctypes.byref(h))
    return st, h


def bf_create_parquet_in(d_words: int, num_bytes: int):
    """Returns (status, handle) of a Parquet split-block filter over caller-owned words."""
    h = _vp()
    st = _lib.bf_create_parquet_in(d_words, num_bytes, ctypes.byref(h))
    return st, h


def bf_parquet_header(num_bytes: int):
    """Returns (status, header bytes) of the format's bloom filter header."""
    buf = (ctypes.c_uint8 * 32)()
    n = _u64(0)
    st = _lib.bf_parquet_header(num_bytes, buf, len(buf), ctypes.byref(n))
    return st, bytes(buf[: n.value]) if st == BF_OK else b""


def bf_parquet_parse_header(blob: bytes):
    """Returns (status, num_bytes, header_len) of a bloom filter header at the
    start of blob."""
    buf = (ctypes.c_uint8 * max(len(blob), 1)).from_buffer_copy(bytes(blob) or b"\0")
    nb, hl = _u64(0), _u64(0)
    st = _lib.bf_parquet_parse_header(buf, len(blob), ctypes.byref(nb), ctypes.byref(hl))
    return st, nb.value, hl.value


def bf_destroy(f) -> int:
    return _lib.bf_destroy(f)


def bf_add(f, d_keys: int, n: int, stream: int = 0) -> int:
    return _lib.bf_add(f, d_keys, n, stream)


def bf_tuned_mapping(op: int, num_blocks: int, words_per_block: int, word_bits: int, k: int,
                     n: int):
    """(status, bf_mapping_t): the default mapping and strategy of an
    operation of n keys on such a filter (host only)."""
    out = bf_mapping_t()
    st = _lib.bf_tuned_mapping(op, num_blocks, words_per_block, word_bits, k, n, ctypes.byref(out))
    return st, out


def bf_add_noalloc(f, d_keys: int, n: int, stream: int = 0) -> int:
    return _lib.bf_add_noalloc(f, d_keys, n, stream)


def bf_contains(f, d_keys: int, n: int, d_out: int, stream: int = 0) -> int:
    return _lib.bf_contains(f, d_keys, n, d_out, stream)


def bf_clear(f, stream: int = 0) -> int:
    return _lib.bf_clear(f, stream)


def bf_info(f):
    """Returns (status, bf_info_t)."""
    info = bf_info_t()
    st = _lib.bf_info(f, ctypes.byref(info))
    return st, info


def bf_add_strategy(f, n: int):
    """Returns (status, BF_STRATEGY_DIRECT or BF_STRATEGY_PARTITIONED): the
    construction an add of n keys takes with the filter's current mapping."""
    out = _u32(0)
    st = _lib.bf_add_strategy(f, n, ctypes.byref(out))
    return st, out.value


def bf_set_mapping(f, op: int, lanes_per_key: int, words_per_lane: int, keys_per_lane: int) -> int:
    return _lib.bf_set_mapping(f, op, lanes_per_key, words_per_lane, keys_per_lane)


def bf_set_mapping_ex(f, op: int, lanes_per_key: int = 0, words_per_lane: int = 0,
                      keys_per_lane: int = 0, atomic_bits: int = 0, max_workgroups: int = 0,
                      strategy: int = 0, workgroup_threads: int = 0) -> int:
    m = bf_mapping_t(lanes_per_key, words_per_lane, keys_per_lane, atomic_bits, max_workgroups,
                     strategy, workgroup_threads)
    return _lib.bf_set_mapping_ex(f, op, ctypes.byref(m))


def bf_export_words(f, dst: int, nbytes: int, stream: int = 0) -> int:
    return _lib.bf_export_words(f, dst, nbytes, stream)


def bf_import_words(f, src: int, nbytes: int, stream: int = 0) -> int:
    return _lib.bf_import_words(f, src, nbytes, stream)


def bf_batch_plan(op: int, filters, d_keys: int, offsets, d_out: int = 0):
    """Returns (status, plan).  filters: handles; offsets: nfilters + 1 ints."""
    arr = (_vp * len(filters))(*[f.value if isinstance(f, _vp) else f for f in filters])
    offs = (_u64 * len(offsets))(*[int(o) for o in offsets])
    plan = _vp()
    st = _lib.bf_batch_plan(op, arr, len(filters), d_keys, offs, d_out, ctypes.byref(plan))
    return st, plan


def bf_batch_launch(plan, stream: int = 0) -> int:
    return _lib.bf_batch_launch(plan, stream)


def bf_batch_launch_direct(plan, stream: int = 0) -> int:
    return _lib.bf_batch_launch_direct(plan, stream)


def bf_batch_launch_per_filter(plan, stream: int = 0) -> int:
    return _lib.bf_batch_launch_per_filter(plan, stream)


def bf_batch_info(plan):
    info = bf_batch_info_t()
    st = _lib.bf_batch_info(plan, ctypes.byref(info))
    return st, info


def bf_batch_destroy(plan) -> int:
    return _lib.bf_batch_destroy(plan)


def bf_strerror(status: int) -> str:
    return _lib.bf_strerror(status).decode()


# ---- torch convenience wrapper ----------------------------------------------

def _stream_ptr(stream) -> int:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class _Filter:
    """Methods shared by every layout; subclasses create the handle."""

    _h = None

    def _adopt(self, st: int, h, what: str) -> None:
        _check(st, what)
        self._h = h
        info = self.info()
        self.device = int(info.device)
        self.layout = int(info.layout)
        self.k = int(info.k)
        self._nbytes = int(info.size_bytes)

    @property
    def handle(self):
        return self._h

    def close(self) -> None:
        if self._h:
            _check(bf_destroy(self._h), "bf_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _keys(self, keys):
        import torch

        if keys.dtype not in (torch.uint64, torch.int64) or not keys.is_cuda or not keys.is_contiguous():
            raise ValueError("keys must be a contiguous uint64/int64 CUDA tensor")
        return keys

    def add(self, keys, stream=None) -> None:
        keys = self._keys(keys)
        _check(bf_add(self._h, keys.data_ptr(), keys.numel(), _stream_ptr(stream)), "bf_add")

    def add_noalloc(self, keys, stream=None) -> None:
        """bf_add_noalloc: as add, with no device allocation (a partitioned
        add uses the library's static scratch array)."""
        keys = self._keys(keys)
        _check(bf_add_noalloc(self._h, keys.data_ptr(), keys.numel(), _stream_ptr(stream)),
               "bf_add_noalloc")

    def contains(self, keys, out=None, stream=None):
        import torch

        keys = self._keys(keys)
        if out is None:
            out = torch.empty(keys.numel(), dtype=torch.uint8, device=keys.device)
        if out.numel() < keys.numel() or out.dtype not in (torch.uint8, torch.bool) or not out.is_contiguous():
            raise ValueError("out must be a contiguous uint8/bool tensor with one byte per key")
        _check(bf_contains(self._h, keys.data_ptr(), keys.numel(), out.data_ptr(),
                           _stream_ptr(stream)), "bf_contains")
        return out

    def clear(self, stream=None) -> None:
        _check(bf_clear(self._h, _stream_ptr(stream)), "bf_clear")

    def info(self) -> bf_info_t:
        st, info = bf_info(self._h)
        _check(st, "bf_info")
        return info

    def add_strategy(self, n: int) -> int:
        """BF_STRATEGY_DIRECT or BF_STRATEGY_PARTITIONED: how an add of n keys
        is built with the current mapping."""
        st, strategy = bf_add_strategy(self._h, n)
        _check(st, "bf_add_strategy")
        return strategy

    def set_mapping(self, op: int, lanes_per_key: int = 0, words_per_lane: int = 0,
                    keys_per_lane: int = 0, atomic_bits: int = 0, max_workgroups: int = 0,
                    strategy: int = 0, workgroup_threads: int = 0) -> None:
        _check(bf_set_mapping_ex(self._h, op, lanes_per_key, words_per_lane, keys_per_lane,
                                 atomic_bits, max_workgroups, strategy, workgroup_threads),
               "bf_set_mapping_ex")

    def words(self, stream=None):
        """A device copy of the words as a torch uint8 tensor."""
        import torch

        out = torch.empty(self.size_bytes(), dtype=torch.uint8, device=f"cuda:{self.device}")
        _check(bf_export_words(self._h, out.data_ptr(), out.numel(), _stream_ptr(stream)),
               "bf_export_words")
        return out

    def load_words(self, src, stream=None) -> None:
        """Overwrites the words from a uint8 tensor of size_bytes bytes."""
        if not src.is_contiguous() or src.numel() * src.element_size() != self.size_bytes():
            raise ValueError("src must be contiguous and exactly size_bytes long")
        _check(bf_import_words(self._h, src.data_ptr(), self.size_bytes(), _stream_ptr(stream)),
               "bf_import_words")

    def size_bytes(self) -> int:
        return self._nbytes


class BloomFilter(_Filter):
    """Sectorized filter (bf_create): keys and results are torch tensors on the GPU."""

    def __init__(self, num_blocks: int, words_per_block: int = 8, word_bits: int = 32,
                 k: int = 8, seed: int = 0):
        self.num_blocks = num_blocks
        self.words_per_block = words_per_block
        self.word_bits = word_bits
        self.seed = seed
        st, h = bf_create(num_blocks, words_per_block, word_bits, k, seed)
        self._adopt(st, h, "bf_create")


class BloomFilterView(_Filter):
    """Sectorized filter over a caller-owned torch tensor (bf_create_in); the
    tensor must stay alive while the filter is used and is not zeroed."""

    def __init__(self, words, num_blocks: int, words_per_block: int = 8, word_bits: int = 32,
                 k: int = 8, seed: int = 0):
        if not words.is_cuda or not words.is_contiguous():
            raise ValueError("words must be a contiguous CUDA tensor")
        self.num_blocks = num_blocks
        self.words_per_block = words_per_block
        self.word_bits = word_bits
        self.seed = seed
        self._words = words  # keeps the storage alive
        st, h = bf_create_in(num_blocks, words_per_block, word_bits, k, seed, words.data_ptr(),
                             words.numel() * words.element_size())
        self._adopt(st, h, "bf_create_in")


class ClassicFilter(_Filter):
    """Classic filter of num_bits bits (bf_create_classic)."""

    def __init__(self, num_bits: int, k: int = 8, seed: int = 0):
        self.num_bits = num_bits
        self.seed = seed
        st, h = bf_create_classic(num_bits, k, seed)
        self._adopt(st, h, "bf_create_classic")


class ChainedHashFilter(_Filter):
    """Sectorized filter with chained pattern hashing (bf_create_chained)."""

    def __init__(self, num_blocks: int, words_per_block: int = 8, word_bits: int = 32,
                 k: int = 8, seed: int = 0):
        self.num_blocks = num_blocks
        self.words_per_block = words_per_block
        self.word_bits = word_bits
        self.seed = seed
        st, h = bf_create_chained(num_blocks, words_per_block, word_bits, k, seed)
        self._adopt(st, h, "bf_create_chained")


class CacheSectorizedFilter(_Filter):
    """Cache-sectorized filter with z = groups word groups (bf_create_csbf)."""

    def __init__(self, num_blocks: int, words_per_block: int = 8, word_bits: int = 32,
                 groups: int = 2, k: int = 8, seed: int = 0):
        self.num_blocks = num_blocks
        self.words_per_block = words_per_block
        self.word_bits = word_bits
        self.groups = groups
        self.seed = seed
        st, h = bf_create_csbf(num_blocks, words_per_block, word_bits, groups, k, seed)
        self._adopt(st, h, "bf_create_csbf")


class ParquetFilter(_Filter):
    """Parquet split-block filter of num_bytes bytes (bf_create_parquet):
    values are int64 / uint64 tensors (DOUBLE columns: their IEEE-754 bits)."""

    def __init__(self, num_bytes: int):
        st, h = bf_create_parquet(num_bytes)
        self._adopt(st, h, "bf_create_parquet")

    @classmethod
    def from_parquet_blob(cls, blob: bytes) -> "ParquetFilter":
        """A filter holding the bitset of a serialized bloom filter (the
        format's header followed by the bitset, as a Parquet file stores it);
        the copy is enqueued on the current stream."""
        import torch

        st, num_bytes, header_len = bf_parquet_parse_header(blob)
        _check(st, "bf_parquet_parse_header")
        if len(blob) < header_len + num_bytes:
            raise ValueError("blob is shorter than its header says")
        f = cls(num_bytes)
        bits = torch.frombuffer(bytearray(blob[header_len:header_len + num_bytes]), dtype=torch.uint8)
        f.load_words(bits.to(f"cuda:{f.device}"))
        return f

    def to_parquet_blob(self) -> bytes:
        """The format's header followed by the bitset, read on the current
        stream (waits for it)."""
        st, header = bf_parquet_header(self.size_bytes())
        _check(st, "bf_parquet_header")
        return header + self.words().cpu().numpy().tobytes()


class BatchPlan:
    """One batched add or contains over many filters (include/bf_batch.h).

    keys: one contiguous uint64/int64 CUDA tensor holding every filter's keys
    back to back; offsets: nfilters + 1 host integers; out (contains): a uint8
    CUDA tensor of the same length as keys.  The tensors must outlive the plan.
    """

    def __init__(self, op: int, filters, keys, offsets, out=None):
        self._keep = (list(filters), keys, out)
        st, plan = bf_batch_plan(op, [f.handle for f in filters], keys.data_ptr(), offsets,
                                 out.data_ptr() if out is not None else 0)
        _check(st, "bf_batch_plan")
        self._plan = plan

    def launch(self, stream=None) -> None:
        _check(bf_batch_launch(self._plan, _stream_ptr(stream)), "bf_batch_launch")

    def launch_direct(self, stream=None) -> None:
        _check(bf_batch_launch_direct(self._plan, _stream_ptr(stream)), "bf_batch_launch_direct")

    def launch_per_filter(self, stream=None) -> None:
        _check(bf_batch_launch_per_filter(self._plan, _stream_ptr(stream)),
               "bf_batch_launch_per_filter")

    def info(self) -> bf_batch_info_t:
        st, info = bf_batch_info(self._plan)
        _check(st, "bf_batch_info")
        return info

    def close(self) -> None:
        if self._plan:
            _check(bf_batch_destroy(self._plan), "bf_batch_destroy")
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The request loop of include/bf_serve.h over a list of BloomFilter."""

    def __init__(self, filters, hbm_budget_bytes: int = 16 << 30, max_inflight: int = 16,
                 nstreams: int = 8, coalesce_max_keys: int = 65536,
                 coalesce_max_requests: int = 256, coalesce_max_tiles: int = 16384):
        self._filters = list(filters)
        cfg = bf_server_config_t(hbm_budget_bytes, max_inflight, nstreams, coalesce_max_keys,
                                 coalesce_max_requests, coalesce_max_tiles)
        arr = (_vp * len(self._filters))(*[f.handle.value for f in self._filters])
        h = _vp()
        _check(_lib.bf_server_create(arr, len(self._filters), ctypes.byref(cfg), ctypes.byref(h)),
               "bf_server_create")
        self._h = h

    @staticmethod
    def requests(ops, filters, keys_ptrs, ns, out_ptrs, arrivals_ns):
        n = len(ops)
        reqs = (bf_request_t * n)()
        for i in range(n):
            reqs[i] = bf_request_t(int(ops[i]), int(filters[i]), int(keys_ptrs[i]), int(ns[i]),
                                   int(out_ptrs[i]) if out_ptrs[i] else None, int(arrivals_ns[i]))
        return reqs

    def replay(self, reqs, serial: bool = False):
        res = (bf_request_result_t * len(reqs))()
        fn = _lib.bf_server_replay_serial if serial else _lib.bf_server_replay
        _check(fn(self._h, reqs, len(reqs), res), "bf_server_replay")
        return res

    def submit(self, req: bf_request_t) -> int:
        rid = _u64()
        _check(_lib.bf_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)), "bf_server_submit")
        return int(rid.value)

    def wait(self, ids):
        arr = (_u64 * len(ids))(*ids)
        res = (bf_request_result_t * len(ids))()
        _check(_lib.bf_server_wait(self._h, arr, len(ids), res), "bf_server_wait")
        return res

    def stats(self) -> bf_server_stats_t:
        st = bf_server_stats_t()
        _check(_lib.bf_server_stats(self._h, ctypes.byref(st)), "bf_server_stats")
        return st

    def close(self) -> None:
        if self._h:
            _check(_lib.bf_server_destroy(self._h), "bf_server_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
