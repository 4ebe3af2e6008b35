"""Helpers for GPU parity tests: device round trips through the C ABI."""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import torch


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def to_device(keys: np.ndarray, offset_elems: int = 0) -> torch.Tensor:
    """Copies uint64 keys to the GPU; with offset_elems > 0 the returned view
    starts that many elements into a larger allocation (misaligned for wide
    per-lane loads)."""
    host = torch.from_numpy(np.ascontiguousarray(keys).view(np.int64))
    if offset_elems == 0:
        return host.to("cuda")
    buf = torch.zeros(keys.size + offset_elems, dtype=torch.int64, device="cuda")
    buf[offset_elems:] = host.to("cuda")
    return buf[offset_elems:]


def valid_mappings(s: int, word_bits: int):
    """Every (theta, phi, kt, atomic_bits) the library compiles for compiled k."""
    out = []
    theta = 1
    while theta <= min(s, 16):
        phi = 1
        while theta * phi <= s:
            for kt in (1, 2, 4):
                out.append((theta, phi, kt, 32))
                if word_bits == 32 and phi >= 2:
                    out.append((theta, phi, kt, 64))
            phi *= 2
        theta *= 2
    return out


_hip = None


def hip():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


def read_device_bytes(dev_ptr: int, offset: int, nbytes: int) -> np.ndarray:
    """Synchronous device-to-host copy of nbytes at dev_ptr + offset."""
    out = np.zeros(nbytes, dtype=np.uint8)
    rc = hip().hipMemcpy(out.ctypes.data, dev_ptr + offset, nbytes, 2)  # DeviceToHost
    assert rc == 0, f"hipMemcpy failed: {rc}"
    return out
