"""The C-ABI library loads, exports every declared symbol and validates its
arguments before touching the GPU (no GPU needed)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2512_15595_amd", "libbf.so")
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def _ensure_built():
    if not os.path.exists(LIB):
        from paper_2512_15595_amd import build

        build.build()


def _declared_functions(path):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(bfb?_[a-z_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_headers_declare_the_boundary():
    names = set()
    for h in HEADERS:
        names |= set(_declared_functions(h))
    for required in ("bf_create", "bf_create_in", "bf_create_classic", "bf_create_csbf",
                     "bf_create_chained",
                     "bf_destroy", "bf_add",
                     "bf_contains", "bf_clear", "bf_info", "bf_add_strategy",
                     "bf_set_mapping", "bf_strerror", "bfb_random_read", "bfb_random_atomic_or",
                     "bfb_gups", "bfb_copy"):
        assert required in names


@pytest.mark.parametrize("header", HEADERS, ids=os.path.basename)
def test_library_exports_every_declared_symbol(header):
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    for name in _declared_functions(header):
        assert hasattr(lib, name), f"{name} declared in {os.path.basename(header)} but not exported"


def test_binding_loads_and_validates_without_gpu():
    _ensure_built()
    from paper_2512_15595_amd import bf

    # invalid parameters are rejected before any HIP call
    for args in [
        (0, 8, 32, 8, 0),           # no blocks
        (2**32 + 1, 8, 32, 8, 0),   # too many blocks
        (4096, 3, 32, 8, 0),        # words per block not a power of two
        (4096, 32, 32, 32, 0),      # more than 16 words
        (4096, 8, 16, 8, 0),        # word width
        (4096, 8, 32, 7, 0),        # k < s
        (4096, 8, 32, 33, 0),       # k > 32
    ]:
        st, h = bf.bf_create(*args)
        assert st == bf.BF_EINVAL, args
        assert not h.value
    # null handles
    assert bf.bf_add(None, 0, 10, 0) == bf.BF_EINVAL
    assert bf.bf_contains(None, 0, 10, 0, 0) == bf.BF_EINVAL
    assert bf.bf_clear(None, 0) == bf.BF_EINVAL
    assert bf.bf_set_mapping(None, 0, 1, 1, 1) == bf.BF_EINVAL
    assert bf.bf_destroy(None) == bf.BF_OK
    st, _ = bf.bf_info(None)
    assert st == bf.BF_EINVAL
    st, _ = bf.bf_add_strategy(None, 1 << 20)
    assert st == bf.BF_EINVAL
    assert bf.bf_strerror(bf.BF_EINVAL) == "invalid argument"
    assert bf.bf_strerror(12345) == "unknown status"


def test_variant_layouts_validate_without_gpu():
    _ensure_built()
    from paper_2512_15595_amd import bf

    for args in [
        (0, 8, 0),                  # no bits
        (96, 8, 0),                 # not a multiple of 64
        ((1 << 40) + 64, 8, 0),     # larger than 2^40 bits
        (1 << 20, 0, 0),            # k = 0
        (1 << 20, 33, 0),           # k > 32
    ]:
        st, h = bf.bf_create_classic(*args)
        assert st == bf.BF_EINVAL, args
        assert not h.value
    for args in [
        (4096, 8, 32, 16, 16, 0),   # z > s
        (4096, 8, 32, 3, 6, 0),     # z not a power of two
        (4096, 8, 32, 4, 6, 0),     # k not a multiple of z
        (4096, 8, 32, 4, 2, 0),     # k < z
        (4096, 8, 32, 2, 34, 0),    # k > 32
        (0, 8, 32, 2, 4, 0),        # no blocks
        (4096, 8, 16, 2, 4, 0),     # word width
        (4096, 6, 32, 2, 4, 0),     # words per block
    ]:
        st, h = bf.bf_create_csbf(*args)
        assert st == bf.BF_EINVAL, args
        assert not h.value
    for args in [(0, 8, 32, 8, 0), (4096, 3, 32, 8, 0), (4096, 8, 16, 8, 0), (4096, 8, 32, 7, 0),
                 (4096, 8, 32, 33, 0), (2**32 + 1, 1, 32, 8, 0)]:
        st, h = bf.bf_create_chained(*args)
        assert st == bf.BF_EINVAL, args
        assert not h.value


def test_create_in_validates_without_gpu():
    _ensure_built()
    from paper_2512_15595_amd import bf

    nb, nbytes = 4096, 4096 * 32
    for args in [
        (nb, 8, 32, 8, 0, 0, nbytes),            # null words
        (nb, 8, 32, 8, 0, 4096, nbytes - 32),    # wrong size
        (nb, 8, 32, 8, 0, 4096 + 128, nbytes),   # not 256-byte aligned
        (nb, 8, 32, 7, 0, 4096, nbytes),         # k < s
        (0, 8, 32, 8, 0, 4096, 0),               # no blocks
    ]:
        st, h = bf.bf_create_in(*args)
        assert st == bf.BF_EINVAL, args
        assert not h.value


def test_bench_library_validates_without_gpu():
    _ensure_built()
    lib = ctypes.CDLL(LIB)
    vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
    lib.bfb_random_read.argtypes = [vp, u64, u32, u32, u64, u32, vp, vp]
    lib.bfb_copy.argtypes = [vp, vp, u64, vp]
    assert lib.bfb_random_read(None, 1 << 20, 32, 1, 100, 0, None, None) == -1
    assert lib.bfb_copy(None, None, 16, None) == -1


def test_product_import_fails_loudly_without_library(tmp_path, monkeypatch):
    """The binding refuses to import when libbf.so is absent (no fallback)."""
    import importlib.util

    src = os.path.join(ROOT, "paper_2512_15595_amd", "bf.py")
    dst = tmp_path / "bf.py"
    dst.write_text(open(src).read())
    spec = importlib.util.spec_from_file_location("bf_copy_without_lib", dst)
    mod = importlib.util.module_from_spec(spec)
    with pytest.raises(ImportError):
        spec.loader.exec_module(mod)
