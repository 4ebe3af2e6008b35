"""bf_add_noalloc (include/bf.h): the add for callers that cannot allocate
device memory.  Its partitioned construction uses the library's static
scratch array; its words must equal those of bf_add (partitioned, workspace
from the pool) bit for bit, on two calls in a row -- the second with a
smaller input, over the array's leftover contents -- and equal the oracle's.
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import log
from paper_2512_15595_amd import workloads

pytestmark = pytest.mark.gpu

NB, S_WORDS, WBITS, K = (16 << 20) // 32, 8, 32, 8   # 16 MiB, 256-bit blocks


def _bf():
    from paper_2512_15595_amd import bf

    return bf


def _dev(keys):
    return torch.from_numpy(np.ascontiguousarray(keys).view(np.int64)).to("cuda")


def _lib():
    from paper_2512_15595_amd import bf

    lib = ctypes.CDLL(bf.LIB_PATH)
    lib.bf_add_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    lib.bf_add_noalloc.restype = ctypes.c_int32
    return lib


@pytest.mark.parametrize("layout", ["sbf_8x32", "sbf_1x64", "csbf_16x64_z4", "classic"])
def test_noalloc_equals_bf_add_on_two_calls(layout):
    bf = _bf()
    lib = _lib()

    def make():
        if layout == "sbf_8x32":
            return bf.BloomFilter(NB, 8, 32, 8, 3), oracle.OracleFilter(NB, 8, 32, 8, 3)
        if layout == "sbf_1x64":
            nb = (16 << 20) // 8
            return bf.BloomFilter(nb, 1, 64, 8, 4), oracle.OracleFilter(nb, 1, 64, 8, 4)
        if layout == "csbf_16x64_z4":
            nb = (16 << 20) // 128
            return (bf.CacheSectorizedFilter(nb, 16, 64, 4, 8, 5),
                    oracle.CsbfOracle(nb, 16, 64, 4, 8, 5))
        return bf.ClassicFilter(1 << 27, 8, 6), oracle.ClassicOracle(1 << 27, 8, 6)

    f_ref, ref = make()
    f_na, _ = make()
    for f in (f_ref, f_na):
        f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
    sizes = (3_000_000, 700_001) if layout != "classic" else (1_000_000, 250_001)
    stream = torch.cuda.current_stream()
    try:
        for call, n in enumerate(sizes):
            keys = workloads.uniform_keys(n, 50 + call)
            d = _dev(keys)
            log(f"noalloc {layout}: call {call + 1} with {n} keys")
            f_ref.add(d)
            rc = lib.bf_add_noalloc(f_na.handle, d.data_ptr(), n, stream.cuda_stream)
            assert rc == 0, bf.bf_strerror(rc)
            torch.cuda.synchronize()
            got, want = f_na.words().cpu().numpy(), f_ref.words().cpu().numpy()
            assert np.array_equal(got, want), f"call {call + 1}"
            ref.add(keys)
            assert np.array_equal(got, ref.bytes), f"call {call + 1} vs oracle"
    finally:
        f_ref.close()
        f_na.close()


def test_noalloc_rejects_adds_beyond_the_array_and_enqueues_nothing():
    bf = _bf()
    lib = _lib()
    f = bf.BloomFilter((1 << 30) // 32, 8, 32, 8, 7)          # 1 GiB
    f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
    n = 16_000_000                                             # needs more than the array
    d = torch.zeros(n, dtype=torch.int64, device="cuda")
    try:
        rc = lib.bf_add_noalloc(f.handle, d.data_ptr(), n, torch.cuda.current_stream().cuda_stream)
        assert rc == bf.BF_ESCRATCH
        assert "scratch" in bf.bf_strerror(rc)
        torch.cuda.synchronize()
        assert int(f.words().count_nonzero().item()) == 0     # nothing was enqueued
        # the direct construction needs no workspace: taken whatever the size
        f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_DIRECT)
        keys = workloads.uniform_keys(100_000, 8)
        dk = _dev(keys)
        assert lib.bf_add_noalloc(f.handle, dk.data_ptr(), keys.size,
                                  torch.cuda.current_stream().cuda_stream) == 0
        torch.cuda.synchronize()
        hits = f.contains(dk)
        assert bool(hits.all().item())
    finally:
        f.close()



def test_noalloc_one_pass_limit_of_a_64_mib_filter():
    """A filter of at most 64 MiB (1024 chunks) is partitioned in one pass,
    about 6 bytes of workspace per key: 40 M keys fit the array and give
    bf_add's words (sampled blocks against the oracle), 46 M do not
    (BF_ESCRATCH, nothing enqueued)."""
    bf = _bf()
    lib = _lib()
    nb = (64 << 20) // 32
    keys = workloads.uniform_keys(46_000_000, 31)
    d = _dev(keys)
    f_na = bf.BloomFilter(nb, 8, 32, 8, 13)
    f_ref = bf.BloomFilter(nb, 8, 32, 8, 13)
    s = torch.cuda.current_stream().cuda_stream
    try:
        for f in (f_na, f_ref):
            f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
        log("noalloc one-pass limit: 46 M keys into 64 MiB (refused)")
        assert lib.bf_add_noalloc(f_na.handle, d.data_ptr(), keys.size, s) == bf.BF_ESCRATCH
        torch.cuda.synchronize()
        assert int(f_na.words().count_nonzero().item()) == 0
        n = 40_000_000
        log("noalloc one-pass limit: 40 M keys into 64 MiB (accepted)")
        assert lib.bf_add_noalloc(f_na.handle, d.data_ptr(), n, s) == 0
        f_ref.add(d[:n])
        got, want = f_na.words().cpu().numpy(), f_ref.words().cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(got, want)
        sel = workloads.rng(32).choice(nb, size=2048, replace=False).astype(np.uint64)
        rows = oracle.block_words(nb, 8, 32, 8, 13, keys[:n], sel)
        assert np.array_equal(got.reshape(nb, 32)[sel.astype(np.int64)], rows)
    finally:
        f_na.close()
        f_ref.close()

def test_noalloc_calls_on_two_streams_do_not_overlap():
    """Two filters, two streams, no caller events: the library orders the
    calls that share the array, so both filters get the oracle's words."""
    bf = _bf()
    fa = bf.BloomFilter(NB, 8, 32, 8, 21)
    fb = bf.BloomFilter(NB, 8, 32, 8, 22)
    for f in (fa, fb):
        f.set_mapping(bf.BF_OP_ADD, strategy=bf.BF_STRATEGY_PARTITIONED)
    ka = [workloads.uniform_keys(2_000_000, 60 + i) for i in range(3)]
    kb = [workloads.uniform_keys(1_500_000, 70 + i) for i in range(3)]
    da, db = [_dev(x) for x in ka], [_dev(x) for x in kb]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    try:
        for x, y in zip(da, db):
            fa.add_noalloc(x, stream=s1)
            fb.add_noalloc(y, stream=s2)
        torch.cuda.synchronize()
        for f, keys, seed in ((fa, ka, 21), (fb, kb, 22)):
            ref = oracle.OracleFilter(NB, 8, 32, 8, seed)
            for x in keys:
                ref.add(x)
            assert np.array_equal(f.words().cpu().numpy(), ref.bytes)
    finally:
        fa.close()
        fb.close()
