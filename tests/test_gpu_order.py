"""Stream order of the bf.h calls on one filter.

Adds commute (OR is commutative and idempotent, Sec. II-A-1), so bf_add
calls on one filter from several streams, with no events of the caller's,
must give the oracle's words under every strategy: the library orders a
partitioned add (which loads whole 64 KiB chunks and stores them back)
against every other add of the filter, and a direct add against the last
partitioned one.  bf_destroy waits for its own filter's work only; the
words of a filter destroyed right after its calls were enqueued are still
read by those calls, and other filters' queued work is untouched.
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

NB, S_WORDS, WBITS, K = (16 << 20) // 32, 8, 32, 8   # 16 MiB filter of 256-bit blocks


def _bf():
    from paper_2512_15595_amd import bf

    return bf


def _dev(keys):
    return torch.from_numpy(np.ascontiguousarray(keys).view(np.int64)).to("cuda")


@pytest.mark.parametrize("order", ["partitioned_first", "direct_first", "interleaved"])
def test_adds_from_two_streams_commute_without_caller_events(order):
    bf = _bf()
    seed = 11
    big = [workloads.uniform_keys(4_000_000, 100 + i) for i in range(3)]
    small = [workloads.uniform_keys(200_000 + 1000 * i, 200 + i) for i in range(6)]
    f = bf.BloomFilter(NB, S_WORDS, WBITS, K, seed)
    d_big = [_dev(x) for x in big]
    d_small = [_dev(x) for x in small]
    assert all(f.add_strategy(x.size) == bf.BF_STRATEGY_PARTITIONED for x in big)
    assert all(f.add_strategy(x.size) == bf.BF_STRATEGY_DIRECT for x in small)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    log(f"order {order}: partitioned adds on one stream, direct adds on another")
    if order == "partitioned_first":
        for x in d_big:
            f.add(x, stream=s1)
        for x in d_small:
            f.add(x, stream=s2)
    elif order == "direct_first":
        for x in d_small:
            f.add(x, stream=s2)
        for x in d_big:
            f.add(x, stream=s1)
    else:
        for i in range(6):
            f.add(d_small[i], stream=s2 if i % 2 == 0 else s1)
            if i < 3:
                f.add(d_big[i], stream=s1 if i % 2 == 0 else s2)
    torch.cuda.synchronize()
    words = f.words().cpu().numpy()
    torch.cuda.synchronize()
    f.close()
    ref = oracle.OracleFilter(NB, S_WORDS, WBITS, K, seed)
    for x in big + small:
        ref.add(x)
    assert np.array_equal(words, ref.bytes)


def test_lookups_ordered_by_the_caller_see_every_add():
    """A lookup on a third stream, ordered after both adds by the caller's
    events, sees the union."""
    bf = _bf()
    a = workloads.uniform_keys(3_000_000, 301)
    b = workloads.uniform_keys(50_000, 302)
    f = bf.BloomFilter(NB, S_WORDS, WBITS, K, 3)
    da, db = _dev(a), _dev(b)
    q = np.concatenate([a[:100_000], b, workloads.uniform_keys(100_000, 303)])
    dq = _dev(q)
    s1, s2, s3 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    f.add(da, stream=s1)
    f.add(db, stream=s2)
    s3.wait_stream(s1)
    s3.wait_stream(s2)
    out = f.contains(dq, stream=s3)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    f.close()
    ref = oracle.OracleFilter(NB, S_WORDS, WBITS, K, 3)
    ref.add(a)
    ref.add(b)
    assert np.array_equal(got, ref.contains(q))
    assert got[: 100_000 + b.size].all()


def test_destroy_waits_for_its_own_filter_only():
    """Destroying a filter right after enqueuing its work: the work still
    reads valid words (results equal the oracle), and a second filter's
    queued work on another stream is unaffected."""
    bf = _bf()
    nb_a = (1 << 30) // 32
    keys_a = workloads.uniform_keys(1 << 26, 401)
    q_a = np.concatenate([keys_a[: 1 << 24], workloads.uniform_keys(1 << 24, 402)])
    keys_b = workloads.uniform_keys(2_000_000, 403)
    q_b = np.concatenate([keys_b[:500_000], workloads.uniform_keys(500_000, 404)])
    fa = bf.BloomFilter(nb_a, S_WORDS, WBITS, K, 5)
    fb = bf.BloomFilter(NB, S_WORDS, WBITS, K, 6)
    dka, dqa, dkb, dqb = _dev(keys_a), _dev(q_a), _dev(keys_b), _dev(q_b)
    out_a = torch.full((q_a.size,), 9, dtype=torch.uint8, device="cuda")
    out_b = torch.full((q_b.size,), 9, dtype=torch.uint8, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    log("destroy: long work on filter A (stream 1), filter B destroyed with its work queued (stream 2)")
    fa.add(dka, stream=s1)
    for _ in range(12):                          # ~10 ms of lookups
        fa.contains(dqa, out=out_a, stream=s1)
    done_a = torch.cuda.Event()
    done_a.record(s1)
    fb.add(dkb, stream=s2)
    fb.contains(dqb, out=out_b, stream=s2)
    fb.close()             # releases B's words behind B's calls; no host wait
    a_pending_after_destroy = not done_a.query()
    log(f"destroy: filter A's work still pending when bf_destroy(B) returned: "
        f"{a_pending_after_destroy}")
    torch.cuda.synchronize()
    assert a_pending_after_destroy, "bf_destroy waited for another filter's work"
    got_a, got_b = out_a.cpu().numpy(), out_b.cpu().numpy()
    fa.close()
    ref_b = oracle.OracleFilter(NB, S_WORDS, WBITS, K, 6)
    ref_b.add(keys_b)
    assert np.array_equal(got_b, ref_b.contains(q_b))
    # filter A: present keys all found; a sample of lookups equals the oracle
    assert got_a[: 1 << 24].all()
    sel = workloads.rng(7).choice(q_a.size, size=1 << 14, replace=False)
    blocks = np.unique([oracle.block_index(oracle.hash_key(int(x), 5), nb_a) for x in q_a[sel]])
    rows = oracle.block_words(nb_a, S_WORDS, WBITS, K, 5, keys_a, blocks)
    index = {int(b): i for i, b in enumerate(blocks)}
    want = []
    for x in q_a[sel]:
        h = oracle.hash_key(int(x), 5)
        row = rows[index[oracle.block_index(h, nb_a)]].view("<u4")
        pat = oracle.pattern(h, S_WORDS, WBITS, K)
        want.append(int(all((int(row[w]) & p) == p for w, p in enumerate(pat))))
    assert np.array_equal(got_a[sel], np.array(want, dtype=np.uint8))


def test_destroy_of_an_idle_filter_and_null_stream_use():
    bf = _bf()
    f = bf.BloomFilter(1024, 8, 32, 8, 0)
    f.close()
    g = bf.BloomFilter(1024, 8, 32, 8, 0)
    keys = _dev(workloads.uniform_keys(1000, 9))
    lib = ctypes.CDLL(bf.LIB_PATH)
    lib.bf_add.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p]
    assert lib.bf_add(g.handle, keys.data_ptr(), 1000, None) == 0   # the null stream
    torch.cuda.synchronize()
    ref = oracle.OracleFilter(1024, 8, 32, 8, 0)
    ref.add(workloads.uniform_keys(1000, 9))
    assert np.array_equal(g.words().cpu().numpy(), ref.bytes)
    g.close()


def test_destroyed_words_return_to_the_device():
    """Filter words come from a stream-ordered pool that gives freed memory
    back at the next synchronization: creating and destroying 4 GiB filters
    repeatedly leaves the device's free memory where it was."""
    bf = _bf()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    keys = _dev(workloads.uniform_keys(1_000_000, 501))
    for i in range(6):
        f = bf.BloomFilter((4 << 30) // 32, 8, 32, 8, i)
        f.add(keys)
        hits = f.contains(keys)
        f.close()
        assert bool(hits.all().item())
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    log(f"free memory before {free0 / 2**30:.2f} GiB, after {free1 / 2**30:.2f} GiB")
    assert free1 >= free0 - (1 << 30)
