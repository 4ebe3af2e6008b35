"""Pins for the CPU oracle (no GPU needed).

Each test ties the oracle to something other than itself: the independent
python-xxhash library, a brute-force set model on tiny filters, closed forms,
special cases of the block rule, and invariants of a Bloom filter.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import xxhash
from hypothesis import given, settings, strategies as st

import brute
import fpr_model
import oracle

M64 = 2**64 - 1
LAYOUTS = [(s, S) for S in (32, 64) for s in (1, 2, 4, 8, 16)]


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _keys(n, seed):
    return _rng(seed).integers(0, 2**64, size=n, dtype=np.uint64)


# --------------------------------------------------------------------------
# xxHash64 (paper Sec. IV-B: the per-key base hash)
# --------------------------------------------------------------------------

def test_xxh64_matches_library_all_lengths():
    rng = _rng(11)
    for length in list(range(0, 80)) + [127, 128, 129, 1000, 4096]:
        data = rng.integers(0, 256, size=length, dtype=np.uint8).tobytes()
        for seed in (0, 1, 0x9E3779B97F4A7C15, M64):
            assert oracle.xxh64(data, seed) == xxhash.xxh64_intdigest(data, seed)


def test_hash_key_matches_library():
    keys = [0, 1, 42, 2**63, M64] + [int(x) for x in _keys(2000, 12)]
    for seed in (0, 7, 2**32 + 5, M64):
        for key in keys:
            want = xxhash.xxh64_intdigest(key.to_bytes(8, "little"), seed)
            assert oracle.hash_key(key, seed) == want


def test_salts_are_derived_odd_and_distinct():
    got = oracle.salts()
    assert got == brute.salts()
    assert all(a % 2 == 1 for a in got)
    assert len(set(got)) == 32
    assert oracle.SALT_SEED == int.from_bytes(b"bf-salts", "little")


# --------------------------------------------------------------------------
# Block rule (Sec. II-A-2) special cases
# --------------------------------------------------------------------------

def test_block_index_power_of_two_is_top_bits():
    hashes = [int(x) for x in _keys(3000, 13)]
    for e in range(0, 33):
        b = 2**e
        for h in hashes:
            want = (h >> 32) >> (32 - e) if e < 32 else (h >> 32)
            assert oracle.block_index(h, b) == want


def test_block_index_single_block_and_range():
    hashes = [int(x) for x in _keys(3000, 14)] + [0, M64]
    for h in hashes:
        assert oracle.block_index(h, 1) == 0
        for b in (3, 5, 1000, 4096, 2**32 - 1, 2**32):
            assert 0 <= oracle.block_index(h, b) < b
    # the largest hash lands in the last block, the smallest in the first
    for b in (3, 5, 2**20 + 7, 2**32):
        assert oracle.block_index(M64, b) == b - 1
        assert oracle.block_index(0, b) == 0


def test_block_choice_is_uniform():
    b = 37
    counts = np.zeros(b)
    for key in _keys(37000, 15):
        counts[oracle.block_index(oracle.hash_key(int(key), 3), b)] += 1
    expected = 1000.0
    chi2 = float(np.sum((counts - expected) ** 2 / expected))
    # 36 degrees of freedom: P(chi2 > 80) is about 3e-5
    assert chi2 < 80


# --------------------------------------------------------------------------
# Pattern rule (Sec. II-A-4 and IV-B) special cases
# --------------------------------------------------------------------------

def test_parameter_validation():
    assert oracle.check_params(4096, 8, 32, 8)
    assert not oracle.check_params(4096, 8, 32, 7)        # k < s
    assert not oracle.check_params(4096, 3, 32, 8)        # s not a power of two
    assert not oracle.check_params(4096, 32, 32, 32)      # s > 16
    assert not oracle.check_params(4096, 8, 16, 8)        # S not 32/64
    assert not oracle.check_params(4096, 8, 32, 33)       # k > 32
    assert not oracle.check_params(0, 8, 32, 8)           # no blocks
    assert oracle.check_params(2**32, 1, 64, 1)
    assert not oracle.check_params(2**32 + 1, 1, 64, 1)


def test_k_equals_s_sets_one_bit_per_word():
    for s, S in LAYOUTS:
        for key in _keys(200, 16):
            pats = oracle.pattern(oracle.hash_key(int(key), 0), s, S, s)
            assert all(bin(p).count("1") == 1 for p in pats)


def test_register_blocked_popcount_bounds():
    for S in (32, 64):
        for k in (1, 4, 8, 16, 32):
            for key in _keys(200, 17):
                (p,) = oracle.pattern(oracle.hash_key(int(key), 0), 1, S, k)
                assert 1 <= bin(p).count("1") <= k
                assert p < 2**S


def test_bits_spread_round_robin_over_words():
    """Bit j lands in word j mod s: with k = s + 1 word 0 holds up to 2 bits."""
    for s, S in LAYOUTS:
        for key in _keys(100, 18):
            h = oracle.hash_key(int(key), 5)
            pats = oracle.pattern(h, s, S, min(32, s + 1))
            counts = [bin(p).count("1") for p in pats]
            assert 1 <= counts[0] <= 2
            assert all(c == 1 for c in counts[1:])


# --------------------------------------------------------------------------
# Brute force on tiny filters: explicit bit-set equality
# --------------------------------------------------------------------------

@pytest.mark.parametrize("s,S", LAYOUTS)
def test_oracle_bits_equal_brute_force(s, S):
    rng = _rng(100 + s * S)
    for b in (1, 2, 3, 5, 8, 64):
        for k in sorted({s, s + 1, 2 * s, 16, 32}):
            if k < s or k > 32:
                continue
            n = int(rng.integers(0, 201))
            seed = int(rng.integers(0, 2**64, dtype=np.uint64))
            keys = rng.integers(0, 2**64, size=n, dtype=np.uint64)
            f = oracle.OracleFilter(b, s, S, k, seed)
            f.add(keys)
            assert brute.triples_of_bytes(f.bytes, s, S) == brute.build(keys, b, s, S, k, seed)
            # lookups: every inserted key plus fresh ones, against set containment
            queries = np.concatenate([keys, rng.integers(0, 2**64, size=300, dtype=np.uint64)])
            got = f.contains(queries)
            bits = brute.build(keys, b, s, S, k, seed)
            want = [brute.contains(bits, int(q), b, s, S, k, seed) for q in queries]
            assert got.tolist() == [int(w) for w in want]


def test_word_layout_is_little_endian():
    """A one-key filter: each set bit p of word (blk, w) is found at byte
    (blk*s + w)*S/8 + p//8, bit p%8."""
    for s, S in LAYOUTS:
        b, k, seed = 7, max(s, 8), 9
        for key in _keys(20, 19):
            f = oracle.OracleFilter(b, s, S, k, seed)
            f.add([key])
            h = oracle.hash_key(int(key), seed)
            blk = oracle.block_index(h, b)
            pats = oracle.pattern(h, s, S, k)
            words = f.words()
            expect = np.zeros(b * s, dtype=np.uint64)
            for w, p in enumerate(pats):
                expect[blk * s + w] = p
            assert [int(x) for x in words] == [int(x) for x in expect]


# --------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------

@settings(max_examples=40, deadline=None)
@given(
    layout=st.sampled_from(LAYOUTS),
    b=st.integers(1, 300),
    extra_k=st.integers(0, 16),
    seed=st.integers(0, M64),
    keys=st.lists(st.integers(0, M64), min_size=0, max_size=120),
)
def test_no_false_negatives_and_order_independence(layout, b, extra_k, seed, keys):
    s, S = layout
    k = min(32, s + extra_k)
    keys = np.array(keys, dtype=np.uint64)
    f = oracle.OracleFilter(b, s, S, k, seed)
    f.add(keys)
    assert np.all(f.contains(keys) == 1)                      # no false negatives
    g = oracle.OracleFilter(b, s, S, k, seed)
    g.add(keys[::-1])                                         # reversed order
    g.add(keys[: len(keys) // 2])                             # duplicates are idempotent
    assert np.array_equal(f.bytes, g.bytes)


@settings(max_examples=30, deadline=None)
@given(
    layout=st.sampled_from(LAYOUTS),
    b=st.integers(1, 200),
    seed=st.integers(0, M64),
    a=st.lists(st.integers(0, M64), max_size=80),
    c=st.lists(st.integers(0, M64), max_size=80),
)
def test_union_is_wordwise_or_and_monotone(layout, b, seed, a, c):
    s, S = layout
    k = max(s, 8)
    fa = oracle.OracleFilter(b, s, S, k, seed)
    fa.add(np.array(a, dtype=np.uint64))
    fc = oracle.OracleFilter(b, s, S, k, seed)
    fc.add(np.array(c, dtype=np.uint64))
    fu = oracle.OracleFilter(b, s, S, k, seed)
    fu.add(np.array(a + c, dtype=np.uint64))
    assert np.array_equal(fu.bytes, fa.bytes | fc.bytes)
    # monotone: adding more keys never clears a bit
    assert np.array_equal(fu.bytes & fa.bytes, fa.bytes)


def test_clear_resets_everything():
    f = oracle.OracleFilter(64, 8, 32, 8, 1)
    f.add(_keys(1000, 20))
    assert f.bytes.any()
    f.clear()
    assert not f.bytes.any()


def test_block_words_matches_full_filter():
    for s, S in ((8, 32), (4, 64), (1, 32), (16, 64)):
        b, k, seed = 5000, max(s, 8), 3
        keys = _keys(40000, 21)
        f = oracle.OracleFilter(b, s, S, k, seed)
        f.add(keys)
        sel = _rng(22).choice(b, size=300, replace=False).astype(np.uint64)
        got = oracle.block_words(b, s, S, k, seed, keys, sel)
        rows = f.bytes.reshape(b, -1)[sel.astype(np.int64)]
        assert np.array_equal(got, rows)


# --------------------------------------------------------------------------
# Statistics: false-positive rate and fill fraction against the closed form
# --------------------------------------------------------------------------

FPR_CASES = [
    # (s, S, k, b, n)      chosen so ~1e4+ false positives come cheaply
    (1, 32, 4, 2048, 8192),
    (1, 64, 8, 1024, 4096),
    (2, 32, 4, 2048, 12000),
    (4, 64, 8, 512, 12000),
    (8, 32, 8, 1024, 24000),
    (16, 64, 16, 128, 10000),
    (8, 64, 12, 256, 12000),
]


@pytest.mark.parametrize("s,S,k,b,n", FPR_CASES)
def test_false_positive_rate_matches_closed_form(s, S, k, b, n):
    p = fpr_model.sbf_fpr(n, b, s, S, k)
    R = 8
    queries = max(200_000, int(math.ceil(2e4 / (R * p))))
    rates = []
    for r in range(R):
        rng = _rng(1000 + r)
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        keys = rng.integers(0, 2**64, size=n, dtype=np.uint64)
        f = oracle.OracleFilter(b, s, S, k, seed)
        f.add(keys)
        fresh = rng.integers(0, 2**64, size=queries, dtype=np.uint64)
        rates.append(float(f.contains(fresh).mean()))
    rates = np.array(rates)
    assert rates.sum() * queries >= 1e4
    se = rates.std(ddof=1) / math.sqrt(R)
    assert abs(rates.mean() - p) <= 4 * se + 0.01 * p, (rates.mean(), p, se)


@pytest.mark.parametrize("s,S,k,b,n", FPR_CASES)
def test_fill_fraction_matches_closed_form(s, S, k, b, n):
    want = fpr_model.sbf_fill_fraction(n, b, s, S, k)
    got = []
    for r in range(4):
        rng = _rng(2000 + r)
        f = oracle.OracleFilter(b, s, S, k, int(rng.integers(0, 2**63)))
        f.add(rng.integers(0, 2**64, size=n, dtype=np.uint64))
        got.append(np.unpackbits(f.bytes).mean())
    total_bits = b * s * S
    # binomial-scale tolerance on the pooled fraction, plus 0.2 % model slack
    tol = 5 * math.sqrt(want * (1 - want) / (4 * total_bits)) + 0.002 * want
    assert abs(np.mean(got) - want) <= tol, (np.mean(got), want)


def test_fpr_model_pins():
    """The model itself: its cover probabilities equal inclusion-exclusion
    with exact rationals, and for one word per block holding one key per
    bit position it reproduces the textbook counts."""
    for d, S, M in ((1, 32, 1), (3, 32, 10), (5, 64, 40), (8, 32, 100)):
        dp = fpr_model.cover_probs(d, S, M)[M]
        assert math.isclose(dp, fpr_model.cover_prob_inclusion_exclusion(d, S, M),
                            rel_tol=1e-9, abs_tol=1e-15)
    # one inserted key, k = s = 1: the query collides iff the same block and bit
    for S in (32, 64):
        b = 10
        want = (1 / b) * (1 / S)
        assert math.isclose(fpr_model.sbf_fpr(1, b, 1, S, 1), want, rel_tol=1e-12)
    # many blocks, few keys per block: approaches the classic Eq. (1) shape
    # when each block's word is large relative to its load
    assert fpr_model.sbf_fpr(0, 100, 8, 32, 8) == 0.0
