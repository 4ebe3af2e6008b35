"""Pins for the oracle's classic (Sec. II-A-1) and cache-sectorized
(Sec. II-A-5) filters (no GPU needed).

Each test ties the oracle to something other than itself: a brute-force set
model on top of the python-xxhash library, the closed form of the fastrange
reduction for power-of-two sizes, the exact reduction of the cache-sectorized
filter with one word per group to the sectorized filter (itself pinned in
test_oracle.py), the structure of a one-key filter, Bloom-filter invariants,
and the false-positive rate and fill fraction against closed forms (for the
classic filter also Eq. (1)).
"""
from __future__ import annotations

import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import brute
import fpr_model
import oracle

M64 = 2**64 - 1


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _keys(n, seed):
    return _rng(seed).integers(0, 2**64, size=n, dtype=np.uint64)


CSBF_LAYOUTS = [(s, S, z) for S in (32, 64) for s in (1, 2, 4, 8, 16)
                for z in (1, 2, 4, 8, 16) if z <= s]


# --------------------------------------------------------------------------
# Classic filter
# --------------------------------------------------------------------------

def test_salts64_derivation():
    """64-bit salts are XXH64 of j under the salt seed, forced odd; their low
    halves are the 32-bit salts of the blocked layouts."""
    got = oracle.salts64()
    assert got == brute.salts64()
    assert all(v & 1 for v in got) and len(set(got)) == 32
    assert [v & 0xFFFFFFFF for v in got] == oracle.salts()


def test_classic_position_power_of_two_is_top_bits():
    """For m = 2^L the fastrange reduction is the top L bits of h * A_j."""
    A = brute.salts64()
    for L in (6, 7, 13, 20, 33, 40):
        m = 1 << L
        for h in _keys(200, L):
            h = int(h)
            for j in (0, 5, 31):
                want = ((h * A[j]) & M64) >> (64 - L)
                assert oracle.classic_position(h, m, j) == want


def test_classic_position_range_and_extremes():
    A = brute.salts64()
    for m in (64, 192, 640, 10_000 * 64, (1 << 40) + 64):
        for h in list(_keys(100, m % 97)) + [0, M64]:
            for j in range(0, 32, 7):
                p = oracle.classic_position(int(h), m, j)
                assert 0 <= p < m
                prod = (int(h) * A[j]) & M64
                # fastrange: p = floor(prod * m / 2^64), so p/m <= prod/2^64 < (p+1)/m
                assert p * 2**64 <= prod * m < (p + 1) * 2**64
    assert oracle.classic_position(0, 640, 3) == 0


def test_classic_params():
    assert not oracle.check_classic_params(0, 8)
    assert not oracle.check_classic_params(100, 8)      # not a multiple of 64
    assert not oracle.check_classic_params(64, 0)
    assert not oracle.check_classic_params(64, 33)
    assert oracle.check_classic_params(64, 1) and oracle.check_classic_params(1 << 33, 32)
    with pytest.raises(ValueError):
        oracle.ClassicOracle(96, 4)


def test_classic_bits_equal_brute_force():
    rng = _rng(7)
    for m in (64, 128, 640, 4096, 1 << 16):
        for k in (1, 3, 8, 16, 32):
            n = int(rng.integers(0, 150))
            seed = int(rng.integers(0, 2**64, dtype=np.uint64))
            keys = rng.integers(0, 2**64, size=n, dtype=np.uint64)
            f = oracle.ClassicOracle(m, k, seed)
            f.add(keys)
            bits = brute.classic_build(keys, m, k, seed)
            assert brute.positions_of_bytes(f.bytes) == bits
            queries = np.concatenate([keys, rng.integers(0, 2**64, size=200, dtype=np.uint64)])
            want = [int(brute.classic_positions(int(q), m, k, seed) <= bits) for q in queries]
            assert f.contains(queries).tolist() == want


def test_classic_one_key_sets_at_most_k_bits():
    for k in (1, 4, 8, 16):
        for key in _keys(30, k):
            f = oracle.ClassicOracle(1 << 12, k, 3)
            f.add([key])
            pop = int(np.unpackbits(f.bytes).sum())
            assert 1 <= pop <= k
            assert pop == len(brute.classic_positions(int(key), 1 << 12, k, 3))


@settings(max_examples=40, deadline=None)
@given(
    words=st.integers(1, 200),
    k=st.integers(1, 32),
    seed=st.integers(0, M64),
    a=st.lists(st.integers(0, M64), max_size=80),
    c=st.lists(st.integers(0, M64), max_size=80),
)
def test_classic_invariants(words, k, seed, a, c):
    m = 64 * words
    ka, kc = np.array(a, dtype=np.uint64), np.array(c, dtype=np.uint64)
    f = oracle.ClassicOracle(m, k, seed)
    f.add(ka)
    f.add(kc)
    assert np.all(f.contains(np.concatenate([ka, kc])) == 1)    # no false negatives
    g = oracle.ClassicOracle(m, k, seed)
    g.add(np.concatenate([kc, ka])[::-1])                       # any order
    assert np.array_equal(f.bytes, g.bytes)
    fa = oracle.ClassicOracle(m, k, seed)
    fa.add(ka)
    assert np.array_equal(f.bytes & fa.bytes, fa.bytes)          # monotone union


def test_classic_words_match_full_filter():
    m, k, seed = 64 * 5000, 8, 77
    keys = _keys(20_000, 3)
    f = oracle.ClassicOracle(m, k, seed)
    f.add(keys)
    sel = np.array([0, 1, 17, 2500, 4999, 333], dtype=np.uint64)
    full = f.bytes.view("<u8")
    got = oracle.classic_words(m, k, seed, keys, sel)
    assert np.array_equal(got, full[sel.astype(np.int64)])
    with pytest.raises(ValueError):
        oracle.classic_words(m, k, seed, keys, [5000])
    with pytest.raises(ValueError):
        oracle.classic_words(m, k, seed, keys, [3, 3])


CLASSIC_FPR_CASES = [
    # (m, k, c): n = m / c distinct keys
    (1 << 18, 4, 8),
    (1 << 18, 8, 8),
    (1 << 20, 8, 16),
    (1 << 16, 2, 4),
]


@pytest.mark.parametrize("m,k,c", CLASSIC_FPR_CASES)
def test_classic_fpr_matches_closed_form(m, k, c):
    n = m // c
    p = fpr_model.classic_fpr(n, m, k)
    R = 6
    queries = max(200_000, int(math.ceil(2e4 / (R * p))))
    rates = []
    for r in range(R):
        rng = _rng(3000 + r)
        f = oracle.ClassicOracle(m, k, int(rng.integers(0, 2**64, dtype=np.uint64)))
        f.add(rng.integers(0, 2**64, size=n, dtype=np.uint64))
        rates.append(float(f.contains(rng.integers(0, 2**64, size=queries,
                                                   dtype=np.uint64)).mean()))
    rates = np.array(rates)
    se = rates.std(ddof=1) / math.sqrt(R)
    assert abs(rates.mean() - p) <= 4 * se + 0.01 * p, (rates.mean(), p, se)


@pytest.mark.parametrize("m,k,c", CLASSIC_FPR_CASES)
def test_classic_fill_fraction_matches_closed_form(m, k, c):
    n = m // c
    want = fpr_model.classic_fill_fraction(n, m, k)
    got = []
    for r in range(4):
        rng = _rng(4000 + r)
        f = oracle.ClassicOracle(m, k, int(rng.integers(0, 2**63)))
        f.add(rng.integers(0, 2**64, size=n, dtype=np.uint64))
        got.append(np.unpackbits(f.bytes).mean())
    tol = 5 * math.sqrt(want * (1 - want) / (4 * m)) + 0.002 * want
    assert abs(np.mean(got) - want) <= tol, (np.mean(got), want)


def test_classic_model_pins():
    """The exact model tends to Eq. (1) as m grows at fixed c, k; its cover
    probability equals the Markov-chain and exact-rational forms."""
    for d, m, M in ((1, 64, 1), (4, 64, 50), (8, 640, 700)):
        want = fpr_model.cover_prob_inclusion_exclusion(d, m, M)
        assert math.isclose(fpr_model.cover_prob_float(d, m, M), want, rel_tol=1e-9)
        assert math.isclose(fpr_model.cover_probs(d, m, M)[M], want, rel_tol=1e-9)
    for c, k in ((8, 4), (16, 8), (32, 8), (16, 11)):
        m = 1 << 26
        exact = fpr_model.classic_fpr(m // c, m, k)
        assert math.isclose(exact, fpr_model.cbf_fpr_eq1(c, k), rel_tol=2e-3), (c, k)
    # one key, k = 1: the query collides iff it draws the same position
    assert math.isclose(fpr_model.classic_fpr(1, 640, 1), 1 / 640, rel_tol=1e-12)


# --------------------------------------------------------------------------
# Cache-sectorized filter
# --------------------------------------------------------------------------

def test_group_salts_derivation():
    got = oracle.group_salts()
    assert got == brute.group_salts()
    assert all(v & 1 for v in got) and len(set(got)) == 16
    assert not set(got) & set(oracle.salts())


def test_csbf_params():
    ok = oracle.check_csbf_params
    assert ok(10, 8, 32, 2, 4) and ok(10, 16, 64, 16, 16) and ok(1, 1, 32, 1, 1)
    assert not ok(10, 8, 32, 16, 16)        # z > s
    assert not ok(10, 8, 32, 3, 6)          # z not a power of two
    assert not ok(10, 8, 32, 4, 6)          # k not a multiple of z
    assert not ok(10, 8, 32, 4, 2)          # k < z
    assert not ok(10, 8, 32, 2, 34)         # k > 32
    assert not ok(0, 8, 32, 2, 4) and not ok((1 << 32) + 1, 8, 32, 2, 4)
    assert not ok(10, 8, 16, 2, 4) and not ok(10, 3, 32, 1, 4)
    with pytest.raises(ValueError):
        oracle.CsbfOracle(10, 8, 32, 4, 6)


@pytest.mark.parametrize("s,S", [(s, S) for S in (32, 64) for s in (1, 2, 4, 8, 16)])
def test_csbf_with_one_word_per_group_is_the_sectorized_filter(s, S):
    """z = s: each group is one word, so the layout is the sectorized one."""
    rng = _rng(50 + s + S)
    for k in sorted({s, 2 * s, 16, 32}):
        if k % s or k > 32:
            continue
        b = int(rng.integers(1, 300))
        seed = int(rng.integers(0, 2**64, dtype=np.uint64))
        keys = rng.integers(0, 2**64, size=2000, dtype=np.uint64)
        a = oracle.CsbfOracle(b, s, S, s, k, seed)
        a.add(keys)
        ref = oracle.OracleFilter(b, s, S, k, seed)
        ref.add(keys)
        assert np.array_equal(a.bytes, ref.bytes)
        q = np.concatenate([keys[:500], rng.integers(0, 2**64, size=3000, dtype=np.uint64)])
        assert np.array_equal(a.contains(q), ref.contains(q))


@pytest.mark.parametrize("s,S,z", CSBF_LAYOUTS)
def test_csbf_bits_equal_brute_force(s, S, z):
    rng = _rng(200 + 7 * s + S + z)
    for b in (1, 2, 3, 17):
        for k in sorted({z, 2 * z, 4 * z, 8, 16}):
            if k % z or k > 32:
                continue
            n = int(rng.integers(0, 150))
            seed = int(rng.integers(0, 2**64, dtype=np.uint64))
            keys = rng.integers(0, 2**64, size=n, dtype=np.uint64)
            f = oracle.CsbfOracle(b, s, S, z, k, seed)
            f.add(keys)
            bits = brute.csbf_build(keys, b, s, S, z, k, seed)
            assert brute.triples_of_bytes(f.bytes, s, S) == bits
            queries = np.concatenate([keys, rng.integers(0, 2**64, size=200, dtype=np.uint64)])
            want = [int(brute.csbf_triples_of_key(int(q), b, s, S, z, k, seed) <= bits)
                    for q in queries]
            assert f.contains(queries).tolist() == want


@pytest.mark.parametrize("s,S,z", CSBF_LAYOUTS)
def test_csbf_one_key_touches_one_word_per_group(s, S, z):
    """A single key sets bits in exactly one word of each group of its block
    (the word of group g lies in words g*s/z .. (g+1)*s/z - 1), at most k/z
    bits per word."""
    k = max(z, 8 - 8 % z) if z <= 8 else 16
    b = 5
    for key in _keys(40, s * S + z):
        f = oracle.CsbfOracle(b, s, S, z, k, 11)
        f.add([key])
        words = f.words().reshape(b, s)
        nz_blocks = np.nonzero(words.any(axis=1))[0]
        assert nz_blocks.size == 1
        row = words[nz_blocks[0]]
        width = s // z
        for g in range(z):
            grp = row[g * width:(g + 1) * width]
            assert np.count_nonzero(grp) == 1
            pop = bin(int(grp[np.nonzero(grp)[0][0]])).count("1")
            assert 1 <= pop <= k // z


@settings(max_examples=40, deadline=None)
@given(
    layout=st.sampled_from(CSBF_LAYOUTS),
    b=st.integers(1, 300),
    mult=st.integers(1, 4),
    seed=st.integers(0, M64),
    keys=st.lists(st.integers(0, M64), max_size=120),
)
def test_csbf_no_false_negatives_and_order_independence(layout, b, mult, seed, keys):
    s, S, z = layout
    k = min(32, z * mult)
    keys = np.array(keys, dtype=np.uint64)
    f = oracle.CsbfOracle(b, s, S, z, k, seed)
    f.add(keys)
    assert np.all(f.contains(keys) == 1)
    g = oracle.CsbfOracle(b, s, S, z, k, seed)
    g.add(keys[::-1])
    g.add(keys[: len(keys) // 2])
    assert np.array_equal(f.bytes, g.bytes)


def test_csbf_block_words_match_full_filter():
    b, s, S, z, k, seed = 3000, 8, 32, 2, 4, 5
    keys = _keys(30_000, 4)
    f = oracle.CsbfOracle(b, s, S, z, k, seed)
    f.add(keys)
    sel = np.array([0, 2999, 1500, 7, 8], dtype=np.uint64)
    got = oracle.csbf_block_words(b, s, S, z, k, seed, keys, sel)
    full = f.bytes.reshape(b, s * S // 8)
    assert np.array_equal(got, full[sel.astype(np.int64)])
    with pytest.raises(ValueError):
        oracle.csbf_block_words(b, s, S, z, k, seed, keys, [3000])


CSBF_FPR_CASES = [
    # (s, S, z, k, b, n)
    (8, 32, 2, 4, 1024, 24000),
    (8, 32, 1, 4, 1024, 16000),
    (8, 32, 4, 8, 1024, 24000),
    (16, 64, 2, 8, 256, 16000),
    (16, 64, 4, 8, 256, 16000),
    (4, 64, 2, 6, 512, 8000),
]


@pytest.mark.parametrize("s,S,z,k,b,n", CSBF_FPR_CASES)
def test_csbf_fpr_matches_closed_form(s, S, z, k, b, n):
    p = fpr_model.csbf_fpr(n, b, s, S, z, k)
    R = 8
    queries = max(200_000, int(math.ceil(2e4 / (R * p))))
    rates = []
    for r in range(R):
        rng = _rng(5000 + r)
        f = oracle.CsbfOracle(b, s, S, z, k, int(rng.integers(0, 2**64, dtype=np.uint64)))
        f.add(rng.integers(0, 2**64, size=n, dtype=np.uint64))
        rates.append(float(f.contains(rng.integers(0, 2**64, size=queries,
                                                   dtype=np.uint64)).mean()))
    rates = np.array(rates)
    assert rates.sum() * queries >= 1e4
    se = rates.std(ddof=1) / math.sqrt(R)
    assert abs(rates.mean() - p) <= 4 * se + 0.01 * p, (rates.mean(), p, se)


@pytest.mark.parametrize("s,S,z,k,b,n", CSBF_FPR_CASES)
def test_csbf_fill_fraction_matches_closed_form(s, S, z, k, b, n):
    want = fpr_model.csbf_fill_fraction(n, b, s, S, z, k)
    got = []
    for r in range(4):
        rng = _rng(6000 + r)
        f = oracle.CsbfOracle(b, s, S, z, k, int(rng.integers(0, 2**63)))
        f.add(rng.integers(0, 2**64, size=n, dtype=np.uint64))
        got.append(np.unpackbits(f.bytes).mean())
    total_bits = b * s * S
    tol = 5 * math.sqrt(want * (1 - want) / (4 * total_bits)) + 0.002 * want
    assert abs(np.mean(got) - want) <= tol, (np.mean(got), want)


def test_csbf_model_pins():
    """With z = s the model is the sectorized model; below a few groups,
    fewer groups (more bits in fewer words) raise the rate; one key, one
    group of four words, k = 1: collision iff same block, word and bit."""
    for s, S, k, b, n in ((8, 32, 8, 1024, 24000), (16, 64, 16, 128, 10000), (4, 32, 8, 500, 4000)):
        assert math.isclose(fpr_model.csbf_fpr(n, b, s, S, s, k),
                            fpr_model.sbf_fpr(n, b, s, S, k), rel_tol=1e-9)
    rates = [fpr_model.csbf_fpr(16000, 256, 16, 64, z, 16) for z in (4, 2, 1)]
    assert all(x < y for x, y in zip(rates, rates[1:]))
    # one key, s = 4 words in one group, k = 1: same block (1/b), same word (1/4),
    # same bit (1/S)
    assert math.isclose(fpr_model.csbf_fpr(1, 10, 4, 32, 1, 1), 1 / 10 / 4 / 32, rel_tol=1e-12)


# --------------------------------------------------------------------------
# Chained pattern hashing (the prior-art rule of Sec. IV-B)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("s,S", [(1, 32), (4, 64), (8, 32), (16, 64)])
def test_chained_bits_equal_brute_force(s, S):
    rng = _rng(400 + s + S)
    for b in (1, 3, 17):
        for k in sorted({s, 2 * s, 16}):
            if k < s or k > 32:
                continue
            n = int(rng.integers(0, 120))
            seed = int(rng.integers(0, 2**64, dtype=np.uint64))
            keys = rng.integers(0, 2**64, size=n, dtype=np.uint64)
            f = oracle.ChainedOracle(b, s, S, k, seed)
            f.add(keys)
            bits = brute.chained_build(keys, b, s, S, k, seed)
            assert brute.triples_of_bytes(f.bytes, s, S) == bits
            queries = np.concatenate([keys, rng.integers(0, 2**64, size=200, dtype=np.uint64)])
            want = [int(brute.chained_triples_of_key(int(q), b, s, S, k, seed) <= bits)
                    for q in queries]
            assert f.contains(queries).tolist() == want


def test_chained_block_rule_is_the_sectorized_one():
    """Only the pattern differs: a one-key chained filter sets bits in the
    same block as the sectorized filter, and its bits differ from it."""
    for key in _keys(50, 9):
        a = oracle.ChainedOracle(97, 4, 32, 8, 5)
        a.add([key])
        b = oracle.OracleFilter(97, 4, 32, 8, 5)
        b.add([key])
        ba = np.nonzero(a.bytes.reshape(97, 16).any(axis=1))[0]
        bb = np.nonzero(b.bytes.reshape(97, 16).any(axis=1))[0]
        assert ba.tolist() == bb.tolist()
    assert not np.array_equal(a.bytes, b.bytes)


@pytest.mark.parametrize("s,S,k,b,n", [(4, 64, 16, 512, 12000), (8, 32, 8, 1024, 24000)])
def test_chained_fpr_matches_closed_form(s, S, k, b, n):
    """Positions from independent full hashes are uniform: the sectorized
    closed form applies unchanged."""
    p = fpr_model.sbf_fpr(n, b, s, S, k)
    R = 6
    queries = max(200_000, int(math.ceil(2e4 / (R * p))))
    rates = []
    for r in range(R):
        rng = _rng(7000 + r)
        f = oracle.ChainedOracle(b, s, S, k, int(rng.integers(0, 2**64, dtype=np.uint64)))
        f.add(rng.integers(0, 2**64, size=n, dtype=np.uint64))
        rates.append(float(f.contains(rng.integers(0, 2**64, size=queries,
                                                   dtype=np.uint64)).mean()))
    rates = np.array(rates)
    se = rates.std(ddof=1) / math.sqrt(R)
    assert abs(rates.mean() - p) <= 4 * se + 0.01 * p, (rates.mean(), p, se)
