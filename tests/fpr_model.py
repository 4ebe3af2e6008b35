"""Closed-form false-positive rate and fill fraction of a sectorized filter.

The paper gives the classic-filter rate, Eq. (1): f(c, k) ~ (1 - e^{-k/c})^k,
and states that under uniform block choice each block of a blocked filter
behaves like a small classic filter holding about n/b keys (Sec. II-A-2).
Written out exactly for the sectorized layout (Sec. II-A-4), under the model
that every pattern bit is an independent uniform position in its word:

* the load l of the query's block is Binomial(n, 1/b);
* word w receives t_w = floor(k/s) + [w < k mod s] bits per key, so l keys
  throw M = l * t_w uniform positions into its S bits;
* the query's own t_w positions are d distinct ones with probability
  S2(t_w, d) * S!/(S-d)! / S^t_w;
* d given positions are all covered by M throws with probability
  sum_i (-1)^i C(d, i) (1 - i/S)^M  (inclusion-exclusion), computed here by an
  equivalent, cancellation-free Markov chain over the number covered;
* words are independent given l, so FPR = sum_l P(l) prod_w q_w(l).

The same model covers the classic filter of Sec. II-A-1 (one "word" of m
bits, n*k throws; ``classic_fpr``) and the cache-sectorized filter of
Sec. II-A-5 (``csbf_fpr``): within the query's block, each of the z groups
has one selected word, whose load is Binomial(l, z/s) keys of k/z bits each,
and the groups are independent given l.

Everything is float64.  This is a model, not an implementation: it pins the
oracle statistically, independent of how the oracle computes bits.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy.stats import binom


def bits_per_word(s: int, k: int) -> list[int]:
    return [k // s + (1 if w < k % s else 0) for w in range(s)]


@lru_cache(maxsize=None)
def _stirling2(t: int, d: int) -> int:
    if t == d:
        return 1
    if d == 0 or d > t:
        return 0
    return d * _stirling2(t - 1, d) + _stirling2(t - 1, d - 1)


def distinct_probs(t: int, S: int) -> list[float]:
    """P(t uniform throws into S bins occupy exactly d bins), d = 0..t."""
    out = []
    for d in range(t + 1):
        falling = math.perm(S, d) if d <= S else 0
        out.append(_stirling2(t, d) * falling / float(S) ** t)
    return out


def cover_probs(d: int, S: int, max_throws: int) -> np.ndarray:
    """cover[M] = P(d given bins are all hit by M uniform throws into S bins)."""
    state = np.zeros(d + 1)
    state[0] = 1.0
    cover = np.empty(max_throws + 1)
    cover[0] = state[d]
    c = np.arange(d + 1)
    p_new = (d - c) / S          # a throw hits a not yet covered given bin
    for m in range(1, max_throws + 1):
        moved = state * p_new
        state = state - moved
        state[1:] += moved[:-1]
        cover[m] = state[d]
    return cover


def cover_prob_inclusion_exclusion(d: int, S: int, M: int) -> float:
    """The same probability by inclusion-exclusion (exact rationals)."""
    from fractions import Fraction

    total = Fraction(0)
    for i in range(d + 1):
        total += (-1) ** i * math.comb(d, i) * Fraction(S - i, S) ** M
    return float(total)


def _load_pmf(n: int, b: int):
    mean = n / b
    lmax = int(mean + 14 * math.sqrt(mean + 1) + 40)
    lmax = min(lmax, n)
    ls = np.arange(lmax + 1)
    return ls, binom.pmf(ls, n, 1.0 / b)


def sbf_fpr(n: int, b: int, s: int, S: int, k: int) -> float:
    """Expected false-positive rate after n distinct keys (model above)."""
    ls, pl = _load_pmf(n, b)
    lmax = int(ls[-1])
    per_l = np.ones(ls.size)
    for t in sorted(set(bits_per_word(s, k))):
        count = bits_per_word(s, k).count(t)
        dp = distinct_probs(t, S)
        q = np.zeros(ls.size)
        for d in range(1, t + 1):
            if dp[d] == 0.0:
                continue
            cov = cover_probs(d, S, lmax * t)
            q += dp[d] * cov[ls * t]
        per_l *= q ** count
    return float(np.sum(pl * per_l))


def sbf_fill_fraction(n: int, b: int, s: int, S: int, k: int) -> float:
    """Expected fraction of set bits after n keys."""
    ls, pl = _load_pmf(n, b)
    acc = np.zeros(ls.size)
    for t in bits_per_word(s, k):
        acc += 1.0 - (1.0 - 1.0 / S) ** (ls * t)
    return float(np.sum(pl * acc / s))


def cbf_fpr_eq1(c: float, k: int) -> float:
    """Eq. (1) of the paper: classic filter, c bits per key."""
    return (1.0 - math.exp(-k / c)) ** k


def cover_prob_float(d: int, m: int, M: int) -> float:
    """P(d given bins of m are all hit by M uniform throws), inclusion-exclusion
    in float64 (fine for the moderate cancellation of the cases used here)."""
    total = 0.0
    for i in range(d + 1):
        total += (-1) ** i * math.comb(d, i) * math.exp(M * math.log1p(-i / m))
    return total


def classic_fpr(n: int, m: int, k: int) -> float:
    """Classic filter of m bits after n distinct keys, k uniform positions each."""
    dp = distinct_probs(k, m)
    return float(sum(dp[d] * cover_prob_float(d, m, n * k) for d in range(1, k + 1)))


def classic_fill_fraction(n: int, m: int, k: int) -> float:
    return 1.0 - math.exp(n * k * math.log1p(-1.0 / m))


def csbf_fpr(n: int, b: int, s: int, S: int, z: int, k: int) -> float:
    """Cache-sectorized filter: z groups of s/z words, k/z bits per selected word."""
    assert k % z == 0 and s % z == 0
    t, width = k // z, s // z
    ls, pl = _load_pmf(n, b)
    lmax = int(ls[-1])
    dp = distinct_probs(t, S)
    q = np.zeros(lmax + 1)                    # q[l] for l keys in the query's word
    for d in range(1, t + 1):
        if dp[d] == 0.0:
            continue
        q += dp[d] * cover_probs(d, S, lmax * t)[np.arange(lmax + 1) * t]
    per_l = np.empty(ls.size)
    for i, L in enumerate(ls):
        w = binom.pmf(np.arange(L + 1), L, 1.0 / width)
        per_l[i] = float(np.dot(w, q[: L + 1])) ** z
    return float(np.sum(pl * per_l))


def csbf_fill_fraction(n: int, b: int, s: int, S: int, z: int, k: int) -> float:
    t, width = k // z, s // z
    ls, pl = _load_pmf(n, b)
    hit = (1.0 - (1.0 - 1.0 / S) ** t) / width   # one key sets a given bit of a word
    return float(np.sum(pl * (1.0 - (1.0 - hit) ** ls)))
