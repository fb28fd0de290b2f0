"""Rice parameters for the Golomb-Rice seed codes (Section 4: a seed costs
0.44n + o(n) bits in expectation with Golomb-Rice codes).

A seed of a leaf is the first success of independent trials with success
probability p per seed, i.e. geometric: P(v) = (1 - p)^v p.  The Rice code
with parameter k spends k bits on v mod 2^k and q + 1 bits on q = v >> k in
unary, so with t = (1 - p)^(2^k) its expected length is

    k + 1 + t / (1 - t)

(P(q >= m) = t^m).  The codec in the library takes one parameter per leaf
size; this module picks the k minimising that expectation, for the plain
search's exact per-seed success probability (ideal loop-free hashing, the
exponential formula over unicyclic components) or for measured mean seeds.
Configuration only: nothing here runs on the search path.
"""
from __future__ import annotations

import functools
import math
from fractions import Fraction

MAX_K = 56


def expected_length(k: int, p: float) -> float:
    """Mean Rice code length in bits of a geometric value with success probability p."""
    if p >= 1.0:
        return k + 1.0
    t = math.exp((2 ** k) * math.log1p(-p))
    return k + 1.0 + t / (1.0 - t)


def optimal_k(p: float) -> int:
    """The Rice parameter with the smallest expected length (ties: the smaller k)."""
    best_k, best = 0, expected_length(0, p)
    for k in range(1, MAX_K + 1):
        e = expected_length(k, p)
        if e < best - 1e-12:
            best_k, best = k, e
    return best_k


def geometric_entropy(p: float) -> float:
    """Entropy in bits of the geometric distribution with success probability p."""
    if p >= 1.0:
        return 0.0
    q = 1.0 - p
    return (-q * math.log2(q) - p * math.log2(p)) / p


def _unicyclic_weight(k: int) -> Fraction:
    """Connected graphs on k cells with k keys, each key an ordered pair of
    distinct cells, divided by k! (keys) and k! (cells): connected functional
    graphs without fixed points, times 2^(k-1) orderings per key pair."""
    functional = sum(Fraction(math.factorial(k), math.factorial(k - j)) * Fraction(k) ** (k - j - 1)
                     for j in range(1, k + 1))
    return (functional - Fraction(k) ** (k - 1)) * 2 ** (k - 1) / math.factorial(k)


@functools.lru_cache(maxsize=1)
def _pseudoforest_series(n_max: int = 64) -> tuple:
    """Coefficients of exp(sum_k w_k z^k) up to z^n_max (the exponential
    formula); they do not depend on the leaf size."""
    w = [Fraction(0)] + [_unicyclic_weight(k) for k in range(1, n_max + 1)]
    series = [Fraction(1)] + [Fraction(0)] * n_max
    for m in range(1, n_max + 1):
        series[m] = sum(k * w[k] * series[m - k] for k in range(1, m + 1)) / m
    return tuple(series)


@functools.lru_cache(maxsize=None)
def success_probability(n: int) -> float:
    """Probability that one seed of an n-key leaf qualifies under ideal
    loop-free hashing: a graph of n keys on n cells is a pseudoforest iff every
    component has as many keys as cells (each unicyclic), counted by the
    exponential formula over such components."""
    if n <= 1:
        return 1.0
    series = _pseudoforest_series(max(64, n))
    return float(Fraction(math.factorial(n)) ** 2 * series[n] / Fraction(n * (n - 1)) ** n)


def plain_table() -> list[int]:
    """k per leaf size 0..64 for the plain search's seeds (start seed 0)."""
    return list(_plain_table())


@functools.lru_cache(maxsize=1)
def _plain_table() -> tuple:
    return tuple(0 if n <= 1 else optimal_k(success_probability(n)) for n in range(65))


def table_from_means(mean_by_n) -> list[int]:
    """k per leaf size from mean values (a mapping or a 65-entry sequence;
    missing sizes get k = 0), taking p = 1 / (mean + 1)."""
    get = mean_by_n.get if hasattr(mean_by_n, "get") else (lambda n, d=None: mean_by_n[n])
    out = []
    for n in range(65):
        m = get(n, None)
        out.append(0 if m is None or m <= 0 else optimal_k(1.0 / (float(m) + 1.0)))
    return out
