"""Exact probabilities for ideal (fully random) hashing -- test infrastructure.

These closed forms are pinned against exhaustive enumeration for tiny n in
test_theory_pins.py and then used as the target of the statistical tests of
the oracle's hash and search.

Model "loop-free": every key draws an ordered pair (h0, h1) of DISTINCT cells
uniformly from [n]; model "self-loop": (h0, h1) uniform from [n]^2, the model
analysed in Section 5.
"""
from fractions import Fraction
from math import comb, e, factorial, pi, sqrt


def connected_functional_graphs(k: int) -> int:
    """Number of connected functional graphs on k labelled nodes:
    sum_{j=1..k} k!/(k-j)! * k^(k-j-1)  (a cycle of length j with rooted trees hanging off it)."""
    total = Fraction(0)
    for j in range(1, k + 1):
        total += Fraction(factorial(k), factorial(k - j)) * Fraction(k) ** (k - j - 1)
    assert total.denominator == 1
    return int(total)


def _exp_series(a, n):
    out = [Fraction(0)] * (n + 1)
    out[0] = Fraction(1)
    for m in range(1, n + 1):
        out[m] = sum(k * a[k] * out[m - k] for k in range(1, m + 1)) / m
    return out


def p_accept(n: int, loops: bool = False) -> Fraction:
    """Probability that n random edges on n nodes form a pseudoforest.

    Each component of a maximal pseudoforest is unicyclic; a connected
    unicyclic component on k nodes with k labelled keys and ordered endpoint
    pairs is counted by c_k * k! * 2^k / 2 (c_k connected functional graphs,
    each undirected component arising from two cycle directions), minus the
    self-loop cycles k^(k-1) when loops are forbidden.  The exponential
    formula over node- and key-labelled components gives the count of
    pseudoforests, divided by the number of configurations."""
    a = [Fraction(0)]
    for k in range(1, n + 1):
        ck = connected_functional_graphs(k)
        if loops:
            # self-loops: a loop on a node is one functional-graph cycle but
            # only one orientation of the pair (h0, h1) -- count per key 2^k / 2
            # for cycles of length >= 2 and 2^k / 2 for loops as well, as both
            # slots of a loop key are the same cell.
            a.append(Fraction(ck * 2 ** (k - 1), factorial(k)))
        else:
            a.append(Fraction((ck - k ** (k - 1)) * 2 ** (k - 1), factorial(k)))
    coeff = _exp_series(a, n)[n]
    denom = (n * n) ** n if loops else (n * (n - 1)) ** n
    return Fraction(factorial(n)) ** 2 * coeff / denom


def q_cover(n: int, loops: bool = False) -> Fraction:
    """Probability that the 2n slots of n keys cover all n cells (inclusion-exclusion)."""
    if loops:
        return sum((-1) ** j * comb(n, j) * Fraction(n - j, n) ** (2 * n) for j in range(n + 1))
    return sum((-1) ** j * comb(n, j) * Fraction((n - j) * (n - j - 1), n * (n - 1)) ** n for j in range(n + 1))


def bijection_probability(n: int) -> Fraction:
    """A random function [n] -> [n] is a bijection with probability n!/n^n (Lemma lem:bruteForce)."""
    return Fraction(factorial(n), n ** n)


def construction_lower_bound(n: int) -> float:
    """Theorem lem:constructionTries: P(exists f) >= (e/2)^(-n) e^(-1) sqrt(pi)."""
    return (e / 2) ** (-n) / e * sqrt(pi)


def expected_tries_bound(n: int) -> float:
    """Theorem thm:shockHashConstruction: expected seeds to try <= (e/2)^n e / sqrt(pi)."""
    return (e / 2) ** n * e / sqrt(pi)


def pseudotree_lower_bound(n: int) -> float:
    """Theorem lem:simpleProof: P(pseudotree) >= (e/2)^(-n) sqrt(pi / (2n))."""
    return (e / 2) ** (-n) * sqrt(pi / (2 * n))


def brute_force_tries(n: int) -> float:
    """Expected brute-force trials e^n / sqrt(2 pi n) (Section 5 after Theorem thm:shockHashConstruction)."""
    return e ** n / sqrt(2 * pi * n)


def filter_lambda() -> float:
    """Root of 2 = lambda / (1 - e^-lambda) (Appendix B), by bisection."""
    lo, hi = 1.0, 2.0
    for _ in range(200):
        mid = (lo + hi) / 2
        if mid / (1 - e ** (-mid)) < 2:
            lo = mid
        else:
            hi = mid
    return (lo + hi) / 2


def filter_base() -> float:
    """b = 2 e^lambda / (lambda e^2) (Appendix B): the filter passes with probability Theta(b^n)."""
    lam = filter_lambda()
    return 2 * e ** lam / (lam * e ** 2)
