"""Pins for the closed forms in tests/theory.py (no GPU, no oracle).

The statistical tests of the oracle compare its measured seed counts against
these formulas, so the formulas themselves are first pinned against
exhaustive enumeration and against values the paper prints.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import theory as T

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _enumerate(n, loops):
    cells = range(n)
    pairs = [(u, v) for u in cells for v in cells if loops or u != v]
    graphs = np.array(list(itertools.product(pairs, repeat=n)), dtype=np.int64)  # (G, n, 2)
    fs = np.array([[(f >> i) & 1 for i in range(n)] for f in range(1 << n)], dtype=np.int64)  # (F, n)
    chosen = np.take_along_axis(graphs[:, None, :, :], fs[None, :, :, None], axis=3)[..., 0]  # (G, F, n)
    onehot = (chosen[..., None] == np.arange(n)).sum(axis=2)  # (G, F, n)
    bij = (onehot == 1).all(axis=2)  # (G, F)
    cover = np.zeros((graphs.shape[0], n), dtype=bool)
    for c in range(n):
        cover[:, c] = (graphs == c).any(axis=(1, 2))
    return graphs, bij, cover.all(axis=1)


@pytest.mark.parametrize("n", [2, 3, 4])
@pytest.mark.parametrize("loops", [False, True])
def test_closed_forms_match_enumeration(n, loops):
    graphs, bij, covered = _enumerate(n, loops)
    total = graphs.shape[0]
    n_accept = int(bij.any(axis=1).sum())
    assert T.p_accept(n, loops) == Fraction(n_accept, total)
    assert T.q_cover(n, loops) == Fraction(int(covered.sum()), total)


def test_connected_functional_graph_counts():
    # c_k for k = 1..6 checked against a direct count of connected maps [k] -> [k].
    for k in range(1, 6):
        count = 0
        for fmap in itertools.product(range(k), repeat=k):
            parent = list(range(k))

            def find(x):
                while parent[x] != x:
                    x = parent[x]
                return x

            for i, j in enumerate(fmap):
                a, b = find(i), find(j)
                if a != b:
                    parent[a] = b
            if len({find(i) for i in range(k)}) == 1:
                count += 1
        assert T.connected_functional_graphs(k) == count


def test_bijection_probability_matches_enumeration():
    for n in (2, 3, 4, 5):
        maps = list(itertools.product(range(n), repeat=n))
        good = sum(1 for m in maps if len(set(m)) == n)
        assert T.bijection_probability(n) == Fraction(good, len(maps))


def _read_curves(name):
    curves = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            label, n, v = line.split()
            curves.setdefault(label, []).append((int(n), float(v)))
    return curves


def test_printed_theory_curves():
    """Fig. 1 (left) prints sample points of the four theory curves."""
    curves = _read_curves("fig1_theory_curves.txt")
    fns = {
        "bruteforce": T.brute_force_tries,
        "rotation_fitting": lambda n: T.brute_force_tries(n) / n,
        "shockhash": T.expected_tries_bound,
        "shockhash_rf": lambda n: T.expected_tries_bound(n) / n,
    }
    for label, pts in curves.items():
        for n, v in pts:
            assert fns[label](n) == pytest.approx(v, rel=2e-5), (label, n)


def test_bounds_hold_for_exact_probabilities():
    """Theorems lem:simpleProof and lem:constructionTries bound the self-loop
    model from below; forbidding self-loops only helps; Lemma
    lem:filterProbability bounds the filter pass rate from above."""
    for n in range(2, 65):
        p_loop = float(T.p_accept(n, loops=True))
        p_free = float(T.p_accept(n))
        assert p_loop >= T.construction_lower_bound(n)
        assert p_loop >= T.pseudotree_lower_bound(n) * (1 - 1e-12)
        assert p_free >= p_loop
        # negative association: P(all covered) <= prod_i P(cell i covered)
        q_loop = float(T.q_cover(n, loops=True))
        assert q_loop <= (1 - (1 - 1 / n) ** (2 * n)) ** n * (1 + 1e-12)
        q_free = float(T.q_cover(n))
        assert q_free <= (1 - (1 - 2 / n) ** n) ** n * (1 + 1e-12)
        assert p_free <= q_free


def test_filter_strength_base():
    """Appendix B: the filter passes with probability Theta(b^n), b ~ 0.836,
    lambda the root of 2 = lambda/(1 - e^-lambda) (the text's 1.597 is a
    rounding of 1.5936).  Successive ratios q_{n+1}/q_n approach b."""
    lam = T.filter_lambda()
    assert lam == pytest.approx(1.5936, abs=1e-4)
    b = T.filter_base()
    assert b == pytest.approx(0.836, abs=5e-4)
    q = {n: T.q_cover(n, loops=True) for n in (300, 301)}
    assert float(q[301] / q[300]) == pytest.approx(b, rel=2e-3)


def test_paper_measured_means_within_model_bracket():
    """Fig. 1 (left) prints ShockHash's measured average successful seed.
    The paper's implementation forbids self-loops but its hash family is not
    given, so the points are only checked to lie between the loop-free ideal
    and the self-loop ideal E[s*] = 1/p - 1 for 8 <= n <= 40."""
    pts = _read_curves("fig1_shockhash_measured.txt")["shockhash"]
    for n, v in pts:
        if n < 8:
            continue
        lo = float(1 / T.p_accept(n)) - 1
        hi = float(1 / T.p_accept(n, loops=True)) - 1
        assert lo < v < hi, (n, lo, v, hi)
