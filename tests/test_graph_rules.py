"""The two graph facts the GPU pair and candidate tests rely on, checked
against the oracle's pseudoforest predicate (components counted by a depth-
first search).  No GPU.

1. Counting exit of the peeling test.  With n edges on n cells, remove per
   round every edge at a cell of degree one.  Over the cells that still have
   an edge, (edges left) - (cells left) stays zero exactly for a pseudoforest
   (Section 2: no component with more edges than nodes); otherwise it turns
   positive in some round.  So "reject when the two counts differ, accept
   when no cell of degree one is left" decides the predicate.
2. Lone-key filter of the bipartite search.  If some key is the only key in
   both of its cells, its edge is a one-edge tree; with n edges on n cells
   another component then has more edges than nodes, so the graph is not a
   pseudoforest.

The rules are written out here from their statements (the kernels' code is
not imported).
"""
import itertools

import numpy as np
import pytest

from workloads import splitmix64


def counting_peel(n, h0, h1):
    """Decision and rounds of the counting-exit peeling rule (model)."""
    inc = [0] * n
    for k in range(n):
        inc[h0[k]] |= 1 << k
        inc[h1[k]] |= 1 << k
    rem = (1 << n) - 1
    for rnd in range(n + 2):
        deg = [bin(inc[c] & rem).count("1") for c in range(n)]
        if bin(rem).count("1") != sum(1 for d in deg if d):
            return False, rnd
        d1 = [c for c in range(n) if deg[c] == 1]
        if not d1:
            return True, rnd
        ones = set(d1)
        for k in range(n):
            if (rem >> k) & 1 and (h0[k] in ones or h1[k] in ones):
                rem &= ~(1 << k)
    raise AssertionError("a round that goes on removes an edge")


def lone_in_both(h0, h1):
    cnt = {}
    for c in list(h0) + list(h1):
        cnt[c] = cnt.get(c, 0) + 1
    return any(cnt[a] == 1 and cnt[b] == 1 for a, b in zip(h0, h1))


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_counting_peel_exhaustive(oracle_mod, n):
    """Every graph of n edges on n cells (loops included) for n <= 4."""
    pairs = list(itertools.product(range(n), repeat=2))
    seen = [0, 0]
    for edges in itertools.product(pairs, repeat=n):
        h0 = [e[0] for e in edges]
        h1 = [e[1] for e in edges]
        want = oracle_mod.is_pseudoforest(n, h0, h1)
        got, _ = counting_peel(n, h0, h1)
        assert got == want, (h0, h1)
        seen[want] += 1
    assert seen[1] > 0 and (seen[0] > 0 or n == 1)


def random_graphs(rng, n, count, covering):
    """`count` loop-free graphs of n edges on n cells, each edge a uniform
    ordered pair of distinct cells; with `covering`, only graphs that cover
    every cell (rejection sampling in batches)."""
    out = []
    while len(out) < count:
        m = 20000
        h0 = rng.integers(0, n, (m, n))
        r = rng.integers(0, n - 1, (m, n))
        h1 = r + (r >= h0)
        if covering:
            hit = np.zeros((m, n), bool)
            np.put_along_axis(hit, h0, True, 1)
            np.put_along_axis(hit, h1, True, 1)
            keep = hit.all(1)
            h0, h1 = h0[keep], h1[keep]
        out += [(list(a), list(b)) for a, b in zip(h0, h1)][: count - len(out)]
    return out


@pytest.mark.parametrize("n", [5, 8, 16, 24, 32, 48, 64])
def test_counting_peel_random(oracle_mod, n):
    """Random loop-free graphs, uniform and covering every cell (the
    candidates the searches send), against the oracle."""
    rng = np.random.default_rng(7000 + n)
    count = 60 if n == 64 else 150
    seen = [0, 0]
    for covering in (False, True):
        for h0, h1 in random_graphs(rng, n, count, covering):
            want = oracle_mod.is_pseudoforest(n, h0, h1)
            got, _ = counting_peel(n, h0, h1)
            assert got == want
            seen[want] += 1
    assert seen[0] > 0


def test_counting_peel_exits_early_on_covering_graphs():
    """On graphs that cover every cell, nearly every rejection comes in the
    first round (a small tree is peeled away at once)."""
    rng = np.random.default_rng(7100)
    rounds = [rnd for ok, rnd in (counting_peel(48, h0, h1) for h0, h1 in random_graphs(rng, 48, 200, True))
              if not ok]
    assert len(rounds) > 150 and np.mean(rounds) < 1.5 and np.median(rounds) == 1


def test_lone_key_pairs_are_never_pseudoforests(oracle_mod):
    """Bipartite pairs under the oracle's cells: every pair with a key alone
    in both of its cells fails the oracle's predicate, and among pairs of
    covering candidates most pairs have such a key."""
    n = 48
    nl = n // 2
    keys = [int(x) for x in splitmix64(7200, n)]
    left, right = {}, {}
    for s in range(6000):
        cells = [oracle_mod.bip_slots(x, s, n) for x in keys]
        lc, rc = [c[0] for c in cells], [c[1] for c in cells]
        if len(set(lc)) == nl and len(left) < 40:
            left[s] = lc
        if len(set(rc)) == n - nl and len(right) < 40:
            right[s] = rc
    assert len(left) >= 10 and len(right) >= 10
    lone = 0
    total = 0
    for a, lc in left.items():
        for b, rc in right.items():
            total += 1
            if lone_in_both(lc, rc):
                lone += 1
                assert not oracle_mod.is_pseudoforest(n, lc, rc), (a, b)
    assert lone > 0.6 * total
