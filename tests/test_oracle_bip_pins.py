"""Pins for the bipartite ShockHash oracle (the outlook of Section 9: two hash
functions of range [n/2], one shifted by n/2; candidates filtered before they
are paired).  No GPU."""
import itertools
import math

import numpy as np
import pytest

from workloads import fixed_leaves, splitmix64


def _valid_masks(h0, h1):
    n = len(h0)
    return [f for f in range(1 << n) if len({h1[i] if (f >> i) & 1 else h0[i] for i in range(n)}) == n]


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_bip_matches_definition(oracle_mod, n):
    """The first pair in the order max(a, b), a, b for which some choice makes
    a bijection, and the smallest such choice, by enumerating all 2^n."""
    keys, offs = fixed_leaves(6, n, 1800 + n)
    rc, A, B, F = oracle_mod.bip_leaf_search(keys, offs)
    assert rc == 0
    for j in range(6):
        leaf = [int(x) for x in keys[int(offs[j]):int(offs[j + 1])]]
        want = None
        for m in range(200):
            order = [(a, m) for a in range(m)] + [(m, b) for b in range(m + 1)]
            for a, b in order:
                h0 = [oracle_mod.bip_slots(x, a, n)[0] for x in leaf]
                h1 = [oracle_mod.bip_slots(x, b, n)[1] for x in leaf]
                valid = _valid_masks(h0, h1)
                if valid:
                    want = (a, b, min(valid))
                    break
            if want:
                break
        assert (int(A[j]), int(B[j]), int(F[j])) == want


def test_bip_filter_does_not_change_results(oracle_mod):
    keys, offs = fixed_leaves(30, 12, 1810)
    a = oracle_mod.bip_leaf_search(keys, offs)
    b = oracle_mod.bip_leaf_search(keys, offs, use_filter=False)
    assert all(np.array_equal(x, y) for x, y in zip(a[1:], b[1:]))


def test_bip_cells_are_uniform_in_their_halves(oracle_mod):
    """left is uniform over [0, n/2), right over [n/2, n) (chi-square, 6 sd)."""
    n = 10
    keys = splitmix64(1811, 20000)
    left = np.zeros(n, np.int64)
    right = np.zeros(n, np.int64)
    for x in keys:
        l, r = oracle_mod.bip_slots(int(x), 3, n)
        left[l] += 1
        right[r] += 1
    assert left[n // 2:].sum() == 0 and right[:n // 2].sum() == 0
    for counts in (left[:n // 2], right[n // 2:]):
        e = counts.sum() / counts.size
        chi2 = float(((counts - e) ** 2 / e).sum())
        dof = counts.size - 1
        assert abs(chi2 - dof) < 6 * math.sqrt(2 * dof)


def test_bip_orientations_are_bijections(oracle_mod):
    keys, offs = fixed_leaves(50, 20, 1812)
    rc, A, B, F = oracle_mod.bip_leaf_search(keys, offs)
    assert rc == 0
    for j in range(50):
        leaf = [int(x) for x in keys[int(offs[j]):int(offs[j + 1])]]
        cells = [oracle_mod.bip_slots(x, int(B[j]), 20)[1] if (int(F[j]) >> i) & 1
                 else oracle_mod.bip_slots(x, int(A[j]), 20)[0] for i, x in enumerate(leaf)]
        assert sorted(cells) == list(range(20))


def test_bip_gain_over_shockhash_grows_exponentially(oracle_mod):
    """The paper expects an exponential reduction of the search: the seeds
    ShockHash needs divided by the seeds bipartite ShockHash draws (the
    larger seed of its pair) grows by a roughly constant factor per added
    key: checked as a steady increase of its logarithm from 16 to 24 to 32."""
    ratios = {}
    for n, L in ((16, 400), (24, 200), (32, 60)):
        keys, offs = fixed_leaves(L, n, 1820 + n)
        _, s, _ = oracle_mod.leaf_search(keys, offs)
        _, a, b, _ = oracle_mod.bip_leaf_search(keys, offs)
        ratios[n] = (s.astype(np.float64) + 1).mean() / (np.maximum(a, b).astype(np.float64) + 1).mean()
    lr = {n: math.log(r) for n, r in ratios.items()}
    assert lr[24] - lr[16] > 0.6 and lr[32] - lr[24] > 0.6, ratios


def test_bip_cap_and_tiny_leaves(oracle_mod):
    keys = splitmix64(1830, 40)
    offs = np.array([0, 0, 1, 40], np.uint64)
    rc, A, B, F = oracle_mod.bip_leaf_search(keys, offs)
    assert rc == 0 and list(A[:2]) == [0, 0] and list(B[:2]) == [0, 0] and list(F[:2]) == [0, 0]
    m = int(max(A[2], B[2]))
    rc, A2, B2, _ = oracle_mod.bip_leaf_search(keys, offs, max_seed=m)
    assert rc == oracle_mod.ENOTFOUND and int(A2[2]) == 2**64 - 1 and int(B2[2]) == 2**64 - 1
