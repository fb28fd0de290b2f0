"""Pins for the oracle's checker `shock_oracle_verify` (no GPU).

verify() judges a claimed (seed, orientation) per leaf with four flags:
  1  the claimed seed does not qualify (no bijective choice f, Section 4)
  2  the orientation is not the canonical one (the smallest valid mask)
  4  some seed in [max(start, s - window), s) qualifies
  8  the claim is "no seed" (UINT64_MAX)
Every expectation below comes from Section 4's definition evaluated by brute
force over all 2^n choices f on small leaves, not from the oracle's search,
so a planted mistake in verify (a wrong flag, an off-by-one window, a window
that ignores the start seed, an orientation check that accepts any valid
mask) fails one of them.
"""
import numpy as np
import pytest

from workloads import fixed_leaves

N = 7


def _valid_masks(oracle_mod, leaf, s):
    """All f (bit i = choice of key i) making key -> h_{f_i}(x_i, s) a bijection."""
    h0, h1 = oracle_mod.leaf_slots(leaf, s)
    n = len(leaf)
    out = []
    for f in range(1 << n):
        cells = {int(h1[i]) if (f >> i) & 1 else int(h0[i]) for i in range(n)}
        if len(cells) == n:
            out.append(f)
    return out


def _qualifying(oracle_mod, leaf, count):
    """The first `count` qualifying seeds of a leaf with their smallest masks, by brute force."""
    found = []
    s = 0
    while len(found) < count:
        v = _valid_masks(oracle_mod, leaf, s)
        if v:
            found.append((s, min(v), v))
        s += 1
    return found


def _verify_one(oracle_mod, leaf, seed, orient, start=0, window=64):
    offs = np.array([0, len(leaf)], np.uint64)
    return int(oracle_mod.verify(leaf, offs, np.array([seed], np.uint64), np.array([orient], np.uint64),
                                 start_seed=start, window=window)[0])


@pytest.fixture(scope="module")
def leaves(oracle_mod):
    keys, offs = fixed_leaves(6, N, 4242)
    out = []
    for j in range(6):
        leaf = keys[int(offs[j]):int(offs[j + 1])]
        out.append((leaf, _qualifying(oracle_mod, leaf, 2)))
    return out


def test_correct_claim_passes(oracle_mod, leaves):
    for leaf, q in leaves:
        s1, f1, _ = q[0]
        assert _verify_one(oracle_mod, leaf, s1, f1, window=10_000) == 0


def test_non_qualifying_seed_sets_bit0(oracle_mod, leaves):
    for leaf, q in leaves:
        (s1, f1, _), (s2, _, _) = q
        bad = [s for s in range(s1 + 1, s2)]
        if not bad:
            continue
        s = bad[0]
        assert not _valid_masks(oracle_mod, leaf, s)
        # window 0 looks at no seed below, so only bit 0 remains
        assert _verify_one(oracle_mod, leaf, s, f1, window=0) == 1
        # a window reaching s1 also reports the qualifying seed below
        assert _verify_one(oracle_mod, leaf, s, f1, window=s - s1) == 1 | 4


def test_wrong_orientation_sets_bit1(oracle_mod, leaves):
    checked_valid = 0
    for leaf, q in leaves:
        s1, f1, valid = q[0]
        # an arbitrary wrong mask
        assert _verify_one(oracle_mod, leaf, s1, f1 ^ 1, window=0) == 2
        # a bit beyond the leaf's n keys
        assert _verify_one(oracle_mod, leaf, s1, f1 | (1 << N), window=0) == 2
        # another VALID orientation (a bijection too) that is not the smallest
        others = [f for f in valid if f != f1]
        for f in others:
            assert f > f1
            assert _verify_one(oracle_mod, leaf, s1, f, window=0) == 2
            checked_valid += 1
    assert checked_valid > 0  # every pseudoforest has at least 2 valid masks (2^c, c >= 1)


def test_window_bound_is_exact(oracle_mod, leaves):
    for leaf, q in leaves:
        (s1, _, _), (s2, f2, _) = q
        gap = s2 - s1
        # claiming the second qualifying seed: the window must reach s1 exactly
        assert _verify_one(oracle_mod, leaf, s2, f2, window=gap) == 4
        assert _verify_one(oracle_mod, leaf, s2, f2, window=gap - 1) == 0
        assert _verify_one(oracle_mod, leaf, s2, f2, window=gap + 100) == 4


def test_window_clips_at_start_seed(oracle_mod, leaves):
    for leaf, q in leaves:
        (s1, _, _), (s2, f2, _) = q
        # seeds below the start are not candidates: s1 is excluded when start > s1
        assert _verify_one(oracle_mod, leaf, s2, f2, start=s1 + 1, window=10_000) == 0
        assert _verify_one(oracle_mod, leaf, s2, f2, start=s1, window=10_000) == 4


def test_not_found_claim_sets_bit3(oracle_mod, leaves):
    leaf, _ = leaves[0]
    assert _verify_one(oracle_mod, leaf, (1 << 64) - 1, 0) == 8


def test_flags_are_per_leaf(oracle_mod, leaves):
    """A batch mixing good and planted claims flags exactly the planted leaves."""
    keys = np.concatenate([leaf for leaf, _ in leaves])
    offs = np.arange(len(leaves) + 1, dtype=np.uint64) * np.uint64(N)
    seeds = np.array([q[0][0] for _, q in leaves], np.uint64)
    orient = np.array([q[0][1] for _, q in leaves], np.uint64)
    seeds[2] = np.uint64(q2 := leaves[2][1][1][0])  # second qualifying seed of leaf 2
    orient[2] = np.uint64(leaves[2][1][1][1])
    orient[4] ^= np.uint64(1)
    flags = oracle_mod.verify(keys, offs, seeds, orient, window=q2 + 1)
    want = np.zeros(len(leaves), np.uint8)
    want[2] = 4
    want[4] = 2
    assert np.array_equal(flags, want)
