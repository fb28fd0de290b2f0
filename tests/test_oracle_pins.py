"""Pins for the CPU oracle (no GPU).

Each test checks the oracle against something other than itself: the
definitions of Sections 4-5 evaluated by brute force (all 2^n choices f),
exhaustive enumeration of tiny graphs, algebraic properties of the frozen
hash, and exact probabilities of ideal hashing (tests/theory.py, itself
pinned by enumeration).
"""
import itertools
import math

import numpy as np
import pytest

import theory as T
from workloads import fixed_leaves, splitmix64

MASK64 = (1 << 64) - 1


# ---------------------------------------------------------------- hash ----

def _inv_xorshift(y, s):
    x = y
    for _ in range(64 // s + 1):
        x = y ^ (x >> s)
    return x & MASK64


def test_fmix64_round_trip(oracle_mod):
    """fmix64 is a bijection; undoing it with the modular inverses of its two
    multipliers and the inverse xorshift recovers the input, which fails for
    any wrong constant or shift in the oracle."""
    c1, c2 = 0xFF51AFD7ED558CCD, 0xC4CEB9FE1A85EC53
    i1, i2 = pow(c1, -1, 1 << 64), pow(c2, -1, 1 << 64)
    xs = [0, 1, 2, MASK64, 0x8000000000000000] + [int(v) for v in splitmix64(99, 200)]
    for x in xs:
        y = oracle_mod.fmix64(x)
        z = _inv_xorshift(y, 33)
        z = (z * i2) & MASK64
        z = _inv_xorshift(z, 33)
        z = (z * i1) & MASK64
        z = _inv_xorshift(z, 33)
        assert z == x


def _fmix64_inverse(y):
    c1, c2 = 0xFF51AFD7ED558CCD, 0xC4CEB9FE1A85EC53
    z = _inv_xorshift(y, 33)
    z = (z * pow(c2, -1, 1 << 64)) & MASK64
    z = _inv_xorshift(z, 33)
    z = (z * pow(c1, -1, 1 << 64)) & MASK64
    return _inv_xorshift(z, 33)


@pytest.mark.parametrize("shared", ["low", "high"])
def test_slots_depend_on_both_halves_of_the_mixed_key(oracle_mod, shared):
    """Keys whose mixed codes agree in one 32-bit half and differ in the other
    must still get unrelated slots: the per-seed product combines both halves,
    so a hash that silently dropped a half would give them identical slots."""
    ys = [int(v) for v in splitmix64(31, 40)]
    for y1 in ys[:20]:
        flip = ys[20 + ys.index(y1)] | 1
        y2 = y1 ^ ((flip << 32) & MASK64) if shared == "low" else y1 ^ (flip & 0xFFFFFFFF)
        x1, x2 = _fmix64_inverse(y1), _fmix64_inverse(y2)
        assert oracle_mod.fmix64(x1) == y1 and oracle_mod.fmix64(x2) == y2
        same = sum(oracle_mod.slots(x1, s, 64) == oracle_mod.slots(x2, s, 64) for s in range(200))
        assert same < 20


@pytest.mark.parametrize("n", [1, 2, 3, 5, 24, 31, 32, 33, 48, 63, 64])
def test_slots_range_and_no_self_loops(oracle_mod, n):
    keys = splitmix64(7, 50)
    for s in range(40):
        for x in keys:
            h0, h1 = oracle_mod.slots(int(x), s, n)
            assert 0 <= h0 < n and 0 <= h1 < n
            if n >= 2:
                assert h0 != h1
            else:
                assert h0 == h1 == 0


def _chi2_ok(counts, expected, dof_sigmas=6.0):
    counts = np.asarray(counts, dtype=np.float64)
    stat = ((counts - expected) ** 2 / expected).sum()
    dof = counts.size - 1
    return stat < dof + dof_sigmas * math.sqrt(2 * dof)


@pytest.mark.parametrize("n", [5, 7, 48])
def test_slot_pairs_uniform_over_distinct_cells(oracle_mod, n):
    """Fully random loop-free hashing: (h0, h1) uniform over ordered pairs of
    distinct cells (footnote on self-loops, Section 5)."""
    keys = splitmix64(11, 64)
    counts = np.zeros((n, n), dtype=np.int64)
    seeds = 6000 if n < 10 else 3000
    for s in range(seeds):
        for x in keys[:16]:
            h0, h1 = oracle_mod.slots(int(x), s, n)
            counts[h0, h1] += 1
    assert counts.trace() == 0
    off = counts[~np.eye(n, dtype=bool)]
    assert _chi2_ok(off, off.sum() / off.size)


@pytest.mark.parametrize("n", [5, 6, 7, 8])
def test_h0_alone_is_bijection_at_lemma_rate(oracle_mod, n):
    """Lemma lem:bruteForce: a random function is a bijection with probability
    n!/n^n; h0 under successive seeds must behave like one."""
    count = 400_000 if n < 8 else 800_000
    keys = splitmix64(1000 + n, n)
    _, _, bij = oracle_mod.seed_stats(keys, 0, count)
    p = float(T.bijection_probability(n))
    sd = math.sqrt(count * p * (1 - p))
    assert abs(bij - count * p) < 5 * sd


# ------------------------------------------- pseudoforest & orientation ----

def _all_f_valid(h0, h1):
    n = len(h0)
    valid = []
    for f in range(1 << n):
        used = set()
        for i in range(n):
            used.add(h1[i] if (f >> i) & 1 else h0[i])
        if len(used) == n:
            valid.append(f)
    return valid


def _components(n, h0, h1):
    label = list(range(n))
    changed = True
    while changed:
        changed = False
        for a, b in zip(h0, h1):
            m = min(label[a], label[b])
            if label[a] != m or label[b] != m:
                label[a] = label[b] = m
                changed = True
    return len(set(label))


@pytest.mark.parametrize("n,loops", [(1, True), (2, True), (3, True), (2, False), (3, False), (4, False)])
def test_pseudoforest_equals_orientability_exhaustive(oracle_mod, n, loops):
    """Eq. pseudoforests-orientable: PF(G) iff some f gives a bijection, over
    every graph with n keys on n cells; when it holds, Eq. orientations-cycles:
    exactly 2^c(G) choices work and the oracle's orientation is the smallest."""
    pairs = [(u, v) for u in range(n) for v in range(n) if loops or u != v]
    for g in itertools.product(pairs, repeat=n):
        h0 = [e[0] for e in g]
        h1 = [e[1] for e in g]
        valid = _all_f_valid(h0, h1)
        pf = oracle_mod.is_pseudoforest(n, h0, h1)
        assert pf == bool(valid), g
        f = oracle_mod.orientation(n, h0, h1)
        if not valid:
            assert f is None
            continue
        assert len(valid) == 2 ** _components(n, h0, h1)
        assert f == min(valid)


@pytest.mark.parametrize("n", [5, 6, 7, 8, 9, 10])
def test_orientation_random_graphs(oracle_mod, n):
    rng = np.random.default_rng(100 + n)
    seen_pf = 0
    for _ in range(300 if n <= 8 else 120):
        h0 = rng.integers(0, n, n)
        r = rng.integers(0, n - 1, n)
        h1 = r + (r >= h0)
        valid = _all_f_valid(list(h0), list(h1))
        assert oracle_mod.is_pseudoforest(n, h0, h1) == bool(valid)
        f = oracle_mod.orientation(n, h0, h1)
        if valid:
            seen_pf += 1
            assert len(valid) == 2 ** _components(n, list(h0), list(h1))
            assert f == min(valid)
        else:
            assert f is None
    assert seen_pf > 0


def test_pseudoforest_with_fewer_edges(oracle_mod):
    # A forest (fewer edges than nodes) is a pseudoforest; a triangle plus a
    # chord is not.
    assert oracle_mod.is_pseudoforest(5, [0, 1, 2], [1, 2, 3])
    assert not oracle_mod.is_pseudoforest(3, [0, 1, 2, 0], [1, 2, 0, 2])


# ---------------------------------------------------------- leaf search ----

def _brute_force_search(oracle_mod, keys, start=0, cap=10_000):
    """Section 4's definition read literally: the smallest s such that some of
    the 2^n choices f makes x -> h_{s,f(x)}(x) a bijection, and the smallest
    such f."""
    n = len(keys)
    for s in range(start, cap):
        h0, h1 = oracle_mod.leaf_slots(keys, s)
        valid = _all_f_valid(list(h0), list(h1))
        if valid:
            return s, min(valid)
    return None, None


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8, 9])
def test_leaf_search_matches_definition(oracle_mod, n):
    keys, offs = fixed_leaves(12 if n <= 7 else 5, n, 300 + n)
    rc, seeds, orient = oracle_mod.leaf_search(keys, offs)
    assert rc == 0
    for j in range(len(offs) - 1):
        leaf = keys[int(offs[j]):int(offs[j + 1])]
        s, f = _brute_force_search(oracle_mod, leaf)
        assert (int(seeds[j]), int(orient[j])) == (s, f)


def test_filter_does_not_change_results(oracle_mod):
    for n in (6, 12, 17, 24):
        keys, offs = fixed_leaves(30, n, 400 + n)
        a = oracle_mod.leaf_search(keys, offs, use_filter=True)
        b = oracle_mod.leaf_search(keys, offs, use_filter=False)
        assert a[0] == b[0] == 0
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_orientation_is_bijection_on_every_result(oracle_mod):
    keys, offs = fixed_leaves(60, 20, 500)
    rc, seeds, orient = oracle_mod.leaf_search(keys, offs)
    assert rc == 0
    for j in range(60):
        leaf = keys[int(offs[j]):int(offs[j + 1])]
        h0, h1 = oracle_mod.leaf_slots(leaf, int(seeds[j]))
        f = int(orient[j])
        slots = [int(h1[i]) if (f >> i) & 1 else int(h0[i]) for i in range(20)]
        assert sorted(slots) == list(range(20))
        assert f < (1 << 20)


def test_resume_and_cap(oracle_mod):
    keys, offs = fixed_leaves(10, 14, 600)
    rc, seeds, orient = oracle_mod.leaf_search(keys, offs)
    assert rc == 0
    for j in range(10):
        leaf = keys[int(offs[j]):int(offs[j + 1])]
        o = np.array([0, 14], dtype=np.uint64)
        s = int(seeds[j])
        # resuming anywhere at or below s* finds s* again
        for start in (0, s // 2, s):
            r = oracle_mod.leaf_search(leaf, o, start_seed=start)
            assert r[0] == 0 and int(r[1][0]) == s and int(r[2][0]) == int(orient[j])
        # resuming past s* finds the next qualifying seed, which is larger
        r = oracle_mod.leaf_search(leaf, o, start_seed=s + 1)
        assert r[0] == 0 and int(r[1][0]) > s
        # a cap at s* (exclusive) reports not-found
        r = oracle_mod.leaf_search(leaf, o, max_seed=s)
        assert r[0] == oracle_mod.ENOTFOUND
        assert r[1][0] == oracle_mod.NOT_FOUND_SEED and int(r[2][0]) == 0


def test_edge_cases(oracle_mod):
    # empty batch
    rc, s, o = oracle_mod.leaf_search(np.zeros(0, np.uint64), np.zeros(1, np.uint64))
    assert rc == 0 and s.size == 0
    # empty leaf and single-key leaf: the first seed tried qualifies
    keys = np.array([123], dtype=np.uint64)
    offs = np.array([0, 0, 1, 1], dtype=np.uint64)
    rc, s, o = oracle_mod.leaf_search(keys, offs, start_seed=5)
    assert rc == 0 and list(s) == [5, 5, 5] and list(o) == [0, 0, 0]
    # two keys: always solvable at the first seed (h1 = 1 - h0)
    keys, offs = fixed_leaves(20, 2, 700)
    rc, s, o = oracle_mod.leaf_search(keys, offs)
    assert rc == 0 and (s == 0).all()
    # leaf larger than 64 keys, decreasing offsets
    keys = splitmix64(1, 65)
    assert oracle_mod.leaf_search(keys, np.array([0, 65], np.uint64))[0] == oracle_mod.EINVAL
    assert oracle_mod.leaf_search(keys, np.array([0, 10, 5], np.uint64))[0] == oracle_mod.EINVAL


def test_duplicate_keys(oracle_mod):
    base = splitmix64(800, 10)
    # two equal keys form a double edge (a 2-cycle): still solvable
    keys = np.concatenate([base, base[:1]])
    rc, s, o = oracle_mod.leaf_search(keys, np.array([0, 11], np.uint64))
    assert rc == 0
    h0, h1 = oracle_mod.leaf_slots(keys, int(s[0]))
    f = int(o[0])
    slots = [int(h1[i]) if (f >> i) & 1 else int(h0[i]) for i in range(11)]
    assert sorted(slots) == list(range(11))
    # three equal keys put three edges on two cells: never a pseudoforest
    keys = np.concatenate([base[:8], base[:1], base[:1]])
    rc, s, o = oracle_mod.leaf_search(keys, np.array([0, 10], np.uint64), max_seed=5000)
    assert rc == oracle_mod.ENOTFOUND and s[0] == oracle_mod.NOT_FOUND_SEED


# ------------------------------------------------------ statistics ----

@pytest.mark.parametrize("n,leaves", [(8, 20000), (12, 8000), (16, 4000), (20, 1500)])
def test_seed_count_matches_ideal_hashing(oracle_mod, n, leaves):
    """Seeds are independent trials: s* + 1 is geometric with the exact
    acceptance probability of loop-free ideal hashing (tests/theory.py).  The
    sample mean must lie within 5 standard errors."""
    keys, offs = fixed_leaves(leaves, n, 2000 + n)
    rc, seeds, _ = oracle_mod.leaf_search(keys, offs)
    assert rc == 0
    p = float(T.p_accept(n))
    tries = seeds.astype(np.float64) + 1
    mu = 1 / p
    sd = math.sqrt(1 - p) / p
    assert abs(tries.mean() - mu) < 5 * sd / math.sqrt(leaves)
    # distribution shape: P(s* >= k) = (1-p)^k at a few quantiles
    for k in (1, int(mu), int(2 * mu)):
        tail = float((seeds >= k).mean())
        expect = (1 - p) ** k
        assert abs(tail - expect) < 5 * math.sqrt(expect * (1 - expect) / leaves) + 1e-12


@pytest.mark.parametrize("n,count", [(16, 60000), (24, 60000), (32, 120000)])
def test_filter_pass_rate_matches_ideal_hashing(oracle_mod, n, count):
    """The bit-mask filter of Section 4 passes with the exact coverage
    probability q'_n, which is below Lemma lem:filterProbability's bound."""
    total_cover = total_pf = 0
    leaves = 4
    for j in range(leaves):
        keys = splitmix64(3000 + 17 * n + j, n)
        c, pf, _ = oracle_mod.seed_stats(keys, 0, count)
        total_cover += c
        total_pf += pf
    N = count * leaves
    q = float(T.q_cover(n))
    assert abs(total_cover - N * q) < 5 * math.sqrt(N * q * (1 - q))
    p = float(T.p_accept(n))
    assert abs(total_pf - N * p) < 5 * math.sqrt(N * p * (1 - p)) + 3
