"""Pins for the oracle's flat ShockHash MPHF (Section 8's flat decomposition;
the two-level scheme of Appendix A.4), its ribbon retrieval (one GF(2)
system per bucket) and its XOR retrieval.  No GPU.

Small leaves keep the oracle's leaf searches fast; the structure does not
depend on the leaf size beyond the parameters."""
import math

import numpy as np
import pytest

from workloads import splitmix64

SMALL = dict(bucket_size=300, leaf_target=12, leaf_max=18)


@pytest.mark.parametrize("rf", [False, True], ids=["plain", "rf"])
@pytest.mark.parametrize("N", [0, 1, 2, 17, 1000, 6000])
def test_mphf_is_a_bijection(oracle_mod, N, rf):
    """The defining property: N distinct keys map one-to-one onto [0, N),
    with plain or rotation-fitting leaves."""
    keys = splitmix64(1100 + N, N)
    rc, lay = oracle_mod.mphf_build(keys, rf=rf, **SMALL)
    assert rc == 0
    assert sorted(lay["positions"].tolist()) == list(range(N))
    if N:
        rc, q = oracle_mod.mphf_query(lay, keys)
        assert rc == 0 and (q == lay["positions"]).all()


def test_layout_invariants(oracle_mod):
    N = 5000
    keys = splitmix64(1201, N)
    rc, lay = oracle_mod.mphf_split(keys, **SMALL)
    assert rc == 0
    B = lay["n_buckets"]
    assert B == math.ceil(N / SMALL["bucket_size"])
    bo, lb, sz = lay["bucket_offset"].astype(np.int64), lay["leaf_base"].astype(np.int64), lay["leaf_sizes"]
    assert bo[0] == 0 and bo[-1] == N and (np.diff(bo) >= 0).all()
    m = np.diff(bo)
    assert (np.diff(lb) == (m + SMALL["leaf_target"] - 1) // SMALL["leaf_target"]).all()
    assert int(sz.max()) <= SMALL["leaf_max"] and int(sz.astype(np.int64).sum()) == N
    for b in range(B):  # a bucket's leaves hold exactly its keys
        assert int(sz[lb[b]:lb[b + 1]].astype(np.int64).sum()) == m[b]
    lk, ki, offs = lay["leaf_keys"], lay["key_index"].astype(np.int64), lay["leaf_offsets"].astype(np.int64)
    assert sorted(ki.tolist()) == list(range(N)) and (keys[ki] == lk).all()
    for j in range(lay["n_leaves"]):
        seg = lk[offs[j]:offs[j + 1]]
        assert seg.size < 2 or (seg[1:] > seg[:-1]).all()  # ascending


def test_bucket_sizes_are_binomial(oracle_mod):
    """Uniform bucketing: sizes have mean N/B and variance N/B (1 - 1/B)."""
    N = 200_000
    keys = splitmix64(1202, N)
    rc, lay = oracle_mod.mphf_split(keys, bucket_size=500, leaf_target=32, leaf_max=64)
    assert rc == 0
    m = np.diff(lay["bucket_offset"].astype(np.int64)).astype(np.float64)
    B = m.size
    mu, var = N / B, N / B * (1 - 1 / B)
    assert abs(m.mean() - mu) < 1e-9
    assert abs(m.var() / var - 1) < 4 * math.sqrt(2 / B)


def test_splitting_seed_bounds_every_leaf(oracle_mod):
    """Tight leaves force nonzero splitting seeds; every leaf still fits."""
    keys = splitmix64(1203, 20000)
    rc, lay = oracle_mod.mphf_split(keys, bucket_size=400, leaf_target=10, leaf_max=14)
    assert rc == 0
    assert int(lay["leaf_sizes"].max()) <= 14
    assert (lay["sigma"] > 0).sum() > 0


def test_mphf_rejects_bad_parameters(oracle_mod):
    keys = splitmix64(1204, 100)
    for bad in (dict(bucket_size=0, leaf_target=8, leaf_max=16), dict(bucket_size=100, leaf_target=20, leaf_max=16),
                dict(bucket_size=100, leaf_target=8, leaf_max=65)):
        rc, _ = oracle_mod.mphf_split(keys, **bad)
        assert rc == oracle_mod.EINVAL


def test_mphf_split_limits(oracle_mod):
    """A bucket may hold 1024 leaves but not 1025 (EINVAL), and a bucket
    whose leaf sizes cannot all fit its window and leaf_max under any of the
    2^16 splitting seeds is not found (a bucket of about 2400 keys in leaves
    of 24 on average, at most 29: about 0.87^96 of the splits fit)."""
    keys = splitmix64(1205, 2050)
    rc, lay = oracle_mod.mphf_split(keys[:2048], bucket_size=4096, leaf_target=2, leaf_max=8)
    assert rc == 0 and lay["n_leaves"] == 1024
    rc, _ = oracle_mod.mphf_split(keys, bucket_size=4096, leaf_target=2, leaf_max=8)
    assert rc == oracle_mod.EINVAL
    rc, _ = oracle_mod.mphf_split(splitmix64(9602, 13700), bucket_size=2406, leaf_target=24, leaf_max=29)
    assert rc == oracle_mod.ENOTFOUND


@pytest.mark.parametrize("N", [1, 10, 1000, 100_000])
def test_xor_retrieval_returns_every_value(oracle_mod, N):
    keys = splitmix64(1300 + N, N)
    values = (splitmix64(1400 + N, N) & np.uint64(1)).astype(np.uint8)
    rc, rho, z = oracle_mod.xor_build(keys, values)
    assert rc == 0
    assert (oracle_mod.xor_get(keys, rho, z) == values).all()
    assert z.size == 3 * oracle_mod.xor_segment(N)


def test_xor_retrieval_peels_at_the_load_the_threshold_allows(oracle_mod):
    """3-hypergraphs with at most 1/1.2218 edges per vertex peel completely
    with high probability (the 2-core threshold for k = 3); at 1.23 cells per
    key the first seed succeeds for large N."""
    N = 200_000
    for start in range(3):
        keys = splitmix64(1500 + start, N)
        rc, rho, _ = oracle_mod.xor_build(keys, np.zeros(N, np.uint8), rho_start=start * 100, max_tries=1)
        assert rc == 0 and rho == start * 100


def test_xor_retrieval_detects_an_unsolvable_system(oracle_mod):
    """Two identical keys with different values share all three cells: the
    pair never peels and no seed solves it."""
    keys = np.concatenate([splitmix64(1600, 50), np.array([7, 7], np.uint64)])
    values = np.zeros(52, np.uint8)
    values[-1] = 1
    rc, _, _ = oracle_mod.xor_build(keys, values, max_tries=8)
    assert rc == oracle_mod.ENOTFOUND


def test_space_accounting_matches_appendix_formula(oracle_mod):
    """Appendix A.4: the prefix sums cost about (N/b) log2 N + (N/n) log2 b
    bits.  The library stores a bucket's key offset in 32 bits relative to its
    block of 16 buckets (plus 64-bit key and leaf offsets per block) and each
    leaf size in 5 bits, which the splitting seed makes possible (every size
    lies in a window of 32): below the formula, whose leaf term spends
    log2 b = 11 bits per leaf, and above half of it."""
    N, b, n = 60_000, 2000, 40
    keys = splitmix64(1700, N)
    rc, lay = oracle_mod.mphf_split(keys, bucket_size=b, leaf_target=n, leaf_max=56)
    assert rc == 0
    B = lay["n_buckets"]
    formula = N / b * math.log2(N) + N / n * math.log2(b)
    stored = B * 32 + -(-(B + 1) // 16) * 128 + lay["n_leaves"] * 5
    assert formula / 2 < stored < formula


def test_bip_pair_rank_is_the_search_order(oracle_mod):
    """The stored value of a bipartite leaf is the rank of its pair in the
    order the search meets pairs (max(a, b), then a, then b), enumerated
    here pair by pair."""
    order = []
    for m in range(40):
        order += [(a, m) for a in range(m)] + [(m, b) for b in range(m + 1)]
    assert len(order) == 40 * 40
    for rank, (a, b) in enumerate(order):
        assert oracle_mod.bip_pair_rank(a, b) == rank, (a, b)
    assert oracle_mod.bip_pair_rank(2**31, 0) == 2**62 + 2**31


@pytest.mark.parametrize("N", [0, 1, 2, 17, 1000, 6000])
def test_bip_mphf_is_a_bijection(oracle_mod, N):
    keys = splitmix64(2600 + N, N)
    rc, lay = oracle_mod.mphf_build(keys, bip=True, **SMALL)
    assert rc == 0
    assert sorted(lay["positions"].tolist()) == list(range(N))


def test_bip_mphf_positions_follow_the_pair_cells(oracle_mod):
    """A bipartite leaf's keys land at offset + left(x, a) or offset +
    right(x, b), by their retrieved choice, for the pair the bipartite search
    found; checked key by key against the oracle's cell function on a 20,000-key
    build with the default layout."""
    keys = splitmix64(2700, 20000)
    rc, lay = oracle_mod.mphf_build(keys, bip=True)
    assert rc == 0
    assert sorted(lay["positions"].tolist()) == list(range(20000))
    lk, offs = lay["leaf_keys"], lay["leaf_offsets"]
    rc, pa, pb, orient = oracle_mod.bip_leaf_search(lk, offs)
    assert rc == 0
    pos_of = {int(k): int(p) for k, p in zip(keys, lay["positions"])}
    for j in range(0, lay["n_leaves"], 37):
        o, n = int(offs[j]), int(offs[j + 1] - offs[j])
        assert int(lay["seeds"][j]) == oracle_mod.bip_pair_rank(int(pa[j]), int(pb[j]))
        for i in range(n):
            x = int(lk[o + i])
            left, _ = oracle_mod.bip_slots(x, int(pa[j]), n)
            _, right = oracle_mod.bip_slots(x, int(pb[j]), n)
            cell = right if (int(orient[j]) >> i) & 1 else left
            assert pos_of[x] == o + cell, (j, i)


# ---- ribbon retrieval (per-bucket GF(2) systems) -----------------------------------

def _brute_canonical(rows_bits, b, cols):
    """Brute force over all 2^cols vectors: (solvable, the solution whose
    non-pivot columns are 0), with pivot columns found by checking whether
    each column lies in the span of the columns before it."""
    m = len(rows_bits)
    col = [sum(((rows_bits[r] >> c) & 1) << r for r in range(m)) for c in range(cols)]
    pivots = []
    span = {0}
    for c in range(cols):
        if col[c] not in span:
            pivots.append(c)
            span = span | {v ^ col[c] for v in span}
    rhs = sum((int(b[r]) & 1) << r for r in range(m))
    sols = []
    for x in range(1 << cols):
        acc = 0
        for c in range(cols):
            if (x >> c) & 1:
                acc ^= col[c]
        if acc == rhs:
            sols.append(x)
    if not sols:
        return False, None
    free = [c for c in range(cols) if c not in pivots]
    canon = [x for x in sols if all(not (x >> c) & 1 for c in free)]
    assert len(canon) == 1  # fixing the free columns leaves exactly one solution
    return True, canon[0]


def test_gf2_solve_matches_brute_force(oracle_mod):
    rng = np.random.default_rng(2800)
    seen = {True: 0, False: 0}
    for trial in range(400):
        m = int(rng.integers(0, 9))
        cols = int(rng.integers(1, 13))
        density = rng.uniform(0.1, 0.6)
        rows_bits = [int(sum(1 << c for c in range(cols) if rng.random() < density)) for _ in range(m)]
        b = rng.integers(0, 2, m).astype(np.uint8)
        rows = np.array([[r] for r in rows_bits], dtype=np.uint64).reshape(m, 1)
        ok, z = oracle_mod.gf2_solve(rows, b, cols)
        want_ok, want = _brute_canonical(rows_bits, b, cols)
        assert ok == want_ok, trial
        seen[ok] += 1
        if ok:
            got = sum(int(z[c]) << c for c in range(cols))
            assert got == want, (trial, rows_bits, list(b))
    assert seen[True] > 50 and seen[False] > 50


def test_gf2_solve_wide_rows(oracle_mod):
    """Several words per row: a random banded system solved by the oracle
    satisfies every equation, and its zeros sit on the columns that lie in the
    span of the columns before them (checked by a second elimination that
    tracks only column independence)."""
    rng = np.random.default_rng(2801)
    m, cols = 150, 200
    W = (cols + 63) // 64
    rows = np.zeros((m, W), np.uint64)
    dense = np.zeros((m, cols), np.uint8)
    for r in range(m):
        s = int(rng.integers(0, cols - 40))
        for c in range(s, s + 40):
            if rng.random() < 0.5 or c == s:
                dense[r, c] = 1
                rows[r, c // 64] |= np.uint64(1 << (c % 64))
    b = rng.integers(0, 2, m).astype(np.uint8)
    ok, z = oracle_mod.gf2_solve(rows, b, cols)
    assert ok
    assert ((dense.astype(np.int64) @ z.astype(np.int64)) % 2 == b).all()
    # independent columns from the left: column c is a pivot iff adding it raises the rank
    basis = {}
    pivots = []
    for c in range(cols):
        v = int("".join(str(int(x)) for x in dense[:, c][::-1]), 2)
        while v:
            top = v.bit_length() - 1
            if top not in basis:
                basis[top] = v
                pivots.append(c)
                break
            v ^= basis[top]
    free = sorted(set(range(cols)) - set(pivots))
    assert (z[free] == 0).all()


def test_ribbon_rows(oracle_mod):
    """Rows start in [0, cols - 64], carry 64 bits with bit 0 set, and start
    uniformly (chi-square over 16 bins)."""
    assert oracle_mod.ribbon_cols(0) == 0
    assert oracle_mod.ribbon_cols(1) == 64 and oracle_mod.ribbon_cols(62) == 64 and oracle_mod.ribbon_cols(63) == 65
    assert oracle_mod.ribbon_cols(3000) == 3060 and oracle_mod.ribbon_cols(3001) == 3062
    cols = 3060
    starts = []
    for i, x in enumerate(splitmix64(2802, 20000)):
        s, c = oracle_mod.ribbon_row(int(x), i % 3, cols)
        assert 0 <= s <= cols - 64 and c & 1
        starts.append(s)
    h, _ = np.histogram(starts, bins=16, range=(0, cols - 63))
    e = len(starts) / 16
    assert ((h - e) ** 2 / e).sum() < 50  # 15 degrees of freedom: p < 1e-4 beyond 45


@pytest.mark.parametrize("m", [1, 5, 63, 64, 65, 500, 3000])
def test_ribbon_returns_every_value(oracle_mod, m):
    keys = splitmix64(2900 + m, m)
    values = (splitmix64(3000 + m, m) & np.uint64(1)).astype(np.uint8)
    rc, rseed, z = oracle_mod.ribbon_build(keys, values)
    assert rc == 0 and rseed < oracle_mod.RIBBON_MAX_SEEDS
    cols = oracle_mod.ribbon_cols(m)
    assert z.size == cols
    got = np.array([oracle_mod.ribbon_get(int(x), rseed, cols, z) for x in keys], np.uint8)
    assert (got == values).all()


def test_ribbon_seeds_are_few_at_two_percent(oracle_mod):
    """With 2 % more columns than keys, buckets of 3000 keys need few seeds:
    over 30 buckets the mean seed stays below 4 and none reaches 32."""
    seeds = []
    for t in range(30):
        keys = splitmix64(3100 + t, 3000)
        values = (splitmix64(3200 + t, 3000) & np.uint64(1)).astype(np.uint8)
        rc, rseed, _ = oracle_mod.ribbon_build(keys, values)
        assert rc == 0
        seeds.append(rseed)
    assert np.mean(seeds) < 4 and max(seeds) < 32, seeds


def test_ribbon_detects_an_unsolvable_bucket(oracle_mod):
    """Two identical keys with different values have identical rows under
    every seed: no seed solves the bucket."""
    keys = np.concatenate([splitmix64(3300, 50), np.array([7, 7], np.uint64)])
    values = np.zeros(52, np.uint8)
    values[-1] = 1
    rc, _, _ = oracle_mod.ribbon_build(keys, values, max_seeds=8)
    assert rc == oracle_mod.ENOTFOUND


def test_leaf_sizes_fit_five_bits(oracle_mod):
    """Every leaf of a bucket of m keys in L leaves holds between
    max(0, floor(m / L) - 16) and that + 31 keys (at most leaf_max)."""
    keys = splitmix64(3400, 60000)
    rc, lay = oracle_mod.mphf_split(keys, bucket_size=3000, leaf_target=40, leaf_max=56)
    assert rc == 0
    bo, lb, sz = lay["bucket_offset"].astype(np.int64), lay["leaf_base"].astype(np.int64), lay["leaf_sizes"]
    for b in range(lay["n_buckets"]):
        m, L = int(bo[b + 1] - bo[b]), int(lb[b + 1] - lb[b])
        lo = oracle_mod.leaf_size_base(m, L)
        assert lo == max(0, m // L - 16)
        s = sz[lb[b]:lb[b + 1]].astype(np.int64)
        assert (s >= lo).all() and (s <= lo + 31).all() and (s <= 56).all(), b


@pytest.mark.parametrize("N", [0, 1, 17, 1000, 6000])
def test_mphf_with_xor_retrieval_is_a_bijection(oracle_mod, N):
    keys = splitmix64(3500 + N, N)
    rc, lay = oracle_mod.mphf_build(keys, retrieval=oracle_mod.RETRIEVAL_XOR, **SMALL)
    assert rc == 0
    assert sorted(lay["positions"].tolist()) == list(range(N))
    if N:
        rc, q = oracle_mod.mphf_query(lay, keys)
        assert rc == 0 and (q == lay["positions"]).all()
