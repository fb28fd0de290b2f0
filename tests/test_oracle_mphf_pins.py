"""Pins for the oracle's flat ShockHash MPHF (Section 8's flat decomposition;
the two-level scheme of Appendix A.4) and its XOR retrieval.  No GPU.

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
    bits.  The structure's bucket and leaf-size parts are within a small
    factor of that (it stores fixed-width words instead of minimal widths)."""
    N, b, n = 60_000, 2000, 40
    keys = splitmix64(1700, N)
    rc, lay = oracle_mod.mphf_split(keys, bucket_size=b, leaf_target=n, leaf_max=64)
    assert rc == 0
    formula = N / b * math.log2(N) + N / n * math.log2(b)
    stored = (lay["n_buckets"] + 1) * 128 + lay["n_buckets"] * 32 + lay["n_leaves"] * 8
    assert formula < stored < 3 * formula


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
