"""GPU parity of bipartite ShockHash (shock_bip_leaf_search_ex) against the
oracle, through the C ABI: (a, b, orientation) bit-exact per leaf."""
import numpy as np
import pytest

from workloads import fixed_leaves, make_workload, splitmix64

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

MAX = np.uint64(0xFFFFFFFFFFFFFFFF)


@pytest.fixture(scope="module")
def shock():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09561_amd as shock
    shock.lib()
    return shock


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def _host(t):
    return t.cpu().numpy().view(np.uint64)


def gpu_bip(shock, keys, offs, **opts):
    print(f"[gpu] bip L={len(offs) - 1} opts={opts}", flush=True)
    k = _dev(keys) if len(keys) else torch.zeros(1, dtype=torch.int64, device="cuda")
    rc, a, b, f, st = shock.bip_leaf_search(k, _dev(offs), **opts)
    torch.cuda.synchronize()
    return rc, _host(a), _host(b), _host(f), st


def oracle_bip(oracle_mod, keys, offs, **kw):
    parts = oracle_mod.parallel(oracle_mod.bip_leaf_search, keys, offs, threads=16, **kw)
    rc = min(p[0] for p in parts)
    return (rc, *[np.concatenate([p[i] for p in parts]) for i in (1, 2, 3)])


def assert_same(g, o, what):
    bad = np.nonzero((g[1] != o[1]) | (g[2] != o[2]) | (g[3] != o[3]))[0]
    assert bad.size == 0, f"{what}: {bad.size} differ, first {bad[:4]}: gpu {g[1][bad[:4]]},{g[2][bad[:4]]} " \
                          f"oracle {o[1][bad[:4]]},{o[2][bad[:4]]}"
    assert g[0] == o[0], what


@pytest.mark.parametrize("n,L", [(2, 200), (3, 200), (5, 200), (8, 200), (16, 200), (24, 120), (32, 80), (40, 48),
                                 (48, 32), (56, 16), (64, 8)])
def test_bip_fixed_n_matches_oracle(shock, oracle_mod, n, L):
    keys, offs = fixed_leaves(L, n, 3000 + n)
    assert_same(gpu_bip(shock, keys, offs), oracle_bip(oracle_mod, keys, offs), f"n={n}")


def test_bip_64_key_leaves_and_the_second_pass(shock, oracle_mod):
    """64 leaves of 64 keys (about 35 candidates per side before the pair):
    with the default pools every leaf equals the oracle and none needs the
    second pass.  With bip_pool = 100 the first pass keeps 50 per side, so
    the leaves past that are searched again with pools of 100: each leaf
    then equals the oracle or, if it needs more than 100 on a side, is
    reported not found (all ones)."""
    keys, offs = fixed_leaves(64, 64, 3110)
    want = oracle_bip(oracle_mod, keys, offs)
    g = gpu_bip(shock, keys, offs)
    print(f"[gpu] bip 64 leaves of 64 keys: stats {g[4]}", flush=True)
    assert_same(g, want, "n=64")
    assert g[4]["second_pass_leaves"] == 0
    h = gpu_bip(shock, keys, offs, bip_pool=100)
    print(f"[gpu] bip 64 leaves of 64 keys, pool 100: stats {h[4]}", flush=True)
    lost = h[1] == MAX
    assert h[4]["second_pass_leaves"] > 0 and lost.sum() <= h[4]["second_pass_leaves"]
    assert (h[2][lost] == MAX).all()
    ok = ~lost
    assert (h[1][ok] == want[1][ok]).all() and (h[2][ok] == want[2][ok]).all() and (h[3][ok] == want[3][ok]).all()
    assert h[0] == (shock.SHOCK_ENOTFOUND if lost.any() else shock.SHOCK_OK)


def test_bip_uneven_batch_and_worker_counts(shock, oracle_mod):
    rng = np.random.default_rng(3100)
    sizes = np.repeat(np.arange(0, 50), 3)
    rng.shuffle(sizes)
    offs = np.zeros(len(sizes) + 1, np.uint64)
    np.cumsum(sizes, out=offs[1:])
    keys = splitmix64(3101, int(offs[-1]))
    want = oracle_bip(oracle_mod, keys, offs)
    for workers in (0, 1, 7, 64):
        assert_same(gpu_bip(shock, keys, offs, workers=workers), want, f"workers={workers}")


def test_bip_cap(shock, oracle_mod):
    keys, offs = fixed_leaves(40, 36, 3102)
    full = gpu_bip(shock, keys, offs)
    cap = int(np.median(np.maximum(full[1], full[2])))
    g = gpu_bip(shock, keys, offs, max_seed=cap)
    assert_same(g, oracle_bip(oracle_mod, keys, offs, max_seed=cap), "capped")
    assert g[0] == shock.SHOCK_ENOTFOUND and (g[1] == MAX).any() and (g[1] != MAX).any()


def test_bip_full_batch_statistics(shock, oracle_mod):
    """The fixed48 batch: every leaf's pair is a pseudoforest with a valid
    orientation (the oracle checks a sample end to end), the seeds drawn are a
    small fraction of the plain search's, and the lone-key filter spares the
    peeling test most pairs."""
    keys, offs = make_workload("fixed48")
    g = gpu_bip(shock, keys, offs)
    assert g[0] == 0
    st = g[4]
    L = len(offs) - 1
    print(f"[gpu] bip fixed48 stats {st}", flush=True)
    assert st["seeds_hashed"] / L < 2000 and st["kernel_ms"] > 0
    assert st["second_pass_leaves"] == 0  # a 48-key leaf gathers a few dozen candidates per side
    # every leaf peels at least its answer; the lone-key filter rejects most
    # candidate pairs (a one-edge tree is common when both halves are covered)
    assert L <= st["pairs_peeled"] < 0.6 * st["pairs_tested"]
    pick = np.random.default_rng(3103).choice(L, 32, replace=False)
    for j in pick:
        o = oracle_mod.bip_leaf_search(keys, offs[j:j + 2])
        assert (int(o[1][0]), int(o[2][0]), int(o[3][0])) == (int(g[1][j]), int(g[2][j]), int(g[3][j])), j


def _pool_adds(oracle_mod, leaf_keys, a, b):
    """Candidates the search adds to each side's pool before it reaches the
    pair (a, b), in its order: every left (right) candidate below m =
    max(a, b), and m itself on the right side when it is a right candidate
    whose pairs with the left pool failed (the answer is then (m, b))."""
    n = len(leaf_keys)
    nl = n // 2
    m = max(a, b)

    def covers(s):
        cells = [oracle_mod.bip_slots(int(x), s, n) for x in leaf_keys]
        return {c[0] for c in cells} == set(range(nl)), {c[1] for c in cells} == set(range(nl, n))

    adds_l = adds_r = 0
    for s in range(m):
        is_l, is_r = covers(s)
        adds_l += is_l
        adds_r += is_r
    if a == m and covers(m)[1]:
        adds_r += 1
    return adds_l, adds_r


@pytest.mark.parametrize("cap", [3, 4])
def test_bip_pool_limit_against_the_oracle(shock, oracle_mod, cap):
    """With bip_pool = cap candidates per side, exactly the leaves whose
    oracle answer comes after candidate cap + 1 on some side are reported
    not found (outputs all ones); every other leaf equals the oracle.  The
    first pass keeps cap / 2, so the leaves between the two limits are found
    by the second pass (25 of these 60 leaves at cap 3, 8 at cap 4; 7 and 3
    go past the limit)."""

    keys, offs = fixed_leaves(60, 12, 3105)
    want = oracle_bip(oracle_mod, keys, offs)
    assert want[0] == 0
    g = gpu_bip(shock, keys, offs, bip_pool=cap)
    over = []
    for j in range(len(offs) - 1):
        lk = keys[int(offs[j]):int(offs[j + 1])]
        al, ar = _pool_adds(oracle_mod, lk, int(want[1][j]), int(want[2][j]))
        over.append(al > cap or ar > cap)
    over = np.array(over)
    print(f"[gpu] bip pool {cap}: {over.sum()} of {len(over)} leaves past it", flush=True)
    assert 0 < over.sum() < len(over)
    second = np.array([max(_pool_adds(oracle_mod, keys[int(offs[j]):int(offs[j + 1])], int(want[1][j]),
                                      int(want[2][j]))) > cap // 2 for j in range(len(offs) - 1)]) & ~over
    print(f"[gpu] bip pool {cap}: {second.sum()} leaves found by the second pass", flush=True)
    assert second.sum() > 0
    # every leaf past the first pass's pool (cap // 2) was searched again
    assert g[4]["second_pass_leaves"] == int(second.sum() + over.sum())
    assert g[0] == shock.SHOCK_ENOTFOUND
    assert (g[1][over] == MAX).all() and (g[2][over] == MAX).all()
    ok = ~over
    assert (g[1][ok] == want[1][ok]).all() and (g[2][ok] == want[2][ok]).all() and (g[3][ok] == want[3][ok]).all()
    # the default pool equals the oracle on the same batch; out-of-range pools are refused
    assert_same(gpu_bip(shock, keys, offs), want, "default pool")
    assert gpu_bip(shock, keys, offs, bip_pool=7169)[0] == shock.SHOCK_EINVAL


def test_bip_edges(shock):
    keys = splitmix64(3104, 3)
    offs = np.array([0, 0, 1, 3], np.uint64)
    rc, a, b, f, _ = gpu_bip(shock, keys, offs)
    assert rc == 0 and list(a[:2]) == [0, 0] and list(b[:2]) == [0, 0] and list(f[:2]) == [0, 0]
    rc, *_ = gpu_bip(shock, keys, offs, max_seed=(1 << 32) + 1)
    assert rc == shock.SHOCK_EINVAL
