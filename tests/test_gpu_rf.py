"""GPU parity of rotation fitting (Section 4, "Rotation Fitting"; partial hash
calculation, Appendix A.2): the HIP library against the CPU oracle, through
the C ABI, bit-exact on (seed, rotation, orientation) per leaf."""
import numpy as np
import pytest

from workloads import fixed_leaves, splitmix64

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


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


def gpu_rf(shock, keys, offsets, **opts):
    print(f"[gpu] rf L={len(offsets) - 1} opts={opts}", flush=True)
    k = _dev(keys) if len(keys) else torch.zeros(1, dtype=torch.int64, device="cuda")
    rc, s, r, f = shock.rf_leaf_search(k, _dev(offsets), **opts)
    torch.cuda.synchronize()
    return rc, _host(s), r.cpu().numpy().astype(np.uint32), _host(f)


def oracle_rf(oracle_mod, keys, offsets, **kw):
    parts = oracle_mod.parallel(oracle_mod.rf_leaf_search, keys, offsets, threads=16, **kw)
    rc = min(p[0] for p in parts) if parts else 0
    cat = [np.concatenate([p[i] for p in parts]) if parts else np.zeros(0, np.uint64) for i in (1, 2, 3)]
    return (rc, *cat)


def assert_same(g, o, what=""):
    rc_g, s_g, r_g, f_g = g
    rc_o, s_o, r_o, f_o = o
    bad = np.nonzero((s_g != s_o) | (r_g != r_o.astype(np.uint32)) | (f_g != f_o))[0]
    assert bad.size == 0, (f"{what}: {bad.size} leaves differ, first {bad[:4]}: gpu {s_g[bad[:4]]}/{r_g[bad[:4]]} "
                           f"oracle {s_o[bad[:4]]}/{r_o[bad[:4]]}")
    assert rc_g == rc_o, what


@pytest.mark.parametrize("n,L", [(2, 300), (3, 300), (5, 300), (8, 300), (16, 300), (24, 200), (31, 100),
                                 (32, 100), (33, 60), (40, 40), (48, 16)])
def test_rf_fixed_n_matches_oracle(shock, oracle_mod, n, L):
    """Default partial hashing: k = 1 up to 32 keys, k = 8 above."""
    keys, offs = fixed_leaves(L, n, 20_000 + n)
    assert_same(gpu_rf(shock, keys, offs), oracle_rf(oracle_mod, keys, offs), f"n={n}")


@pytest.mark.parametrize("n,k", [(24, 8), (20, 8), (40, 1), (36, 1)])
def test_rf_explicit_partial_k(shock, oracle_mod, n, k):
    keys, offs = fixed_leaves(40, n, 21_000 + n + k)
    g = gpu_rf(shock, keys, offs, partial_k=k)
    assert_same(g, oracle_rf(oracle_mod, keys, offs, partial_k=k), f"n={n} k={k}")


def test_rf_uneven_batch(shock, oracle_mod):
    rng = np.random.default_rng(9)
    sizes = np.repeat(np.arange(0, 45), 2)
    rng.shuffle(sizes)
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offs[1:])
    keys = splitmix64(91, int(offs[-1]))
    assert_same(gpu_rf(shock, keys, offs), oracle_rf(oracle_mod, keys, offs), "uneven")


LAUNCHES = [
    dict(mode=1),
    dict(mode=1, block_iters=3),
    dict(mode=2, block_iters=1, workers=64),
    dict(mode=2, block_iters=5, workers=4096, waves_per_wg=2),
    dict(mode=2, workers=8, waves_per_wg=8),
    dict(mode=2, team=1, waves_per_wg=4),
    dict(mode=2, team=2, waves_per_wg=16, workers=128),
]


@pytest.mark.parametrize("opts", LAUNCHES, ids=[str(o) for o in LAUNCHES])
def test_rf_launch_invariance(shock, oracle_mod, opts):
    """Any launch form and claim size gives the same result (races in claims,
    helpers and the encoded minimum would show up here)."""
    rng = np.random.default_rng(11)
    sizes = rng.integers(26, 42, size=48)
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offs[1:])
    keys = splitmix64(92, int(offs[-1]))
    assert_same(gpu_rf(shock, keys, offs, **opts), oracle_rf(oracle_mod, keys, offs), str(opts))


@pytest.mark.parametrize("start", [0, 5, 13, 1000, 12345])
def test_rf_start_seed_unaligned(shock, oracle_mod, start):
    """Partial hashing groups seeds by s - s mod 8 whatever the start seed."""
    keys, offs = fixed_leaves(24, 36, 22_000 + start)
    g = gpu_rf(shock, keys, offs, start_seed=start)
    assert_same(g, oracle_rf(oracle_mod, keys, offs, start_seed=start), f"start={start}")
    assert (g[1] >= start).all()


def test_rf_max_seed_and_resume(shock, oracle_mod):
    keys, offs = fixed_leaves(30, 30, 93)
    full = gpu_rf(shock, keys, offs)
    cap = int(np.median(full[1]))
    g = gpu_rf(shock, keys, offs, max_seed=cap)
    o = oracle_rf(oracle_mod, keys, offs, max_seed=cap)
    assert g[0] == shock.SHOCK_ENOTFOUND
    assert_same(g, o, "capped")
    miss = g[1] == np.uint64(shock.NOT_FOUND_SEED)
    assert miss.any() and (~miss).any()
    assert (g[2][miss] == 0).all() and (g[3][miss] == 0).all()
    # resuming at the cap finds the leaves that were missing
    r = gpu_rf(shock, keys, offs, start_seed=cap)
    assert (r[1][miss] == full[1][miss]).all() and (r[2][miss] == full[2][miss]).all()


def test_rf_edge_leaves(shock):
    offs = np.array([0, 0, 1, 1, 3], dtype=np.uint64)
    keys = splitmix64(94, 3)
    rc, s, r, f = gpu_rf(shock, keys, offs, start_seed=7)
    assert rc == 0
    assert list(s[:3]) == [7, 7, 7] and list(r[:3]) == [0, 0, 0] and list(f[:3]) == [0, 0, 0]
    empty = gpu_rf(shock, np.zeros(0, np.uint64), np.zeros(1, np.uint64))
    assert empty[0] == 0 and empty[1].size == 0


def test_rf_n64_window(shock, oracle_mod):
    """64-key leaves are too slow for a whole oracle search; the oracle
    restarted a little below the GPU's seed must land on the same candidate."""
    keys, offs = fixed_leaves(4, 64, 95)
    g = gpu_rf(shock, keys, offs)
    assert g[0] == 0
    for j in range(4):
        s = int(g[1][j])
        o = oracle_mod.rf_leaf_search(keys, offs[j:j + 2], start_seed=max(0, s - 600))
        assert (int(o[1][0]), int(o[2][0]), int(o[3][0])) == (s, int(g[2][j]), int(g[3][j])), j


def test_rf_rejects_bad_options(shock):
    keys, offs = fixed_leaves(2, 10, 96)
    rc = gpu_rf(shock, keys, offs, partial_k=3)[0]
    assert rc == shock.SHOCK_EINVAL
    rc = gpu_rf(shock, keys, offs, max_seed=(1 << 57) + 1)[0]
    assert rc == shock.SHOCK_EINVAL


def test_rf_context_async_matches_sync(shock, oracle_mod):
    keys, offs = fixed_leaves(64, 34, 97)
    want = gpu_rf(shock, keys, offs)
    ctx = shock.SearchContext(256)
    try:
        k, o = _dev(keys), _dev(offs)
        s = torch.empty(64, dtype=torch.int64, device="cuda")
        f = torch.empty(64, dtype=torch.int64, device="cuda")
        r = torch.empty(64, dtype=torch.int32, device="cuda")
        print("[gpu] rf context", flush=True)
        assert ctx.rf_search_async(k, o, s, r, f, leaf_size_hint=34) == 0
        rc, st = ctx.wait()
        assert rc == 0
        assert (_host(s) == want[1]).all() and (r.cpu().numpy().astype(np.uint32) == want[2]).all()
        assert (_host(f) == want[3]).all()
    finally:
        ctx.close()
