"""The search that allocates nothing (shock_leaf_search_noalloc), through the C ABI.

It must give the same seeds and orientations as shock_leaf_search_ex in
persistent mode, on two calls in a row, the second with a smaller batch (the
fixed per-GPU scratch array keeps the first call's contents), reject batches
beyond its stated limits before launching anything, and report the batch's
own errors.
"""
import numpy as np
import pytest

from workloads import fixed_leaves, uneven_leaves

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


def _both(shock, keys, offs, **opts):
    """(rc, seeds, orient) of the allocating search and of the no-alloc one."""
    k, o = _dev(keys), _dev(offs)
    L = len(offs) - 1
    print(f"[gpu] no-alloc vs allocating search: L={L} opts={opts}", flush=True)
    rc_a, s_a, f_a = shock.leaf_search(k, o, **opts)
    torch.cuda.synchronize()
    s_b = torch.full((L,), -7, dtype=torch.int64, device="cuda")
    f_b = torch.full((L,), -7, dtype=torch.int64, device="cuda")
    rc_b = shock.leaf_search_noalloc(k, o, s_b, f_b, **opts)
    torch.cuda.synchronize()
    return (rc_a, _host(s_a), _host(f_a)), (rc_b, _host(s_b), _host(f_b))


def _same(a, b, what):
    assert a[0] == b[0] == 0, (what, a[0], b[0])
    bad = np.nonzero((a[1] != b[1]) | (a[2] != b[2]))[0]
    assert bad.size == 0, f"{what}: {bad.size} leaves differ, first {bad[:5]}"


def test_two_calls_second_smaller(shock):
    keys, offs = uneven_leaves(3000, 24, 44, 901, 902)
    a, b = _both(shock, keys, offs)
    _same(a, b, "first call, 3000 uneven leaves")
    keys2, offs2 = fixed_leaves(257, 40, 903)
    a2, b2 = _both(shock, keys2, offs2)
    _same(a2, b2, "second call, 257 leaves of 40 keys")


def test_launch_options_and_oracle(shock, oracle_mod):
    keys, offs = fixed_leaves(200, 32, 904)
    rc_o, s_o, f_o = oracle_mod.leaf_search(keys, offs)
    for opts in (dict(), dict(workers=64, spl=1, waves_per_wg=2), dict(team=1, spl=4)):
        a, b = _both(shock, keys, offs, **opts)
        _same(a, b, f"opts {opts}")
        assert (b[1] == s_o).all() and (b[2] == f_o).all(), opts


def test_limits_rejected_before_launch(shock):
    cap = shock.SHOCK_NOALLOC_MAX_LEAVES
    L = cap + 1
    offs = np.arange(L + 1, dtype=np.uint64) * np.uint64(2)
    keys = np.arange(2 * L, dtype=np.uint64)
    s = torch.full((L,), -7, dtype=torch.int64, device="cuda")
    f = torch.full((L,), -7, dtype=torch.int64, device="cuda")
    print(f"[gpu] no-alloc limit: L={L}", flush=True)
    rc = shock.leaf_search_noalloc(_dev(keys), _dev(offs), s, f)
    assert rc == shock.SHOCK_EINVAL
    assert int((s != -7).sum()) == 0 and int((f != -7).sum()) == 0
    small_k, small_o = fixed_leaves(4, 8, 905)
    s4 = torch.zeros(4, dtype=torch.int64, device="cuda")
    f4 = torch.zeros(4, dtype=torch.int64, device="cuda")
    assert shock.leaf_search_noalloc(_dev(small_k), _dev(small_o), s4, f4,
                                     workers=shock.SHOCK_NOALLOC_MAX_WORKERS + 16) == shock.SHOCK_EINVAL
    assert shock.leaf_search_noalloc(_dev(small_k), _dev(small_o), s4, f4,
                                     mode=shock.SHOCK_MODE_PLAIN_PER_LEAF) == shock.SHOCK_EINVAL


def test_batch_errors(shock):
    # a leaf of 65 keys, and offsets reaching past the keys buffer: EINVAL, outputs untouched
    keys, _ = fixed_leaves(1, 65, 906)
    offs = np.array([0, 65], dtype=np.uint64)
    s = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    f = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    print("[gpu] no-alloc error paths", flush=True)
    assert shock.leaf_search_noalloc(_dev(keys), _dev(offs), s, f) == shock.SHOCK_EINVAL
    keys, _ = fixed_leaves(2, 10, 907)
    offs = np.array([0, 10, 30], dtype=np.uint64)
    s2 = torch.full((2,), -7, dtype=torch.int64, device="cuda")
    f2 = torch.full((2,), -7, dtype=torch.int64, device="cuda")
    assert shock.leaf_search_noalloc(_dev(keys), _dev(offs), s2, f2) == shock.SHOCK_EINVAL
    assert int((s2 != -7).sum()) == 0
    # a repeated key with check_dups
    keys, offs = fixed_leaves(3, 12, 908)
    keys[13] = keys[14]
    s3 = torch.full((3,), -7, dtype=torch.int64, device="cuda")
    f3 = torch.full((3,), -7, dtype=torch.int64, device="cuda")
    assert shock.leaf_search_noalloc(_dev(keys), _dev(offs), s3, f3, check_dups=True) == shock.SHOCK_EDUPKEY
    # a cap no leaf reaches: ENOTFOUND with the marker
    keys, offs = fixed_leaves(5, 40, 909)
    s5 = torch.zeros(5, dtype=torch.int64, device="cuda")
    f5 = torch.zeros(5, dtype=torch.int64, device="cuda")
    assert shock.leaf_search_noalloc(_dev(keys), _dev(offs), s5, f5, max_seed=3) == shock.SHOCK_ENOTFOUND
    assert (_host(s5) == np.uint64(0xFFFFFFFFFFFFFFFF)).any()
