"""Randomised GPU parity of the flat MPHF: key counts, bucket sizes, leaf
targets and bounds, leaf kinds (plain, rotation fitting, bipartite) and
retrievals (ribbon, XOR) drawn from a fixed-seed generator.  Each case
compares every stored part and every key's position with the oracle's
build, or, where the parameters leave some bucket without a splitting seed,
the error status."""
import numpy as np
import pytest

from workloads import splitmix64

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CASES = 12
RIBBON, XOR = 0, 1


@pytest.fixture(scope="module")
def shock():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09561_amd as shock
    shock.lib()
    return shock


def _case(i):
    rng = np.random.default_rng(9500 + i)
    N = int(rng.choice([0, 1, 2, int(rng.integers(3, 300)), int(rng.integers(300, 30000))], p=[.05, .05, .05, .25, .6]))
    kind = str(rng.choice(["plain", "rf", "bip"]))
    leaf_target = int(rng.integers(4, 25))
    leaf_max = int(min(36, leaf_target + int(rng.integers(4, 16))))
    params = dict(bucket_size=int(rng.integers(40, 2500)), leaf_target=leaf_target, leaf_max=leaf_max)
    retrieval = int(rng.choice([RIBBON, XOR]))
    return N, kind, params, retrieval


@pytest.mark.parametrize("i", range(CASES))
def test_random_mphf(shock, oracle_mod, i):
    N, kind, params, retrieval = _case(i)
    keys = splitmix64(9600 + i, N)
    print(f"[gpu] random mphf case {i}: N={N} {kind} {params} retrieval={retrieval}", flush=True)
    rc_o, lay = oracle_mod.mphf_build(keys, rf=kind == "rf", bip=kind == "bip", retrieval=retrieval, **params)
    k = torch.from_numpy(keys.view(np.int64)).cuda() if N else torch.zeros(0, dtype=torch.int64, device="cuda")
    try:
        m = shock.MPHF(k, rotation_fitting=kind == "rf", bipartite=kind == "bip", retrieval=retrieval, **params)
    except shock.ShockError as e:
        assert rc_o != 0 and e.status == rc_o, (rc_o, e.status)
        return
    try:
        torch.cuda.synchronize()
        assert rc_o == 0
        ex = m.export()
        for f in ("bucket_offset", "leaf_base", "sigma", "leaf_sizes", "seeds"):
            assert (ex[f] == lay[f]).all(), f
        assert ex["retrieval"] == lay["retrieval"]
        if retrieval == XOR:
            assert ex["rho"] == lay["rho"] and (ex["z"] == lay["z"]).all()
        else:
            assert (ex["rseed"] == lay["rseed"]).all() and (ex["rbit_offset"] == lay["rbit_offset"]).all()
            assert (ex["z"] == lay["z"]).all()
        if N:
            pos = m.query(k).cpu().numpy().view(np.uint64)
            assert (pos == lay["positions"]).all()
            assert sorted(pos.tolist()) == list(range(N))
    finally:
        m.close()


@pytest.mark.parametrize("N,want", [(2048, 0), (2050, -1)])
def test_leaves_per_bucket_limit(shock, oracle_mod, N, want):
    """One bucket of 1024 leaves builds and equals the oracle; 1025 is
    refused by both."""
    keys = splitmix64(1205, 2050)[:N]
    params = dict(bucket_size=4096, leaf_target=2, leaf_max=8)
    rc_o, lay = oracle_mod.mphf_build(keys, **params)
    assert rc_o == want
    k = torch.from_numpy(keys.view(np.int64)).cuda()
    print(f"[gpu] mphf leaves-per-bucket limit N={N}", flush=True)
    if want != 0:
        with pytest.raises(shock.ShockError) as e:
            shock.MPHF(k, **params)
        assert e.value.status == want
        return
    m = shock.MPHF(k, **params)
    try:
        ex = m.export()
        assert (ex["seeds"] == lay["seeds"]).all() and (ex["z"] == lay["z"]).all()
        assert (m.query(k).cpu().numpy().view(np.uint64) == lay["positions"]).all()
    finally:
        m.close()


def test_failed_split_after_a_larger_build(shock, oracle_mod):
    """A build whose buckets cannot all be split (13700 keys, buckets of 2406,
    leaves of at most 29) right after a larger build on the same thread: the
    cached scratch then holds the larger build's leaf offsets.  The failing
    bucket's leaves are still written (empty), so the kernels queued behind
    the split read none of those offsets, and the build returns the oracle's
    status."""
    big = splitmix64(9700, 300000)
    m = shock.MPHF(torch.from_numpy(big.view(np.int64)).cuda())
    torch.cuda.synchronize()
    m.close()
    keys = splitmix64(9602, 13700)
    params = dict(bucket_size=2406, leaf_target=24, leaf_max=29)
    print(f"[gpu] failed split after a larger build: {params}", flush=True)
    rc_o, _ = oracle_mod.mphf_build(keys, rf=True, retrieval=RIBBON, **params)
    assert rc_o == shock.SHOCK_ENOTFOUND
    with pytest.raises(shock.ShockError) as e:
        shock.MPHF(torch.from_numpy(keys.view(np.int64)).cuda(), rotation_fitting=True, retrieval=RIBBON, **params)
    assert e.value.status == shock.SHOCK_ENOTFOUND
    torch.cuda.synchronize()
