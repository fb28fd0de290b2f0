"""Randomised GPU parity: leaf-size mixes and launch options drawn from a
fixed-seed generator, each case compared leaf by leaf with the oracle for the
plain search, rotation fitting and bipartite ShockHash.  The fixed cases in
the other files pin chosen option sets; these cover combinations nobody
picked (claim sizes against worker counts, team mode against waves per
workgroup, resume points, partial-hash periods) on batches with empty,
single-key and ragged leaves."""
import numpy as np
import pytest

from workloads import splitmix64

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

MAX_SEED = 1 << 22
CASES = 24


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


def _case(i):
    rng = np.random.default_rng(9000 + i)
    L = int(rng.integers(1, 260))
    sizes = rng.integers(0, 33, L)
    small = rng.random(L) < 0.08  # some empty, single-key and tiny leaves
    sizes[small] = rng.integers(0, 4, int(small.sum()))
    wide = rng.random(L) < 0.08  # and some above 32 keys (64-bit coverage masks)
    sizes[wide] = rng.integers(33, 45, int(wide.sum()))
    # a few edge sizes at random places
    for v in (0, 1, 2, 36):
        sizes[int(rng.integers(L))] = v
    offs = np.zeros(L + 1, np.uint64)
    np.cumsum(sizes.astype(np.uint64), out=offs[1:])
    keys = splitmix64(9100 + i, int(offs[-1]))
    opts = dict(
        spl=int(rng.choice([0, 1, 2, 4])),
        block_iters=int(rng.choice([0, 1, 2, 5, 16])),
        waves_per_wg=int(rng.choice([0, 1, 2, 4, 8, 16])),
        workers=int(rng.choice([0, 1, 7, 64, 333, 2048])),
        team=int(rng.choice([0, 1, 2])),
    )
    start = int(rng.choice([0, 0, 0, 1000]))
    return keys, offs, opts, start, int(rng.choice([0, 1, 8])), rng


def _oracle(oracle_mod, fn, keys, offs, **kw):
    parts = oracle_mod.parallel(fn, keys, offs, threads=16, **kw)
    rc = min(p[0] for p in parts)
    return (rc, *[np.concatenate([p[k] for p in parts]) for k in range(1, len(parts[0]))])


@pytest.mark.parametrize("i", range(CASES))
def test_random_plain(shock, oracle_mod, i):
    keys, offs, opts, start, _, _ = _case(i)
    print(f"[gpu] random plain case {i}: L={len(offs) - 1} start={start} {opts}", flush=True)
    want = _oracle(oracle_mod, oracle_mod.leaf_search, keys, offs, start_seed=start, max_seed=MAX_SEED)
    rc, s, f = shock.leaf_search(_dev(keys), _dev(offs), start_seed=start, max_seed=MAX_SEED, **opts)
    torch.cuda.synchronize()
    assert rc == want[0]
    assert (_host(s) == want[1]).all() and (_host(f) == want[2]).all()


@pytest.mark.parametrize("i", range(CASES))
def test_random_rotation_fitting(shock, oracle_mod, i):
    keys, offs, opts, start, pk, _ = _case(i)
    opts = {k: v for k, v in opts.items() if k != "spl"}  # rotation fitting has its own seeds per lane
    print(f"[gpu] random rf case {i}: L={len(offs) - 1} start={start} partial_k={pk} {opts}", flush=True)
    want = _oracle(oracle_mod, oracle_mod.rf_leaf_search, keys, offs, start_seed=start, max_seed=MAX_SEED,
                   partial_k=pk)
    rc, s, r, f = shock.rf_leaf_search(_dev(keys), _dev(offs), start_seed=start, max_seed=MAX_SEED, partial_k=pk,
                                       **opts)
    torch.cuda.synchronize()
    assert rc == want[0]
    assert (_host(s) == want[1]).all() and (r.cpu().numpy() == want[2].astype(np.int64)).all()
    assert (_host(f) == want[3]).all()


@pytest.mark.parametrize("i", range(CASES))
def test_random_bipartite(shock, oracle_mod, i):
    keys, offs, opts, _, _, _ = _case(i)
    workers = opts["workers"]
    print(f"[gpu] random bip case {i}: L={len(offs) - 1} workers={workers}", flush=True)
    want = _oracle(oracle_mod, oracle_mod.bip_leaf_search, keys, offs, max_seed=MAX_SEED)
    rc, a, b, f, _ = shock.bip_leaf_search(_dev(keys), _dev(offs), workers=workers, max_seed=MAX_SEED)
    torch.cuda.synchronize()
    assert rc == want[0]
    assert (_host(a) == want[1]).all() and (_host(b) == want[2]).all() and (_host(f) == want[3]).all()
