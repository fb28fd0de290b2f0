"""Full-size workloads on the GPU, in the launch form the benchmark uses.

Checks every leaf with the oracle at its claimed seed (the seed qualifies,
the orientation is the canonical one, and no seed in a window below it
qualifies), re-runs the whole oracle search on a fixed random sample of
leaves (bit-exact), and checks that the mean seed count matches ideal
loop-free hashing (a property that holds at any size).
"""
import math

import numpy as np
import pytest

import theory as T
from workloads import WORKLOADS, make_workload

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

THREADS = 16


@pytest.fixture(scope="module")
def shock():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09561_amd as shock
    shock.lib()
    return shock


CASES = [
    # workload, launch options, verify window, sampled leaves for the full oracle search
    ("plain24", dict(mode=1), 256, 64),
    ("fixed40", dict(), 64, 48),
    ("fixed48", dict(), 32, 24),
    ("uneven32_56", dict(), 16, 16),
    ("hard60", dict(), 16, 4),
]


@pytest.mark.parametrize("name,opts,window,sample", CASES, ids=[c[0] for c in CASES])
def test_full_workload(shock, oracle_mod, name, opts, window, sample):
    keys, offs = make_workload(name)
    L = len(offs) - 1
    print(f"[gpu] full workload {name}: {L} leaves, opts {opts}", flush=True)
    k = torch.from_numpy(keys.view(np.int64)).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    rc, s_d, f_d = shock.leaf_search(k, o, **opts)
    torch.cuda.synchronize()
    assert rc == shock.SHOCK_OK
    seeds = s_d.cpu().numpy().view(np.uint64)
    orient = f_d.cpu().numpy().view(np.uint64)
    sizes = np.diff(offs).astype(np.int64)
    short = sizes < 64
    assert ((orient[short] >> sizes[short].astype(np.uint64)) == 0).all()  # no bits beyond n

    # every leaf: claimed seed qualifies, canonical orientation, window below
    flags = np.concatenate(oracle_mod.parallel(oracle_mod.verify, keys, offs, seeds, orient,
                                               threads=THREADS, window=window))
    bad = np.nonzero(flags)[0]
    assert bad.size == 0, f"{bad.size} leaves fail verification, first {bad[:5]} flags {flags[bad[:5]]}"

    # a fixed random sample: the whole oracle search, bit-exact
    rng = np.random.default_rng(12345)
    pick = np.sort(rng.choice(L, size=min(sample, L), replace=False))
    from concurrent.futures import ThreadPoolExecutor

    def one(j):
        sub = offs[j:j + 2]
        return oracle_mod.leaf_search(keys, sub)

    with ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(one, pick))
    for j, (rc_o, s_o, f_o) in zip(pick, res):
        assert rc_o == 0
        assert int(s_o[0]) == int(seeds[j]) and int(f_o[0]) == int(orient[j]), j

    # statistics: mean of s*+1 per leaf size matches 1/p'_n within 6 standard errors
    for n in np.unique(sizes):
        sel = sizes == n
        m = int(sel.sum())
        if m < 200:
            continue
        p = float(T.p_accept(int(n)))
        mu, sd = 1 / p, math.sqrt(1 - p) / p
        mean = float((seeds[sel].astype(np.float64) + 1).mean())
        assert abs(mean - mu) < 6 * sd / math.sqrt(m), (name, int(n), mean, mu)
