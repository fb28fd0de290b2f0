"""Full-size workloads on the GPU, in the launch form the benchmark uses.

Every leaf of every workload is compared bit for bit (seed, orientation and,
for rotation fitting, rotation) with the oracle's full search, stored in
tests/golden/oracle_<name>.npz by tests/golden/make_oracle_outputs.py (which
calls only the oracle and the input generators).  The inputs are regenerated
here and checked against the digest stored with the results.  The mean seed
count per leaf size is also checked against ideal loop-free hashing, a
property that holds at any size.
"""
import math
import os

import numpy as np
import pytest

import theory as T
from workloads import inputs_digest, make_workload

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def shock():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09561_amd as shock
    shock.lib()
    return shock


def load_golden(name, keys, offs):
    z = np.load(os.path.join(GOLDEN, f"oracle_{name}.npz"))
    assert str(z["inputs"]) == inputs_digest(keys, offs), f"{name}: golden file is for other inputs"
    return z


def first_diffs(a, b, k=5):
    bad = np.nonzero(a != b)[0]
    return bad.size, bad[:k]


CASES = [
    # golden file, workload, search, launch options
    ("plain24", "plain24", "plain", dict(mode=1)),
    ("fixed40", "fixed40", "plain", dict()),
    ("fixed48", "fixed48", "plain", dict()),
    ("uneven32_56", "uneven32_56", "plain", dict()),
    ("hard60", "hard60", "plain", dict()),
    ("full64", "full64", "plain", dict()),
    ("rf_fixed48", "fixed48", "rf", dict()),
    ("rf_full64", "full64", "rf", dict()),
]


@pytest.mark.parametrize("name,workload,kind,opts", CASES, ids=[c[0] for c in CASES])
def test_full_workload_every_leaf(shock, name, workload, kind, opts):
    keys, offs = make_workload(workload)
    gold = load_golden(name, keys, offs)
    L = len(offs) - 1
    print(f"[gpu] full workload {name}: {L} leaves, {kind}, opts {opts}", flush=True)
    k = torch.from_numpy(keys.view(np.int64)).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    if kind == "plain":
        rc, s_d, f_d = shock.leaf_search(k, o, **opts)
    else:
        rc, s_d, r_d, f_d = shock.rf_leaf_search(k, o, **opts)
    torch.cuda.synchronize()
    assert rc == shock.SHOCK_OK
    seeds = s_d.cpu().numpy().view(np.uint64)
    orient = f_d.cpu().numpy().view(np.uint64)
    n_bad, first = first_diffs(seeds, gold["seeds"].astype(np.uint64))
    assert n_bad == 0, f"{name}: {n_bad} seeds differ, first leaves {first}"
    n_bad, first = first_diffs(orient, gold["orient"])
    assert n_bad == 0, f"{name}: {n_bad} orientations differ, first leaves {first}"
    if kind == "rf":
        rot = r_d.cpu().numpy().astype(np.uint32)
        n_bad, first = first_diffs(rot, gold["rot"])
        assert n_bad == 0, f"{name}: {n_bad} rotations differ, first leaves {first}"
        return

    # statistics: mean of s*+1 per leaf size matches 1/p'_n within 6 standard errors
    sizes = np.diff(offs).astype(np.int64)
    for n in np.unique(sizes):
        sel = sizes == n
        m = int(sel.sum())
        if m < 200:
            continue
        p = float(T.p_accept(int(n)))
        mu, sd = 1 / p, math.sqrt(1 - p) / p
        mean = float((seeds[sel].astype(np.float64) + 1).mean())
        assert abs(mean - mu) < 6 * sd / math.sqrt(m), (name, int(n), mean, mu)
