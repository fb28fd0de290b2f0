"""The stored full-size oracle results (no GPU).

tests/golden/oracle_<name>.npz hold the oracle's seed and orientation for
every leaf of every full-size workload; the GPU tests compare against them.
These tests check that each file still belongs to its inputs and to the
current oracle, and use the files as what they also are: the oracle's
searches at production leaf sizes (24 to 64 keys, millions of seeds per
leaf), whose seed counts must follow ideal loop-free hashing (Section 5's
exact success probability per seed) just as the small-n statistical pins do.
"""
import math
import os

import numpy as np
import pytest

import theory as T
from workloads import inputs_digest, make_workload

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

FILES = [
    ("plain24", "plain24", "plain"),
    ("fixed40", "fixed40", "plain"),
    ("fixed48", "fixed48", "plain"),
    ("uneven32_56", "uneven32_56", "plain"),
    ("hard60", "hard60", "plain"),
    ("full64", "full64", "plain"),
    ("rf_fixed48", "fixed48", "rf"),
    ("rf_full64", "full64", "rf"),
]


def _load(name):
    path = os.path.join(GOLDEN, f"oracle_{name}.npz")
    assert os.path.exists(path), f"{path} is missing: run tests/golden/make_oracle_outputs.py"
    return np.load(path)


@pytest.mark.parametrize("name,workload,kind", FILES, ids=[f[0] for f in FILES])
def test_golden_belongs_to_inputs_and_oracle(oracle_mod, name, workload, kind):
    keys, offs = make_workload(workload)
    z = _load(name)
    L = len(offs) - 1
    assert str(z["inputs"]) == inputs_digest(keys, offs)
    assert str(z["kind"]) == kind
    seeds, orient = z["seeds"].astype(np.uint64), z["orient"]
    assert seeds.shape == (L,) and orient.shape == (L,)
    sizes = np.diff(offs).astype(np.uint64)
    short = sizes < 64
    assert ((orient[short] >> sizes[short]) == 0).all()  # no bits beyond a leaf's keys
    # re-run the oracle on the cheapest leaves (smallest seeds) and a few others
    order = np.argsort(seeds, kind="stable")
    pick = list(order[:6])
    if seeds.mean() < 1e5:
        pick += list(np.random.default_rng(7).choice(L, size=min(6, L), replace=False))
    for j in sorted(set(int(p) for p in pick)):
        sub = offs[j:j + 2]
        if kind == "plain":
            rc, s, f = oracle_mod.leaf_search(keys, sub)
            assert rc == 0 and (int(s[0]), int(f[0])) == (int(seeds[j]), int(orient[j])), j
        else:
            rc, s, r, f = oracle_mod.rf_leaf_search(keys, sub)
            assert rc == 0, j
            assert (int(s[0]), int(r[0]), int(f[0])) == (int(seeds[j]), int(z["rot"][j]), int(orient[j])), j


@pytest.mark.parametrize("name,workload", [(f[0], f[1]) for f in FILES if f[2] == "plain"],
                         ids=[f[0] for f in FILES if f[2] == "plain"])
def test_orientations_are_bijections(oracle_mod, name, workload):
    """The stored orientation makes x -> h_{f(x)}(x, s) a bijection (Section 4),
    on a sample of leaves of every file, evaluated slot by slot."""
    keys, offs = make_workload(workload)
    z = _load(name)
    L = len(offs) - 1
    for j in np.random.default_rng(11).choice(L, size=min(20, L), replace=False):
        leaf = keys[int(offs[j]):int(offs[j + 1])]
        h0, h1 = oracle_mod.leaf_slots(leaf, int(z["seeds"][j]))
        f = int(z["orient"][j])
        cells = sorted(int(h1[i]) if (f >> i) & 1 else int(h0[i]) for i in range(len(leaf)))
        assert cells == list(range(len(leaf))), j


@pytest.mark.parametrize("name,workload", [(f[0], f[1]) for f in FILES if f[2] == "plain"],
                         ids=[f[0] for f in FILES if f[2] == "plain"])
def test_seed_counts_match_ideal_hashing_at_full_size(name, workload):
    """Per leaf size with at least 200 leaves: the mean of s*+1 lies within 5
    standard errors of 1/p'_n, and the fraction of leaves needing more than
    the median of the geometric law lies within 5 standard errors of 1/2."""
    keys, offs = make_workload(workload)
    z = _load(name)
    seeds = z["seeds"].astype(np.float64)
    sizes = np.diff(offs).astype(np.int64)
    checked = 0
    for n in np.unique(sizes):
        sel = sizes == n
        m = int(sel.sum())
        if m < 200:
            continue
        p = float(T.p_accept(int(n)))
        mu, sd = 1 / p, math.sqrt(1 - p) / p
        mean = float((seeds[sel] + 1).mean())
        assert abs(mean - mu) < 5 * sd / math.sqrt(m), (int(n), mean, mu)
        # P(s* + 1 > k) = (1 - p)^k; its median
        k_med = math.log(0.5) / math.log1p(-p)
        frac = float(((seeds[sel] + 1) > k_med).mean())
        assert abs(frac - 0.5) < 5 * 0.5 / math.sqrt(m), (int(n), frac)
        checked += 1
    assert checked > 0 or name == "full64"
