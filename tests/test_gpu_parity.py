"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Bit-exact comparison of (seed, orientation) per leaf on seeded inputs, at
sizes the oracle finishes in seconds (several blocks, ragged tails, uneven
leaf sizes), plus launch-configuration invariance (the race test for block
claiming and work stealing), edge cases and error paths.
"""
import ctypes
import os

import numpy as np
import pytest

from workloads import fixed_leaves, make_workload, splitmix64, uneven_leaves

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


def gpu_search(shock, keys, offsets, **opts):
    print(f"[gpu] L={len(offsets) - 1} opts={opts}", flush=True)
    k = _dev(keys) if len(keys) else torch.zeros(1, dtype=torch.int64, device="cuda")
    rc, s, f = shock.leaf_search(k, _dev(offsets), **opts)
    torch.cuda.synchronize()
    return rc, _host(s), _host(f)


def assert_same(a, b, what=""):
    rc_a, s_a, f_a = a
    rc_b, s_b, f_b = b
    bad = np.nonzero((s_a != s_b) | (f_a != f_b))[0]
    assert bad.size == 0, f"{what}: {bad.size} leaves differ, first {bad[:5]}: gpu {s_a[bad[:5]]} oracle {s_b[bad[:5]]}"
    assert rc_a == rc_b, what


@pytest.mark.parametrize("n", [2, 3, 5, 8, 13, 16, 24, 31, 32, 33])
def test_fixed_n_matches_oracle(shock, oracle_mod, n):
    L = 300 if n <= 24 else 80
    keys, offs = fixed_leaves(L, n, 10_000 + n)
    g = gpu_search(shock, keys, offs)
    o = oracle_mod.leaf_search(keys, offs)
    assert o[0] == 0
    assert_same(g, o, f"n={n}")


def test_uneven_batch_matches_oracle(shock, oracle_mod):
    # every size 0..40 several times, shuffled, so blocks straddle many tails
    rng = np.random.default_rng(5)
    sizes = np.repeat(np.arange(0, 41), 3)
    rng.shuffle(sizes)
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offs[1:])
    keys = splitmix64(77, int(offs[-1]))
    g = gpu_search(shock, keys, offs)
    o = oracle_mod.parallel(oracle_mod.leaf_search, keys, offs)
    o_s = np.concatenate([r[1] for r in o])
    o_f = np.concatenate([r[2] for r in o])
    assert_same(g, (0, o_s, o_f), "uneven")


def test_large_leaves_sample_matches_oracle(shock, oracle_mod):
    # n in 41..56: a few leaves each, the oracle needs ~1 s per leaf at n = 56
    sizes = np.array([41, 44, 47, 48, 48, 50, 52, 53, 56], dtype=np.uint64)
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offs[1:])
    keys = splitmix64(4242, int(offs[-1]))
    g = gpu_search(shock, keys, offs)
    o = oracle_mod.parallel(oracle_mod.leaf_search, keys, offs, threads=len(sizes))
    o_s = np.concatenate([r[1] for r in o])
    o_f = np.concatenate([r[2] for r in o])
    assert_same(g, (0, o_s, o_f), "large")


LAUNCH_CONFIGS = [
    dict(spl=1, block_iters=1, waves_per_wg=1, workers=3),
    dict(spl=2, block_iters=3, waves_per_wg=4, workers=64),
    dict(spl=4, block_iters=1, waves_per_wg=16, workers=256),
    dict(spl=2, block_iters=64, waves_per_wg=2),
    dict(spl=1, block_iters=2, waves_per_wg=8, workers=2048),
    dict(mode=1, spl=2, block_iters=1),
    dict(mode=1, spl=4, block_iters=2, workers=512),
    dict(team=2, waves_per_wg=4, block_iters=2),
    dict(team=2, waves_per_wg=16, workers=64, block_iters=1),
]


@pytest.mark.parametrize("cfg", LAUNCH_CONFIGS, ids=[str(i) for i in range(len(LAUNCH_CONFIGS))])
def test_launch_configuration_invariance(shock, oracle_mod, cfg):
    """Block size, seeds per lane, waves per workgroup, worker count and launch
    mode change only how seeds are shared out, never the result."""
    keys, offs = uneven_leaves(150, 20, 36, 31337, 31338)
    o = oracle_mod.parallel(oracle_mod.leaf_search, keys, offs)
    o_s = np.concatenate([r[1] for r in o])
    o_f = np.concatenate([r[2] for r in o])
    g = gpu_search(shock, keys, offs, **cfg)
    assert_same(g, (0, o_s, o_f), str(cfg))


def test_hard_leaves_many_helpers(shock, oracle_mod):
    """Fewer leaves than workers: most workers help; the smallest seed must
    still win whatever block finishes first."""
    keys, offs = fixed_leaves(6, 44, 999)
    o = oracle_mod.parallel(oracle_mod.leaf_search, keys, offs, threads=6)
    o_s = np.concatenate([r[1] for r in o])
    o_f = np.concatenate([r[2] for r in o])
    for cfg in (dict(block_iters=1), dict(block_iters=8), dict(spl=4, block_iters=1, workers=4096)):
        g = gpu_search(shock, keys, offs, **cfg)
        assert_same(g, (0, o_s, o_f), str(cfg))


def test_start_seed_and_cap(shock, oracle_mod):
    keys, offs = fixed_leaves(40, 20, 555)
    rc, s, f = oracle_mod.leaf_search(keys, offs)
    assert rc == 0
    # resume from a midpoint: oracle and GPU agree
    start = int(np.median(s))
    o = oracle_mod.leaf_search(keys, offs, start_seed=start)
    g = gpu_search(shock, keys, offs, start_seed=start)
    assert_same(g, o, "resume")
    # a cap below some leaves' answers: those leaves report UINT64_MAX / 0
    cap = int(np.percentile(s, 40))
    o = oracle_mod.leaf_search(keys, offs, max_seed=cap)
    assert o[0] == oracle_mod.ENOTFOUND
    g = gpu_search(shock, keys, offs, max_seed=cap)
    assert g[0] == shock.SHOCK_ENOTFOUND
    assert_same(g, o, "cap")


def test_edge_leaves(shock, oracle_mod):
    # empty leaves, single keys, pairs, and a full 64-key leaf
    sizes = [0, 1, 2, 0, 1, 3, 64, 0]
    offs = np.zeros(len(sizes) + 1, dtype=np.uint64)
    np.cumsum(np.array(sizes, dtype=np.uint64), out=offs[1:])
    keys = splitmix64(2024, int(offs[-1]))
    g = gpu_search(shock, keys, offs)
    assert g[0] == 0
    # every leaf, the 64-key one included (its answer is about 8.9e6 seeds
    # in: a few seconds of oracle time), against the full oracle search
    o = oracle_mod.leaf_search(keys, offs)
    assert_same(g, o, "edge leaves")
    # and under another launch form
    g2 = gpu_search(shock, keys, offs, spl=1, block_iters=1, workers=128)
    assert_same(g2, o, "edge leaves, one-unit claims")


def test_duplicate_keys(shock, oracle_mod):
    base = splitmix64(800, 12)
    two = np.concatenate([base, base[:1]])            # a double edge: solvable
    three = np.concatenate([base[:9], base[:1], base[:1]])  # three parallel edges: never
    keys = np.concatenate([two, three])
    offs = np.array([0, len(two), len(two) + len(three)], dtype=np.uint64)
    o = oracle_mod.leaf_search(keys, offs, max_seed=20000)
    g = gpu_search(shock, keys, offs, max_seed=20000)
    assert o[0] == oracle_mod.ENOTFOUND and g[0] == shock.SHOCK_ENOTFOUND
    assert_same(g, o, "dups")
    rc, _, _ = gpu_search(shock, keys, offs, check_dups=True)
    assert rc == shock.SHOCK_EDUPKEY


def test_invalid_batches_leave_outputs_untouched(shock):
    keys = splitmix64(1, 200)
    past_end = np.array([0, 60, 120, 180, 240], np.uint64)  # the last leaf reaches past the 200 keys
    for offs in (np.array([0, 65], np.uint64), np.array([0, 10, 5], np.uint64), past_end):
        k, o = _dev(keys), _dev(offs)
        L = len(offs) - 1
        s = torch.full((L,), 12345, dtype=torch.int64, device="cuda")
        f = torch.full((L,), 678, dtype=torch.int64, device="cuda")
        rc, _, _ = shock.leaf_search(k, o, out_seeds=s, out_orient=f)
        torch.cuda.synchronize()
        assert rc == shock.SHOCK_EINVAL
        assert (s == 12345).all() and (f == 678).all()


def test_leaves_past_the_keys_are_rejected_by_every_search(shock):
    """A batch whose offsets reach past the keys tensor is SHOCK_EINVAL for the
    plain, rotation-fitting and bipartite searches and for a context (the
    binding passes the keys' length), and no key beyond the tensor is read."""
    keys = _dev(splitmix64(2, 100))
    offs = _dev(np.array([0, 50, 110], np.uint64))
    print("[gpu] offsets past the keys", flush=True)
    rc, _, _ = shock.leaf_search(keys, offs)
    assert rc == shock.SHOCK_EINVAL
    rc, _, _, _ = shock.rf_leaf_search(keys, offs)
    assert rc == shock.SHOCK_EINVAL
    rc, *_ = shock.bip_leaf_search(keys, offs)
    assert rc == shock.SHOCK_EINVAL
    ctx = shock.SearchContext(4)
    s = torch.zeros(2, dtype=torch.int64, device="cuda")
    f = torch.zeros(2, dtype=torch.int64, device="cuda")
    assert ctx.search_async(keys, offs, s, f) == 0
    assert ctx.wait()[0] == shock.SHOCK_EINVAL
    torch.cuda.synchronize()


def test_cancel_flag(shock):
    """A raised cancel flag (pinned host memory) stops the search; unfinished
    leaves report no seed."""
    flag = torch.ones(1, dtype=torch.int32).pin_memory()
    keys, offs = fixed_leaves(64, 56, 11)
    rc, s, f = gpu_search(shock, keys, offs, cancel_ptr=flag.data_ptr())
    assert rc == shock.SHOCK_ECANCELED
    assert (s == MAX).all() and (f == 0).all()


def test_stats_are_reported(shock):
    keys, offs = fixed_leaves(256, 24, 3)
    gpu_search(shock, keys, offs)
    st = shock.shock_last_stats()
    assert st["seeds_tested"] > 0 and st["kernel_ms"] > 0 and st["pf_checks"] >= 256


@pytest.mark.parametrize("L", [1, 3, 10, 100])
def test_small_batches_with_default_workers_match_oracle(shock, oracle_mod, L):
    """Small batches launch with the default worker count sized to the batch
    (about one wave per leaf, at least 512) instead of every resident wave;
    plain 40-key and rotation-fitting 48-key leaves still equal the oracle."""
    keys, offs = fixed_leaves(L, 40, 12_000 + L)
    g = gpu_search(shock, keys, offs)
    st = shock.shock_last_stats()
    assert 512 <= st["workers"] <= max(512, 4 * L), st
    o = oracle_mod.parallel(oracle_mod.leaf_search, keys, offs)
    assert_same(g, (0, np.concatenate([r[1] for r in o]), np.concatenate([r[2] for r in o])), f"plain L={L}")
    Lr = min(L, 20)  # the oracle's rotation fitting takes about 0.3 s per 48-key leaf
    keys, offs = fixed_leaves(Lr, 48, 12_100 + L)
    rc, s, r, f = shock.rf_leaf_search(_dev(keys), _dev(offs))
    torch.cuda.synchronize()
    o = oracle_mod.parallel(oracle_mod.rf_leaf_search, keys, offs)
    assert rc == 0 and all(x[0] == 0 for x in o)
    s_o, r_o, f_o = (np.concatenate([x[i] for x in o]) for i in (1, 2, 3))
    assert (_host(s) == s_o).all() and (r.cpu().numpy() == r_o).all() and (_host(f) == f_o).all()
