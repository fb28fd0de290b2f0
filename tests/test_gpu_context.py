"""GPU tests of the asynchronous context API and HIP-graph replays, checked
against the CPU oracle (bit-exact) and against the synchronous entry point."""
import numpy as np
import pytest

from workloads import fixed_leaves, splitmix64, uneven_leaves

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


def _oracle(oracle_mod, keys, offs):
    parts = oracle_mod.parallel(oracle_mod.leaf_search, keys, offs)
    return np.concatenate([p[1] for p in parts]), np.concatenate([p[2] for p in parts])


def test_two_contexts_in_flight(shock, oracle_mod):
    ka, oa = uneven_leaves(200, 20, 34, 101, 102)
    kb, ob = fixed_leaves(120, 30, 103)
    sa, fa = _oracle(oracle_mod, ka, oa)
    sb, fb = _oracle(oracle_mod, kb, ob)
    ca, cb = shock.SearchContext(256), shock.SearchContext(256)
    st_a, st_b = torch.cuda.Stream(), torch.cuda.Stream()
    dka, doa, dkb, dob = _dev(ka), _dev(oa), _dev(kb), _dev(ob)
    outs = [torch.zeros(len(oa) - 1, dtype=torch.int64, device="cuda") for _ in range(2)] + \
           [torch.zeros(len(ob) - 1, dtype=torch.int64, device="cuda") for _ in range(2)]
    torch.cuda.synchronize()
    print("[gpu] two contexts", flush=True)
    assert ca.search_async(dka, doa, outs[0], outs[1], stream=st_a.cuda_stream, leaf_size_hint=28) == 0
    assert cb.search_async(dkb, dob, outs[2], outs[3], stream=st_b.cuda_stream, leaf_size_hint=30) == 0
    rc_a, stats_a = ca.wait()
    rc_b, stats_b = cb.wait()
    assert rc_a == 0 and rc_b == 0
    assert (_host(outs[0]) == sa).all() and (_host(outs[1]) == fa).all()
    assert (_host(outs[2]) == sb).all() and (_host(outs[3]) == fb).all()
    assert stats_a["seeds_tested"] > 0 and stats_b["kernel_ms"] > 0
    ca.close()
    cb.close()


def test_graph_replays_match_eager(shock, oracle_mod):
    """Capture once, replay several times with eager work and synchronisation
    between replays; every replay must equal the eager result."""
    keys, offs = uneven_leaves(300, 16, 40, 201, 202)
    s_ref, f_ref = _oracle(oracle_mod, keys, offs)
    dk, do = _dev(keys), _dev(offs)
    L = len(offs) - 1
    s_out = torch.zeros(L, dtype=torch.int64, device="cuda")
    f_out = torch.zeros(L, dtype=torch.int64, device="cuda")
    ctx = shock.SearchContext(L)
    stream = torch.cuda.Stream()
    assert ctx.capture(dk, do, s_out, f_out, stream=stream.cuda_stream, leaf_size_hint=28) == 0
    other_k, other_o = fixed_leaves(50, 24, 203)
    for rep in range(3):
        print(f"[gpu] graph replay {rep}", flush=True)
        s_out.zero_()
        f_out.zero_()
        torch.cuda.synchronize()
        assert ctx.launch_graph(stream=stream.cuda_stream) == 0
        rc, st = ctx.wait()
        assert rc == 0
        assert (_host(s_out) == s_ref).all() and (_host(f_out) == f_ref).all(), f"replay {rep}"
        # eager work between replays: a synchronous search of another batch
        rc2, _, _ = shock.leaf_search(_dev(other_k), _dev(other_o))
        torch.cuda.synchronize()
        assert rc2 == 0


def test_graph_replay_sees_new_buffer_contents(shock, oracle_mod):
    k1, offs = fixed_leaves(100, 22, 301)
    k2, _ = fixed_leaves(100, 22, 302)
    dk, do = _dev(k1), _dev(offs)
    s_out = torch.zeros(100, dtype=torch.int64, device="cuda")
    f_out = torch.zeros(100, dtype=torch.int64, device="cuda")
    ctx = shock.SearchContext(128)
    assert ctx.capture(dk, do, s_out, f_out, leaf_size_hint=22) == 0
    for keys in (k1, k2, k1):
        print("[gpu] replay with new keys", flush=True)
        dk.copy_(_dev(keys))
        torch.cuda.synchronize()
        assert ctx.launch_graph() == 0
        rc, _ = ctx.wait()
        assert rc == 0
        rc_o, s_o, f_o = oracle_mod.leaf_search(keys, offs)
        assert (_host(s_out) == s_o).all() and (_host(f_out) == f_o).all()


def test_async_invalid_batch(shock):
    keys = splitmix64(1, 300)
    offs = np.array([0, 40, 20, 100], dtype=np.uint64)
    ctx = shock.SearchContext(8)
    s = torch.full((3,), 7, dtype=torch.int64, device="cuda")
    f = torch.full((3,), 9, dtype=torch.int64, device="cuda")
    print("[gpu] async invalid", flush=True)
    assert ctx.search_async(_dev(keys), _dev(offs), s, f) == 0
    rc, _ = ctx.wait()
    assert rc == shock.SHOCK_EINVAL
    assert (s == 7).all() and (f == 9).all()
    # the same context works again afterwards
    k2, o2 = fixed_leaves(5, 12, 5)
    s2 = torch.zeros(5, dtype=torch.int64, device="cuda")
    f2 = torch.zeros(5, dtype=torch.int64, device="cuda")
    assert ctx.search_async(_dev(k2), _dev(o2), s2, f2, leaf_size_hint=12) == 0
    assert ctx.wait()[0] == 0


def test_claim_table_and_plain_async(shock, oracle_mod):
    """Per-leaf-size claim sizes (as the autotuner supplies) and the plain
    per-leaf mode on a context never change outputs."""
    keys, offs = uneven_leaves(120, 18, 44, 401, 402)
    s_ref, f_ref = _oracle(oracle_mod, keys, offs)
    rng = np.random.default_rng(7)
    table = [int(v) for v in rng.integers(1, 40, 65)]
    L = len(offs) - 1
    ctx = shock.SearchContext(L)
    for opts in (dict(block_iters_by_n=table), dict(block_iters_by_n=table, spl=4, waves_per_wg=8),
                 dict(mode=shock.SHOCK_MODE_PLAIN_PER_LEAF, leaf_size_hint=30)):
        print(f"[gpu] ctx opts {list(opts)}", flush=True)
        s = torch.zeros(L, dtype=torch.int64, device="cuda")
        f = torch.zeros(L, dtype=torch.int64, device="cuda")
        assert ctx.search_async(_dev(keys), _dev(offs), s, f, **opts) == 0
        assert ctx.wait()[0] == 0
        assert (_host(s) == s_ref).all() and (_host(f) == f_ref).all()
