"""GPU tests of the serving loop: every request's result is the same alone and
in the mix (bit-exact), admission respects the HBM budget, batches overlap,
and the timeout and rejection paths work."""
import numpy as np
import pytest

from workloads import splitmix64

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shock():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2308_09561_amd as shock
    shock.lib()
    return shock


def _alone(shock, keys, offs):
    k = torch.from_numpy(np.ascontiguousarray(keys).view(np.int64)).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    rc, s, f = shock.leaf_search(k, o)
    torch.cuda.synchronize()
    assert rc == 0
    return s.cpu().numpy().view(np.uint64), f.cpu().numpy().view(np.uint64)


def _requests(n, base_seed, sizes, arrivals):
    from paper_2308_09561_amd.serving import Request
    return [Request(rid=i, arrival=arrivals[i], keys=splitmix64(base_seed + i, sizes[i])) for i in range(n)]


def test_results_identical_alone_and_in_mix(shock, oracle_mod):
    from paper_2308_09561_amd.serving import LeafServer
    sizes = [1000, 4800, 47, 2500, 1, 9999, 3000, 700, 12000, 5000]
    reqs = _requests(len(sizes), 9000, sizes, [0.0] * len(sizes))
    srv = LeafServer(hbm_budget_bytes=8 << 20, slots=3, leaf_size=24, max_batch_leaves=1024)
    print("[gpu] serving mix", flush=True)
    rep = srv.run(reqs, realtime=False)
    srv.close()
    summ = rep.summary()
    assert summ["completed"] == len(sizes)
    assert rep.max_batches_in_flight >= 2, summ
    for r in reqs:
        s, f = _alone(shock, r.keys, r.offsets)
        assert (r.seeds == s).all() and (r.orient == f).all(), r.rid
    # and a sample of leaves against the oracle
    r = reqs[3]
    o = oracle_mod.leaf_search(r.keys, r.offsets[:9])
    assert (o[1] == r.seeds[:8]).all() and (o[2] == r.orient[:8]).all()


def test_budget_is_respected_and_large_requests_rejected(shock):
    from paper_2308_09561_amd.serving import LeafServer, footprint, leaf_offsets
    sizes = [3000] * 6 + [200000]
    reqs = _requests(len(sizes), 9100, sizes, [0.0] * len(sizes))
    one = footprint(3000, len(leaf_offsets(3000, 24)) - 1)
    budget = 2 * one + 100
    srv = LeafServer(hbm_budget_bytes=budget, slots=4, leaf_size=24, max_batch_leaves=4096)
    print("[gpu] serving budget", flush=True)
    rep = srv.run(reqs, realtime=False)
    srv.close()
    assert rep.max_bytes_in_flight <= budget
    assert [r.status for r in reqs] == ["done"] * 6 + ["rejected"]


def test_queued_requests_time_out(shock):
    from paper_2308_09561_amd.serving import LeafServer
    sizes = [20000] * 8
    reqs = _requests(len(sizes), 9200, sizes, [0.0] * len(sizes))
    for r in reqs:
        r.deadline = 1e-3  # only what is admitted at once can make it
    srv = LeafServer(hbm_budget_bytes=64 << 20, slots=1, leaf_size=48, max_batch_leaves=600)
    print("[gpu] serving timeout", flush=True)
    rep = srv.run(reqs, realtime=False)
    srv.close()
    st = [r.status for r in reqs]
    assert st.count("done") >= 1 and st.count("timeout") >= 1
    assert all(s in ("done", "timeout") for s in st)


def test_realtime_stream_reports_latency(shock):
    from paper_2308_09561_amd.serving import LeafServer, synthetic_stream
    reqs = synthetic_stream(12, rate_per_s=400.0, seed=77, min_keys=1000, max_keys=20000)
    srv = LeafServer(hbm_budget_bytes=32 << 20, slots=4, leaf_size=48)
    print("[gpu] serving realtime", flush=True)
    rep = srv.run(reqs, realtime=True)
    srv.close()
    summ = rep.summary()
    assert summ["completed"] == 12
    assert summ["p50_ms"] > 0 and summ["p99_ms"] >= summ["p50_ms"]
    for r in reqs:
        assert r.latency() >= 0 and r.admitted >= r.arrival - 1e-6


@pytest.mark.parametrize("kind", ["plain", "bipartite"])
def test_mphf_server_builds_complete_functions(shock, kind):
    """Requests served as complete MPHF builds (plain or bipartite leaves):
    every request completes, its function is a bijection (checked by the
    server), the budget holds, and builds overlap."""
    from paper_2308_09561_amd.serving import MphfServer, mphf_footprint, synthetic_stream
    reqs = synthetic_stream(10, rate_per_s=1000.0, seed=79, min_keys=2000, max_keys=60000)
    budget = 3 * mphf_footprint(60000)
    srv = MphfServer(hbm_budget_bytes=budget, slots=3, bucket_size=600, leaf_target=24, leaf_max=36, verify=True,
                     bipartite=kind == "bipartite")
    print(f"[gpu] mphf serving, {kind} leaves", flush=True)
    rep = srv.run(reqs, realtime=False)
    srv.close()
    summ = rep.summary()
    assert summ["completed"] == 10 and rep.max_bytes_in_flight <= budget
    assert all(r.info["bijection"] for r in reqs)
    assert summ["p99_ms"] >= summ["p50_ms"] > 0 and 1.5 < summ["bits_per_key"] < 3.0
    assert rep.max_batches_in_flight >= 2
