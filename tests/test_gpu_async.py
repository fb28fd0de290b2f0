"""The asynchronous boundary through the C ABI: searches enqueued on a
caller's stream with their status read by shock_stream_status, and the
request queue bound to a device and an HBM budget (shock_submit / shock_poll).
Every result must equal the synchronous search's, leaf by leaf."""
import time

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


def _sync(shock, keys, offs, **opts):
    rc, s, f = shock.leaf_search(_dev(keys), _dev(offs), **opts)
    torch.cuda.synchronize()
    return rc, _host(s), _host(f)


def _wait_status(shock, stream):
    deadline = time.time() + 60
    while True:
        rc = shock.stream_status(stream.cuda_stream)
        if rc != shock.SHOCK_EPENDING:
            return rc
        assert time.time() < deadline, "stream status stayed pending"
        time.sleep(0.0005)


def test_async_search_on_a_stream_equals_sync(shock):
    st = torch.cuda.Stream()
    batches = [uneven_leaves(500, 16, 40, 700, 701), fixed_leaves(3000, 32, 702), fixed_leaves(7, 44, 703)]
    for i, (keys, offs) in enumerate(batches):
        L = len(offs) - 1
        print(f"[gpu] async search {i}: L={L}", flush=True)
        with torch.cuda.stream(st):
            k, o = _dev(keys), _dev(offs)
            s = torch.empty(L, dtype=torch.int64, device="cuda")
            f = torch.empty(L, dtype=torch.int64, device="cuda")
        rc = shock.leaf_search_async(k, o, s, f, stream=st.cuda_stream, leaf_size_hint=int(offs[-1]) // L)
        assert rc == shock.SHOCK_OK
        assert _wait_status(shock, st) == shock.SHOCK_OK
        st.synchronize()
        ref = _sync(shock, keys, offs)
        assert (_host(s) == ref[1]).all() and (_host(f) == ref[2]).all(), i


def test_async_calls_back_to_back_report_the_last(shock):
    """Two calls queued on one stream without waiting (the second larger, so
    the stream's scratch grows); the status is the last call's."""
    st = torch.cuda.Stream()
    k1, o1 = fixed_leaves(100, 24, 704)
    k2, o2 = fixed_leaves(5000, 24, 705)
    outs = []
    print("[gpu] async back to back", flush=True)
    with torch.cuda.stream(st):
        for keys, offs in ((k1, o1), (k2, o2)):
            L = len(offs) - 1
            k, o = _dev(keys), _dev(offs)
            s = torch.empty(L, dtype=torch.int64, device="cuda")
            f = torch.empty(L, dtype=torch.int64, device="cuda")
            assert shock.leaf_search_async(k, o, s, f, stream=st.cuda_stream, leaf_size_hint=24) == 0
            outs.append((k, o, s, f, keys, offs))
    assert _wait_status(shock, st) == shock.SHOCK_OK
    st.synchronize()
    for _, _, s, f, keys, offs in outs:
        ref = _sync(shock, keys, offs)
        assert (_host(s) == ref[1]).all() and (_host(f) == ref[2]).all()
    # a capped search on the same stream: its status replaces the last one
    k3, o3 = fixed_leaves(4, 40, 706)
    s3 = torch.zeros(4, dtype=torch.int64, device="cuda")
    f3 = torch.zeros(4, dtype=torch.int64, device="cuda")
    assert shock.leaf_search_async(_dev(k3), _dev(o3), s3, f3, stream=st.cuda_stream, max_seed=2) == 0
    assert _wait_status(shock, st) == shock.SHOCK_ENOTFOUND


def test_async_invalid_batch_and_unknown_stream(shock):
    st = torch.cuda.Stream()
    assert shock.stream_status(st.cuda_stream) == shock.SHOCK_EINVAL  # nothing enqueued on it yet
    keys = splitmix64(707, 300)
    offs = np.array([0, 40, 20, 100], dtype=np.uint64)
    s = torch.full((3,), 7, dtype=torch.int64, device="cuda")
    f = torch.full((3,), 9, dtype=torch.int64, device="cuda")
    print("[gpu] async invalid", flush=True)
    assert shock.leaf_search_async(_dev(keys), _dev(offs), s, f, stream=st.cuda_stream) == 0
    assert _wait_status(shock, st) == shock.SHOCK_EINVAL
    assert (s == 7).all() and (f == 9).all()
    # options checked before enqueueing
    k, o = fixed_leaves(2, 8, 708)
    assert shock.leaf_search_async(_dev(k), _dev(o), s, f, stream=st.cuda_stream, spl=3) == shock.SHOCK_EINVAL


def test_rf_async_equals_sync(shock):
    keys, offs = fixed_leaves(300, 40, 709)
    L = len(offs) - 1
    k, o = _dev(keys), _dev(offs)
    rc, s_ref, r_ref, f_ref = shock.rf_leaf_search(k, o)
    torch.cuda.synchronize()
    assert rc == 0
    st = torch.cuda.Stream()
    s = torch.empty(L, dtype=torch.int64, device="cuda")
    r = torch.empty(L, dtype=torch.int32, device="cuda")
    f = torch.empty(L, dtype=torch.int64, device="cuda")
    print("[gpu] rf async", flush=True)
    torch.cuda.synchronize()
    assert shock.rf_leaf_search_async(k, o, s, r, f, stream=st.cuda_stream, leaf_size_hint=40) == 0
    assert _wait_status(shock, st) == shock.SHOCK_OK
    st.synchronize()
    assert torch.equal(s, s_ref) and torch.equal(r, r_ref) and torch.equal(f, f_ref)


def _poll_all(q, tickets, timeout=120):
    res = {}
    deadline = time.time() + timeout
    while len(res) < len(tickets):
        for t in tickets:
            if t in res:
                continue
            done, rc, info, s, f = q.poll(t)
            if done:
                res[t] = (rc, info, s, f)
        assert time.time() < deadline, f"{len(tickets) - len(res)} requests never completed"
        time.sleep(0.0005)
    return res


def test_queue_results_equal_each_request_alone(shock):
    rng = np.random.default_rng(710)
    reqs = []
    for i in range(24):
        L = int(rng.integers(1, 400))
        lo, hi = (16, 40) if i % 2 else (24, 24)
        reqs.append(uneven_leaves(L, lo, hi, 7100 + i, 7200 + i))
    budget = 3 * shock.queue_batch_bytes(400, 400 * 40)
    q = shock.RequestQueue(hbm_budget_bytes=budget, slots=3, max_batch_leaves=800, max_batch_keys=800 * 40)
    print(f"[gpu] queue: {len(reqs)} requests, budget {budget}", flush=True)
    try:
        tickets = []
        for keys, offs in reqs:
            rc, t = q.submit(keys, offs)
            assert rc == shock.SHOCK_OK
            tickets.append(t)
        res = _poll_all(q, tickets)
        st = q.stats()
    finally:
        q.close()
    assert st["completed"] == len(reqs) and st["max_bytes_in_flight"] <= budget, st
    assert st["batches"] >= 2 and st["max_batches_in_flight"] >= 2, st
    for (keys, offs), t in zip(reqs, tickets):
        rc, info, s, f = res[t]
        assert rc == shock.SHOCK_OK
        assert info["done_ns"] >= info["admit_ns"] >= info["submit_ns"] > 0
        ref = _sync(shock, keys, offs)
        assert (s == ref[1]).all() and (f == ref[2]).all(), t


def test_queue_rejections_cancel_and_empty_requests(shock):
    q = shock.RequestQueue(hbm_budget_bytes=4 << 20, slots=1, max_batch_leaves=2000, max_batch_keys=2000 * 48)
    print("[gpu] queue edges", flush=True)
    try:
        # larger than the budget or a batch: not queued
        big_k, big_o = fixed_leaves(3000, 48, 711)
        assert q.submit(big_k, big_o)[0] == shock.SHOCK_ENOMEM
        # malformed (a leaf of 65 keys): checked on the host
        k65 = splitmix64(712, 65)
        assert q.submit(k65, np.array([0, 65], np.uint64))[0] == shock.SHOCK_EINVAL
        # empty request: done at once
        rc, t0 = q.submit(np.zeros(0, np.uint64), np.zeros(1, np.uint64))
        assert rc == 0
        done, rc, info, s, f = q.poll(t0)
        assert done and rc == 0 and len(s) == 0
        # a heavy request occupies the only slot; the next one is withdrawn while queued
        hk, ho = fixed_leaves(1500, 48, 713)
        rc, th = q.submit(hk, ho)
        assert rc == 0
        lk, lo = fixed_leaves(10, 24, 714)
        rc, tl = q.submit(lk, lo)
        assert rc == 0
        c = q.cancel(tl)
        res = _poll_all(q, [th, tl])
        assert res[th][0] == shock.SHOCK_OK
        if c == shock.SHOCK_OK:
            assert res[tl][0] == shock.SHOCK_ECANCELED
        else:  # already admitted alongside the heavy one
            assert c == shock.SHOCK_EPENDING and res[tl][0] == shock.SHOCK_OK
        assert q.poll(th)[1] == shock.SHOCK_EINVAL  # tickets retire once reported done
        ref = _sync(shock, hk, ho)
        assert (res[th][2] == ref[1]).all() and (res[th][3] == ref[2]).all()
    finally:
        q.close()


def test_queue_random_stream_with_cancels(shock, oracle_mod):
    """200 requests of random sizes (empty ones, single leaves, up to 1500
    leaves of 1 to 40 keys) under a budget of a few batches, submitted in
    bursts with random cancels and polls in between: every request ends
    exactly once, a cancelled one either as cancelled or with its full
    result, every result equals the oracle's leaf by leaf, and the budget
    holds throughout."""
    rng = np.random.default_rng(720)
    reqs = []
    for i in range(200):
        L = int(rng.choice([0, 1, int(rng.integers(2, 200)), int(rng.integers(200, 1500))], p=[.05, .1, .6, .25]))
        sizes = rng.integers(1, 41, L)
        offs = np.zeros(L + 1, np.uint64)
        np.cumsum(sizes.astype(np.uint64), out=offs[1:])
        reqs.append((splitmix64(7300 + i, int(offs[-1])), offs))
    budget = 3 * shock.queue_batch_bytes(1500, 1500 * 40)
    q = shock.RequestQueue(hbm_budget_bytes=budget, slots=int(rng.integers(1, 5)), max_batch_leaves=3000,
                           max_batch_keys=3000 * 40)
    print(f"[gpu] queue random stream: {len(reqs)} requests, budget {budget}", flush=True)
    tickets, cancelled, res = {}, set(), {}
    try:
        i = 0
        while i < len(reqs):
            for _ in range(int(rng.integers(1, 12))):  # a burst of submits
                if i == len(reqs):
                    break
                rc, t = q.submit(*reqs[i])
                assert rc == shock.SHOCK_OK, i
                tickets[t] = i
                i += 1
            open_t = [t for t in tickets if t not in res]
            for t in rng.choice(open_t, size=min(len(open_t), int(rng.integers(0, 3))), replace=False):
                c = q.cancel(int(t))
                assert c in (shock.SHOCK_OK, shock.SHOCK_EPENDING, shock.SHOCK_EINVAL)
                if c == shock.SHOCK_OK:
                    cancelled.add(int(t))
            for t in list(open_t):
                done, rc, info, s, f = q.poll(t)
                if done:
                    res[t] = (rc, s, f)
            time.sleep(float(rng.uniform(0, 0.003)))
        deadline = time.time() + 120
        while len(res) < len(tickets):
            for t in tickets:
                if t not in res:
                    done, rc, info, s, f = q.poll(t)
                    if done:
                        res[t] = (rc, s, f)
            assert time.time() < deadline, f"{len(tickets) - len(res)} requests never completed"
            time.sleep(0.0005)
        st = q.stats()
    finally:
        q.close()
    assert st["max_bytes_in_flight"] <= budget and st["submitted"] == len(reqs), st
    assert st["completed"] == len(reqs) and st["cancelled"] == len(cancelled), st
    keys_all = np.concatenate([k for k, _ in reqs])
    offs_all = np.zeros(1, np.uint64)
    for _, o in reqs:
        offs_all = np.concatenate([offs_all, o[1:] + offs_all[-1]])
    parts = oracle_mod.parallel(oracle_mod.leaf_search, keys_all, offs_all, threads=16)
    want_s = np.concatenate([p[1] for p in parts])
    want_f = np.concatenate([p[2] for p in parts])
    first = np.concatenate([[0], np.cumsum([len(o) - 1 for _, o in reqs])])
    n_cancel = 0
    for t, i in tickets.items():
        rc, s, f = res[t]
        assert (rc == shock.SHOCK_ECANCELED) == (t in cancelled), (i, rc)  # withdrawn exactly when cancel said so
        if rc == shock.SHOCK_ECANCELED:
            n_cancel += 1
            continue
        assert rc == shock.SHOCK_OK, (i, rc)
        a, b = int(first[i]), int(first[i + 1])
        assert (s == want_s[a:b]).all() and (f == want_f[a:b]).all(), i
    print(f"[gpu] queue random stream: {n_cancel} cancelled, {len(reqs) - n_cancel} checked", flush=True)
