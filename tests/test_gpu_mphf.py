"""GPU parity of the flat ShockHash MPHF (include/shockmphf.h) against the
oracle: every stored part bit-exact (bucket offsets, leaf bases, splitting
seeds, leaf sizes, leaf seeds, and the retrieval: each bucket's ribbon seed
and bits, or the XOR system's seed and cells), every key's position equal,
and the bijection onto [0, N) at full size."""
import numpy as np
import pytest

from workloads import splitmix64

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

SMALL = dict(bucket_size=300, leaf_target=12, leaf_max=18)


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


RIBBON, XOR = 0, 1


def _same_retrieval(ex, lay):
    """The GPU's retrieval parts equal the oracle's."""
    assert ex["retrieval"] == lay["retrieval"]
    if ex["retrieval"] == XOR:
        return ex["rho"] == lay["rho"] and (ex["z"] == lay["z"]).all()
    return ((ex["rseed"] == lay["rseed"]).all() and (ex["rbit_offset"] == lay["rbit_offset"]).all()
            and (ex["z"] == lay["z"]).all())


def _oracle_struct(lay, ex, **kw):
    """The oracle's layout with the GPU's exported seeds and retrieval, for
    the oracle's query over the GPU structure."""
    d = dict(lay, seeds=ex["seeds"], retrieval=ex["retrieval"], rho=ex["rho"], z=ex["z"], leaf_target=40, **kw)
    if ex["retrieval"] == RIBBON:
        d.update(rseed=ex["rseed"], rbit_offset=ex["rbit_offset"])
    return d


def _build(shock, keys, **params):
    print(f"[gpu] mphf build N={len(keys)} {params}", flush=True)
    k = _dev(keys) if len(keys) else torch.zeros(0, dtype=torch.int64, device="cuda")
    m = shock.MPHF(k, **params)
    torch.cuda.synchronize()
    return m, k


@pytest.mark.parametrize("ret", [RIBBON, XOR], ids=["ribbon", "xor"])
@pytest.mark.parametrize("rf", [False, True], ids=["plain", "rf"])
@pytest.mark.parametrize("N", [1, 2, 17, 1000, 6000])
def test_mphf_matches_oracle(shock, oracle_mod, N, rf, ret):
    keys = splitmix64(2100 + N, N)
    m, k = _build(shock, keys, rotation_fitting=rf, retrieval=ret, **SMALL)
    try:
        rc, lay = oracle_mod.mphf_build(keys, rf=rf, retrieval=ret, **SMALL)
        assert rc == 0
        ex = m.export()
        assert (ex["bucket_offset"] == lay["bucket_offset"]).all()
        assert (ex["leaf_base"] == lay["leaf_base"]).all()
        assert (ex["sigma"] == lay["sigma"]).all()
        assert (ex["leaf_sizes"] == lay["leaf_sizes"]).all()
        assert (ex["seeds"] == lay["seeds"]).all()
        assert _same_retrieval(ex, lay)
        pos = _host(m.query(k))
        torch.cuda.synchronize()
        assert (pos == lay["positions"]).all()
        assert sorted(pos.tolist()) == list(range(N))
    finally:
        m.close()


@pytest.mark.parametrize("rows", [1, 120, 256])
def test_ribbon_row_capacity_moves_buckets_to_the_walk_with_equal_results(shock, oracle_mod, rows):
    """The ribbon solver by column blocks hands a bucket to the sequential walk
    when a block holds more rows than ribbon_rows; either way the ribbon seeds
    and bits are the oracle's.  One row sends every bucket of two or more keys
    to the walk, 120 some of them (buckets of about 300 keys put about 80
    rows in a block, plus the rows left from the block before; 5 of these 20
    buckets pass 120 at a seed tried), 256 none."""
    N = 6000
    keys = splitmix64(2150, N)
    m, k = _build(shock, keys, ribbon_rows=rows, **SMALL)
    try:
        rc, lay = oracle_mod.mphf_build(keys, rf=False, retrieval=RIBBON, **SMALL)
        assert rc == 0
        ex, info = m.export(), m.info()
        print(f"[gpu] ribbon_rows={rows}: walked {info['ribbon_walked']} of {info['n_buckets']}", flush=True)
        assert _same_retrieval(ex, lay)
        assert (ex["seeds"] == lay["seeds"]).all()
        sizes = np.diff(lay["bucket_offset"].astype(np.int64))
        if rows == 1:
            assert info["ribbon_walked"] == int((sizes >= 2).sum())
        elif rows == 120:
            assert 0 < info["ribbon_walked"] < info["n_buckets"]
        else:
            assert info["ribbon_walked"] == 0
        pos = _host(m.query(k))
        assert (pos == lay["positions"]).all()
    finally:
        m.close()
    with pytest.raises(shock.ShockError):
        shock.MPHF(k, ribbon_rows=257, **SMALL)


def test_mphf_default_parameters_full_size(shock, oracle_mod):
    """200,000 keys with the default layout (buckets of 3000, leaves of 40 on
    average, at most 56, ribbon retrieval): the layout equals the oracle's
    split, a sample of leaves has the oracle's seeds, a sample of buckets has
    the oracle's ribbon seed and bits, the oracle's query over the exported
    structure equals the GPU query for every key, the positions are a
    permutation of [0, N), and the space is at most 1.65 bits per key."""
    N = 200_000
    keys = splitmix64(2200, N)
    m, k = _build(shock, keys)
    try:
        info = m.info()
        print(f"[gpu] mphf info {info}", flush=True)
        assert info["n_keys"] == N and 1.5 < info["bits_per_key"] <= 1.65
        assert info["ribbon_walked"] == 0  # every bucket by column blocks
        pos_t = m.query(k)
        srt, _ = torch.sort(pos_t)
        assert torch.equal(srt, torch.arange(N, device="cuda", dtype=torch.int64))
        ex = m.export()
        rc, lay = oracle_mod.mphf_split(keys, 3000, 40, 56)
        assert rc == 0
        for f in ("bucket_offset", "leaf_base", "sigma", "leaf_sizes"):
            assert (ex[f] == lay[f]).all(), f
        offs = lay["leaf_offsets"]
        pick = np.random.default_rng(2201).choice(lay["n_leaves"], 24, replace=False)
        for j in pick:
            _, s, _ = oracle_mod.leaf_search(lay["leaf_keys"], offs[j:j + 2])
            assert int(s[0]) == int(ex["seeds"][j]), j
        # ribbon systems of sampled buckets, from the GPU's own choices (the
        # positions' structure is checked by the full query below)
        pos = _host(pos_t)
        struct = _oracle_struct(lay, ex)
        for b in np.random.default_rng(2202).choice(lay["n_buckets"], 4, replace=False):
            o0, o1 = int(lay["bucket_offset"][b]), int(lay["bucket_offset"][b + 1])
            bk = lay["leaf_keys"][o0:o1]
            vals = np.array([oracle_mod.ribbon_get(int(x), int(ex["rseed"][b]), oracle_mod.ribbon_cols(o1 - o0),
                                                   ex["z"][int(ex["rbit_offset"][b]):]) for x in bk], np.uint8)
            rc, r_o, z_o = oracle_mod.ribbon_build(bk, vals)
            assert rc == 0 and r_o == int(ex["rseed"][b]), b
            assert (z_o == ex["z"][int(ex["rbit_offset"][b]):int(ex["rbit_offset"][b + 1])]).all(), b
        rc, want = oracle_mod.mphf_query(struct, keys)
        assert rc == 0 and (pos == want).all()
    finally:
        m.close()


def test_mphf_queries_of_other_keys_stay_in_range(shock):
    keys = splitmix64(2300, 5000)
    m, k = _build(shock, keys, **SMALL)
    try:
        others = _dev(splitmix64(2301, 4000))
        p = _host(m.query(others))
        assert ((p < 5000) | (p == np.uint64(0xFFFFFFFFFFFFFFFF))).all()
    finally:
        m.close()


def test_mphf_errors(shock):
    keys = np.concatenate([splitmix64(2400, 500), splitmix64(2400, 3)])  # three keys repeat
    with pytest.raises(shock.ShockError) as e:
        _build(shock, keys, **SMALL)
    assert e.value.status == shock.SHOCK_EDUPKEY
    for bad in (dict(bucket_size=0), dict(leaf_target=60, leaf_max=56), dict(leaf_max=65)):
        with pytest.raises(shock.ShockError) as e:
            _build(shock, splitmix64(2401, 100), **bad)
        assert e.value.status == shock.SHOCK_EINVAL
    # bipartite leaves have no duplicate check: repeated keys leave the
    # retrieval unsolvable for every seed, which is reported as not found
    with pytest.raises(shock.ShockError) as e:
        _build(shock, keys, bipartite=True, **SMALL)
    assert e.value.status == shock.SHOCK_ENOTFOUND
    with pytest.raises(shock.ShockError) as e:
        _build(shock, splitmix64(2401, 100), bipartite=True, rotation_fitting=True)
    assert e.value.status == shock.SHOCK_EINVAL
    m, _ = _build(shock, np.zeros(0, np.uint64), **SMALL)
    try:
        assert m.info()["n_keys"] == 0
        p = _host(m.query(_dev(splitmix64(2402, 10))))
        assert (p == np.uint64(0xFFFFFFFFFFFFFFFF)).all()
    finally:
        m.close()


def test_concurrent_builds_and_searches_from_threads(shock):
    """Synchronous calls from several host threads on their own streams run
    concurrently; each thread keeps its own scratch, so results equal the
    serial ones."""
    from concurrent.futures import ThreadPoolExecutor
    from workloads import fixed_leaves

    batches = [fixed_leaves(256, 30 + i, 2500 + i) for i in range(4)]

    def search(i):
        keys, offs = batches[i]
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            rc, s, f = shock.leaf_search(_dev(keys), _dev(offs), stream=stream.cuda_stream)
            stream.synchronize()
        return rc, _host(s), _host(f)

    print("[gpu] serial searches", flush=True)
    serial = [search(i) for i in range(4)]
    print("[gpu] threaded searches", flush=True)
    with ThreadPoolExecutor(4) as ex:
        threaded = list(ex.map(search, range(4)))
    for a, b in zip(serial, threaded):
        assert a[0] == b[0] == 0 and (a[1] == b[1]).all() and (a[2] == b[2]).all()

    def build(i):
        keys = splitmix64(2600 + i, 3000 + 500 * i)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            k = _dev(keys)
            m = shock.MPHF(k, stream=stream.cuda_stream, **SMALL)
            p = _host(m.query(k, stream=stream.cuda_stream))
            stream.synchronize()
            m.close()
        return p

    print("[gpu] threaded builds", flush=True)
    with ThreadPoolExecutor(3) as ex:
        outs = list(ex.map(build, range(3)))
    for i, p in enumerate(outs):
        assert sorted(p.tolist()) == list(range(3000 + 500 * i))
        assert (p == build(i)).all()


def test_mphf_rotation_fitting_full_size(shock, oracle_mod):
    """200,000 keys, default layout, rotation-fitting leaves: the oracle's
    query over the exported structure equals the GPU query for every key, a
    sample of leaves has the oracle's candidates, and the positions are a
    permutation of [0, N)."""
    N = 200_000
    keys = splitmix64(2700, N)
    m, k = _build(shock, keys, rotation_fitting=True)
    try:
        pos_t = m.query(k)
        srt, _ = torch.sort(pos_t)
        assert torch.equal(srt, torch.arange(N, device="cuda", dtype=torch.int64))
        ex = m.export()
        rc, lay = oracle_mod.mphf_split(keys, 3000, 40, 56)
        assert rc == 0
        for f in ("bucket_offset", "leaf_base", "sigma", "leaf_sizes"):
            assert (ex[f] == lay[f]).all(), f
        offs = lay["leaf_offsets"]
        for j in np.random.default_rng(2701).choice(lay["n_leaves"], 24, replace=False):
            _, s, r, _ = oracle_mod.rf_leaf_search(lay["leaf_keys"], offs[j:j + 2])
            n = int(offs[j + 1] - offs[j])
            want = int(s[0]) * n + int(r[0]) if n >= 2 else int(s[0])
            assert want == int(ex["seeds"][j]), j
        struct = _oracle_struct(lay, ex, rf=True, partial_k=0)
        rc, want = oracle_mod.mphf_query(struct, keys)
        assert rc == 0 and (_host(pos_t) == want).all()
    finally:
        m.close()


def test_build_arena_reuse_across_sizes(shock, oracle_mod):
    """Builds on one thread reuse a cached scratch arena: a large build, then
    smaller ones (stale contents must not leak into them), then a larger one
    (the arena grows), then again after the cache is released; every build
    equals the oracle's."""
    sizes = [6000, 17, 1000, 0, 9000, 2500]
    for step, N in enumerate(sizes):
        if step == 4:
            assert shock.shock_release_scratch() == 0
        keys = splitmix64(2300 + step, N)
        m, k = _build(shock, keys, rotation_fitting=bool(step % 2), **SMALL)
        try:
            rc, lay = oracle_mod.mphf_build(keys, rf=bool(step % 2), **SMALL)
            assert rc == 0
            ex = m.export()
            assert (ex["seeds"] == lay["seeds"]).all(), step
            assert _same_retrieval(ex, lay), step
            if N:
                pos = _host(m.query(k))
                torch.cuda.synchronize()
                assert (pos == lay["positions"]).all(), step
        finally:
            m.close()


@pytest.mark.parametrize("rf", [False, True], ids=["plain", "rf"])
def test_mphf_more_buckets_than_the_lds_histogram(shock, oracle_mod, rf):
    """9000 buckets: above the 8192 that the layout's LDS histograms hold, so
    the bucket count and scatter take their global-atomic form; the result
    must still equal the oracle's."""
    params = dict(bucket_size=10, leaf_target=5, leaf_max=10)
    keys = splitmix64(2400 + rf, 90000)
    m, k = _build(shock, keys, rotation_fitting=rf, **params)
    try:
        rc, lay = oracle_mod.mphf_build(keys, rf=rf, **params)
        assert rc == 0
        ex = m.export()
        assert len(ex["bucket_offset"]) == 9001
        assert (ex["bucket_offset"] == lay["bucket_offset"]).all()
        assert (ex["leaf_sizes"] == lay["leaf_sizes"]).all()
        assert (ex["seeds"] == lay["seeds"]).all() and _same_retrieval(ex, lay)
        pos = _host(m.query(k))
        torch.cuda.synchronize()
        assert (pos == lay["positions"]).all()
    finally:
        m.close()


@pytest.mark.parametrize("N", [65536, 65537])
def test_mphf_retrieval_on_both_sides_of_the_one_workgroup_limit(shock, oracle_mod, N):
    """Retrieval systems of up to 2^16 keys are solved by one workgroup, larger
    ones by the multi-launch rounds; at the limit and one key above it the
    retrieval seed and cells equal the oracle's."""
    keys = splitmix64(2500 + N, N)
    m, k = _build(shock, keys, retrieval=XOR, **SMALL)
    try:
        rc, lay = oracle_mod.mphf_build(keys, retrieval=XOR, **SMALL)
        assert rc == 0
        ex = m.export()
        assert (ex["seeds"] == lay["seeds"]).all()
        assert _same_retrieval(ex, lay)
        pos = _host(m.query(k))
        torch.cuda.synchronize()
        assert (pos == lay["positions"]).all()
    finally:
        m.close()


@pytest.mark.parametrize("N", [1, 2, 17, 1000, 6000])
def test_mphf_bipartite_leaves_match_oracle(shock, oracle_mod, N):
    """Bipartite leaves: every stored part (the leaf values are the ranks of
    the seed pairs) and every position bit-exact against the oracle."""
    keys = splitmix64(2800 + N, N)
    m, k = _build(shock, keys, bipartite=True, **SMALL)
    try:
        rc, lay = oracle_mod.mphf_build(keys, bip=True, **SMALL)
        assert rc == 0
        ex = m.export()
        for f in ("bucket_offset", "leaf_base", "sigma", "leaf_sizes", "seeds"):
            assert (ex[f] == lay[f]).all(), f
        assert _same_retrieval(ex, lay)
        pos = _host(m.query(k))
        torch.cuda.synchronize()
        assert (pos == lay["positions"]).all()
        assert sorted(pos.tolist()) == list(range(N))
    finally:
        m.close()


def test_mphf_bipartite_leaves_full_size(shock, oracle_mod):
    """200,000 keys with the default layout and bipartite leaves: a bijection,
    the layout and a sample of leaf values equal the oracle's, and the
    oracle's query over the exported structure equals the GPU query."""
    N = 200_000
    keys = splitmix64(2900, N)
    m, k = _build(shock, keys, bipartite=True)
    try:
        pos_t = m.query(k)
        srt, _ = torch.sort(pos_t)
        assert torch.equal(srt, torch.arange(N, device="cuda", dtype=torch.int64))
        ex = m.export()
        rc, lay = oracle_mod.mphf_split(keys, 3000, 40, 56)
        assert rc == 0
        offs = lay["leaf_offsets"]
        pick = np.random.default_rng(2901).choice(lay["n_leaves"], 64, replace=False)
        for j in pick:
            _, a, b, _ = oracle_mod.bip_leaf_search(lay["leaf_keys"], offs[j:j + 2])
            assert int(ex["seeds"][j]) == oracle_mod.bip_pair_rank(int(a[0]), int(b[0])), j
        struct = _oracle_struct(lay, ex, bip=True)
        rc, want = oracle_mod.mphf_query(struct, keys)
        assert rc == 0 and (_host(pos_t) == want).all()
    finally:
        m.close()


def test_ribbon_large_buckets_block_solver_and_global_walk(shock, oracle_mod):
    """Two buckets of about 7250 keys: the block solver takes them (its
    stage, counts and indices fit the LDS), and with ribbon_rows = 1 every
    bucket goes to the walk, whose slots for buckets this large live in
    global memory (more than 64 KB of LDS).  Both give the oracle's ribbon
    seeds and bits."""
    N = 14500
    params = dict(bucket_size=7250, leaf_target=40, leaf_max=56, bipartite=True)
    keys = splitmix64(2160, N)
    rc, lay = oracle_mod.mphf_build(keys, bucket_size=7250, leaf_target=40, leaf_max=56, bip=True, retrieval=RIBBON)
    assert rc == 0
    assert int(np.diff(lay["bucket_offset"].astype(np.int64)).max()) > 7000
    for rows in (0, 1):
        m, k = _build(shock, keys, ribbon_rows=rows, **params)
        try:
            ex, info = m.export(), m.info()
            assert info["ribbon_walked"] == (info["n_buckets"] if rows == 1 else 0)
            assert _same_retrieval(ex, lay), rows
            pos = _host(m.query(k))
            assert (pos == lay["positions"]).all()
        finally:
            m.close()


@pytest.mark.parametrize("bucket_size,seed", [(3000, 2170), (5000, 2171), (7250, 2172)])
def test_ribbon_second_launch_widths(shock, oracle_mod, bucket_size, seed):
    """Twelve buckets whose oracle ribbon seeds reach 2 and more, so the
    second ribbon launch runs.  Its width (seeds tried at once per bucket)
    is what the LDS holds for the largest bucket: five waves at buckets of
    about 3000 keys (two rounds, seed 9 is needed), four at 5000 and two at
    7250 (three rounds, seed 6).  Every width gives the oracle's seeds, bits
    and positions."""
    N = 12 * bucket_size
    keys = splitmix64(seed, N)
    print(f"[gpu] ribbon second launch: buckets of {bucket_size}", flush=True)
    rc, lay = oracle_mod.mphf_build(keys, bucket_size=bucket_size, leaf_target=40, leaf_max=56, bip=True,
                                    retrieval=RIBBON)
    assert rc == 0
    rs = np.asarray(lay["rseed"], dtype=np.int64)
    assert rs.max() >= 2
    m, k = _build(shock, keys, bucket_size=bucket_size, leaf_target=40, leaf_max=56, bipartite=True)
    try:
        ex, info = m.export(), m.info()
        assert info["ribbon_walked"] == 0
        assert info["max_rseed"] == int(rs.max())
        assert _same_retrieval(ex, lay)
        pos = _host(m.query(k))
        assert (pos == lay["positions"]).all()
    finally:
        m.close()
