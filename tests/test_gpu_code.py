"""GPU parity of the leaf query and the Golomb-Rice seed codes
(include/shockcode.h) against the oracle, through the C ABI: query positions,
both code streams and the index bit-exact, decoding the exact inverse."""
import math

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


def _dev(a, dtype=np.uint64):
    a = np.ascontiguousarray(a, dtype=dtype)
    view = np.int64 if dtype == np.uint64 else np.int32
    return torch.from_numpy(a.view(view)).cuda()


def _host(t):
    return t.cpu().numpy().view(np.uint64)


def _query(shock, keys, offs, seeds, orient, rot=None, partial_k=0):
    print(f"[gpu] query L={len(offs) - 1} rf={rot is not None}", flush=True)
    k = _dev(keys) if len(keys) else torch.zeros(1, dtype=torch.int64, device="cuda")
    if rot is None:
        rc, pos = shock.leaf_query(k, _dev(offs), _dev(seeds), _dev(orient))
    else:
        rc, pos = shock.rf_leaf_query(k, _dev(offs), _dev(seeds), _dev(rot, np.uint32), _dev(orient), partial_k)
    torch.cuda.synchronize()
    return rc, _host(pos)


# ---------------------------------------------------------------- query ----

def test_query_matches_oracle_on_uneven_leaves(shock, oracle_mod):
    keys, offs = uneven_leaves(500, 0, 40, 901, 902)
    _, s, f = oracle_mod.leaf_search(keys, offs)
    rc, pos = _query(shock, keys, offs, s, f)
    _, want = oracle_mod.leaf_query(keys, offs, s, f)
    assert rc == 0 and (pos == want).all()
    assert sorted(pos.tolist()) == list(range(int(offs[-1])))  # a minimal perfect hash of the batch


def test_query_of_missing_seeds_and_arbitrary_choices(shock, oracle_mod):
    """Not only search results: any seeds (UINT64_MAX included) and any
    orientation bits give the oracle's positions."""
    keys, offs = uneven_leaves(300, 0, 64, 903, 904)
    rng = np.random.default_rng(905)
    s = rng.integers(0, 1 << 40, size=300, dtype=np.uint64)
    s[::7] = MAX
    f = splitmix64(906, 300)
    rc, pos = _query(shock, keys, offs, s, f)
    _, want = oracle_mod.leaf_query(keys, offs, s, f)
    assert rc == 0 and (pos == want).all()


@pytest.mark.parametrize("partial_k", [0, 1, 8])
def test_rf_query_matches_oracle(shock, oracle_mod, partial_k):
    keys, offs = uneven_leaves(200, 0, 64, 907, 908)
    rng = np.random.default_rng(909 + partial_k)
    s = rng.integers(0, 1 << 50, size=200, dtype=np.uint64)
    sizes = np.diff(offs).astype(np.int64)
    r = np.array([rng.integers(0, max(n, 1)) for n in sizes], dtype=np.uint32)
    f = splitmix64(910, 200)
    rc, pos = _query(shock, keys, offs, s, f, rot=r, partial_k=partial_k)
    _, want = oracle_mod.rf_leaf_query(keys, offs, s, r, f, partial_k=partial_k)
    assert rc == 0 and (pos == want).all()


def test_rf_query_of_search_results_is_a_bijection(shock, oracle_mod):
    keys, offs = uneven_leaves(150, 1, 44, 911, 912)
    k, o = _dev(keys), _dev(offs)
    rc, s, r, f = shock.rf_leaf_search(k, o)
    assert rc == 0
    rc, pos = shock.rf_leaf_query(k, o, s, r, f)
    torch.cuda.synchronize()
    pos = _host(pos)
    assert rc == 0 and sorted(pos.tolist()) == list(range(int(offs[-1])))
    _, want = oracle_mod.rf_leaf_query(keys, offs, _host(s), r.cpu().numpy().astype(np.uint32), _host(f))
    assert (pos == want).all()


def test_query_full_batch_after_search(shock, oracle_mod):
    """The fixed48 batch: search then query on the GPU; the positions are a
    permutation of [0, N), and a sample of leaves equals the oracle's query."""
    keys, offs = make_workload("fixed48")
    k, o = _dev(keys), _dev(offs)
    print("[gpu] fixed48 search + query", flush=True)
    rc, s, f = shock.leaf_search(k, o)
    assert rc == 0
    rc, pos = shock.leaf_query(k, o, s, f)
    torch.cuda.synchronize()
    assert rc == 0
    pos_t = pos.clone()
    srt, _ = torch.sort(pos_t)
    assert torch.equal(srt, torch.arange(int(offs[-1]), device="cuda", dtype=torch.int64))
    pos = _host(pos)
    s, f = _host(s), _host(f)
    for j in np.random.default_rng(913).choice(len(offs) - 1, 40, replace=False):
        sub = offs[j:j + 2]
        _, want = oracle_mod.leaf_query(keys, sub, s[j:j + 1], f[j:j + 1])
        assert (pos[int(sub[0]):int(sub[1])] == want[int(sub[0]):int(sub[1])]).all(), j


def test_query_edge_cases(shock, oracle_mod):
    keys = splitmix64(914, 3)
    offs = np.array([0, 0, 1, 1, 3], dtype=np.uint64)
    s = np.array([0, 5, 0, 9], dtype=np.uint64)
    f = np.array([0, 0, 0, 2], dtype=np.uint64)
    rc, pos = _query(shock, keys, offs, s, f)
    _, want = oracle_mod.leaf_query(keys, offs, s, f)
    assert rc == 0 and (pos == want).all() and pos[0] == 0
    rc, pos = _query(shock, np.zeros(0, np.uint64), np.zeros(1, np.uint64), np.zeros(0, np.uint64),
                     np.zeros(0, np.uint64))
    assert rc == 0 and pos.size == 0


# ------------------------------------------------------------ Rice codes ----

def _encode(shock, values, offs, table):
    print(f"[gpu] rice encode L={len(offs) - 1}", flush=True)
    v = _dev(values) if len(values) else torch.zeros(1, dtype=torch.int64, device="cuda")
    rc, fx, un, idx, bits = shock.rice_encode(v, _dev(offs), table)
    torch.cuda.synchronize()
    return rc, _host(fx), _host(un), _host(idx), bits


def _random_batch(L, seed, k_max=56, p=0.3):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(0, 65, size=L)
    offs = np.zeros(L + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offs[1:])
    table = rng.integers(0, k_max + 1, size=65).tolist()
    q = rng.geometric(p, size=L) - 1
    low = np.array([int(rng.integers(0, 1 << table[n], dtype=np.uint64)) if table[n] else 0 for n in sizes],
                   dtype=np.uint64)
    ks = np.array([table[n] for n in sizes], dtype=np.uint64)
    return (q.astype(np.uint64) << ks) | low, offs, table


@pytest.mark.parametrize("L", [1, 63, 64, 65, 1000, 4097])
def test_rice_encode_matches_oracle(shock, oracle_mod, L):
    values, offs, table = _random_batch(L, 920 + L)
    g = _encode(shock, values, offs, table)
    o = oracle_mod.rice_encode(values, offs, np.array(table, np.uint8))
    assert g[0] == 0 and o[0] == 0
    assert g[4] == o[4]
    assert (g[1] == o[1]).all() and (g[2] == o[2]).all() and (g[3] == o[3]).all()


@pytest.mark.parametrize("L", [1, 64, 1000, 4097])
def test_rice_decode_round_trip(shock, oracle_mod, L):
    values, offs, table = _random_batch(L, 930 + L, p=0.05)
    v = _dev(values)
    o = _dev(offs)
    rc, fx, un, idx, bits = shock.rice_encode(v, o, table)
    assert rc == 0
    print(f"[gpu] rice decode L={L}", flush=True)
    rc, back = shock.rice_decode(fx, un, idx, o, table)
    torch.cuda.synchronize()
    assert rc == 0 and (_host(back) == values).all()
    # and the oracle decodes the GPU's streams
    rc, ob = oracle_mod.rice_decode(_host(fx), _host(un), offs, np.array(table, np.uint8))
    assert rc == 0 and (ob == values).all()


def test_rice_long_unary_segments(shock, oracle_mod):
    """k = 0 everywhere and large quotients: a block's unary segment spans
    many 64-word chunks."""
    L = 300
    offs = np.arange(L + 1, dtype=np.uint64)
    values = np.random.default_rng(940).integers(0, 5000, size=L).astype(np.uint64)
    table = [0] * 65
    g = _encode(shock, values, offs, table)
    o = oracle_mod.rice_encode(values, offs, np.array(table, np.uint8))
    assert g[0] == 0 and g[4] == o[4] and (g[2] == o[2]).all() and (g[3] == o[3]).all()
    rc, back = shock.rice_decode(_dev(g[1]), _dev(g[2]), _dev(g[3]), _dev(offs), table)
    torch.cuda.synchronize()
    assert rc == 0 and (_host(back) == values).all()


def test_rice_errors(shock):
    offs = np.array([0, 1], np.uint64)
    table = [3] * 65
    rc, *_ = _encode(shock, np.array([8 << 32], np.uint64), offs, table)
    assert rc == shock.SHOCK_EINVAL
    bad = [57] + [0] * 64
    rc, *_ = _encode(shock, np.array([1], np.uint64), offs, bad)
    assert rc == shock.SHOCK_EINVAL
    rc, *_ = _encode(shock, np.zeros(0, np.uint64), np.zeros(1, np.uint64), table)
    assert rc == 0


def test_rice_codes_of_real_seeds(shock, oracle_mod):
    """The fixed48 batch's seeds with the plain table: streams equal the
    oracle's, decoding restores them, and the mean code length matches the
    expected length for the exact success probability (Section 4's
    0.44n + o(n) bits) within 5 standard errors."""
    from paper_2308_09561_amd import rice
    import theory as T
    keys, offs = make_workload("fixed48")
    k, o = _dev(keys), _dev(offs)
    print("[gpu] fixed48 search + rice", flush=True)
    rc, s, _ = shock.leaf_search(k, o)
    assert rc == 0
    table = rice.plain_table()
    rc, fx, un, idx, bits = shock.rice_encode(s, o, table)
    assert rc == 0
    seeds = _host(s)
    want = oracle_mod.rice_encode(seeds, offs, np.array(table, np.uint8))
    assert want[4] == bits and (_host(fx) == want[1]).all() and (_host(un) == want[2]).all()
    assert (_host(idx) == want[3]).all()
    rc, back = shock.rice_decode(fx, un, idx, o, table)
    torch.cuda.synchronize()
    assert rc == 0 and (_host(back) == seeds).all()
    L = len(offs) - 1
    lengths = table[48] + 1 + (seeds >> np.uint64(table[48])).astype(np.float64)
    p = float(T.p_accept(48))
    assert abs(sum(bits) / L - rice.expected_length(table[48], p)) < 5 * lengths.std() / math.sqrt(L)
