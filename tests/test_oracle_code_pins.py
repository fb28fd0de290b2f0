"""Pins for the oracle's leaf query (Section 4: a key x is answered by
h_{s, f(x)}(x)) and its Golomb-Rice seed codes (Section 4: 0.44n + o(n) bits
per seed in expectation), and for the package's Rice-parameter helper.  No
GPU."""
import math

import numpy as np
import pytest

import theory as T
from workloads import fixed_leaves, splitmix64, uneven_leaves


# ---------------------------------------------------------------- query ----

def _is_bijection(pos, offs):
    for j in range(len(offs) - 1):
        a, b = int(offs[j]), int(offs[j + 1])
        if sorted(int(x) for x in pos[a:b]) != list(range(a, b)):
            return False
    return True


def test_query_is_a_minimal_perfect_hash_on_every_leaf(oracle_mod):
    """Eq. pseudoforests-orientable: the seed's orientation makes the leaf's
    keys land on distinct cells, so the query maps the batch one-to-one onto
    [0, N)."""
    keys, offs = uneven_leaves(300, 0, 24, 801, 802)
    rc, s, f = oracle_mod.leaf_search(keys, offs)
    assert rc == 0
    rc, pos = oracle_mod.leaf_query(keys, offs, s, f)
    assert rc == 0
    assert _is_bijection(pos, offs)
    assert sorted(pos.tolist()) == list(range(int(offs[-1])))


def test_query_breaks_when_any_single_choice_flips(oracle_mod):
    """All n cells are taken, and a key's other slot is a different cell, so
    moving any one key there collides with the key that holds it."""
    keys, offs = fixed_leaves(12, 16, 803)
    rc, s, f = oracle_mod.leaf_search(keys, offs)
    for j in range(12):
        sub = offs[j:j + 2]
        for i in range(16):
            g = f[j:j + 1] ^ np.uint64(1 << i)
            _, pos = oracle_mod.leaf_query(keys, sub, s[j:j + 1], g)
            assert not _is_bijection(pos - sub[0] + sub[0], sub), (j, i)


def test_query_of_tiny_and_missing_leaves(oracle_mod):
    keys = splitmix64(804, 3)
    offs = np.array([0, 0, 1, 3], dtype=np.uint64)
    rc, s, f = oracle_mod.leaf_search(keys, offs)
    rc, pos = oracle_mod.leaf_query(keys, offs, s, f)
    assert pos[0] == 0 and sorted(pos[1:].tolist()) == [1, 2]
    s2 = s.copy()
    s2[2] = np.uint64(0xFFFFFFFFFFFFFFFF)
    _, pos = oracle_mod.leaf_query(keys, offs, s2, f)
    assert pos[1] == np.uint64(0xFFFFFFFFFFFFFFFF) and pos[2] == np.uint64(0xFFFFFFFFFFFFFFFF)


def test_rf_query_is_a_minimal_perfect_hash(oracle_mod):
    keys, offs = uneven_leaves(120, 2, 40, 805, 806)
    rc, s, r, f = oracle_mod.rf_leaf_search(keys, offs)
    assert rc == 0
    rc, pos = oracle_mod.rf_leaf_query(keys, offs, s, r, f)
    assert rc == 0 and _is_bijection(pos, offs)
    # the plain query of the same seeds (rotation ignored) is not a bijection in general
    _, plain = oracle_mod.leaf_query(keys, offs, s, f)
    assert not _is_bijection(plain, offs)


# ------------------------------------------------------------ Rice codes ----

def _bits(words, count):
    return "".join(str((int(words[p // 64]) >> (p % 64)) & 1) for p in range(count))


def test_rice_hand_example(oracle_mod):
    """Four 3-key leaves, k = 1, values 0, 1, 5, 2.  Worked by hand from the
    code's definition: low bits 0, 1, 1, 0 give the fixed stream 0110;
    quotients 0, 0, 2, 1 give the unary stream 1 | 1 | 001 | 01.  As 64-bit
    words, least significant bit first: fixed 0b0110 = 0x6, unary 0b1010011
    = 0x53."""
    offs = np.array([0, 3, 6, 9, 12], dtype=np.uint64)
    k = np.zeros(65, np.uint8)
    k[3] = 1
    rc, fx, un, idx, bits = oracle_mod.rice_encode(np.array([0, 1, 5, 2], np.uint64), offs, k)
    assert rc == 0 and bits == (4, 7)
    assert _bits(fx, 4) == "0110" and _bits(un, 7) == "1100101"
    assert int(fx[0]) == 0x6 and int(un[0]) == 0x53
    assert idx.tolist() == [0, 0, 4, 7]
    rc, v = oracle_mod.rice_decode(fx, un, offs, k)
    assert rc == 0 and v.tolist() == [0, 1, 5, 2]


def test_rice_textbook_codes(oracle_mod):
    """Rice codes of 0..11 with k = 2 (divisor 4): v = 4q + r is q zeros, a
    one, and r in two bits, least significant first."""
    k = np.zeros(65, np.uint8)
    k[1] = 2
    for v in range(12):
        rc, fx, un, _, bits = oracle_mod.rice_encode(np.array([v], np.uint64), np.array([0, 1], np.uint64), k)
        q, r = divmod(v, 4)
        assert bits == (2, q + 1)
        assert _bits(un, q + 1) == "0" * q + "1"
        assert _bits(fx, 2) == f"{r & 1}{r >> 1}"


def test_rice_roundtrip_and_index(oracle_mod):
    rng = np.random.default_rng(807)
    L = 1000
    sizes = rng.integers(0, 65, size=L)
    offs = np.zeros(L + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offs[1:])
    k = rng.integers(0, 57, size=65).astype(np.uint8)
    k[0] = 0
    k[5] = 56
    q = rng.geometric(0.4, size=L) - 1
    low = np.array([int(rng.integers(0, 1 << int(k[n]), dtype=np.uint64)) if k[n] else 0 for n in sizes],
                   dtype=np.uint64)
    values = (q.astype(np.uint64) << k[sizes].astype(np.uint64)) | low
    rc, fx, un, idx, bits = oracle_mod.rice_encode(values, offs, k)
    assert rc == 0
    assert bits == (int(k[sizes].astype(np.int64).sum()), int((q + 1).sum()))
    rc, back = oracle_mod.rice_decode(fx, un, offs, k)
    assert rc == 0 and (back == values).all()
    # index: partial sums of the lengths at every 64th leaf and at the end
    fl = np.concatenate([[0], np.cumsum(k[sizes].astype(np.int64))])
    ul = np.concatenate([[0], np.cumsum(q + 1)])
    for m in range((L + 63) // 64):
        assert (int(idx[2 * m]), int(idx[2 * m + 1])) == (int(fl[64 * m]), int(ul[64 * m]))
    m = (L + 63) // 64
    assert (int(idx[2 * m]), int(idx[2 * m + 1])) == (int(fl[-1]), int(ul[-1]))


def test_rice_rejects_huge_quotients_and_short_streams(oracle_mod):
    k = np.zeros(65, np.uint8)
    k[1] = 3
    offs = np.array([0, 1], np.uint64)
    rc, *_ = oracle_mod.rice_encode(np.array([8 << 32], np.uint64), offs, k)
    assert rc == oracle_mod.EINVAL
    rc, *_ = oracle_mod.rice_encode(np.array([(8 << 32) - 1], np.uint64), offs, k, fixed_words=1, unary_words=1)
    assert rc == oracle_mod.EINVAL  # needs 2^32 unary bits


@pytest.mark.parametrize("p", [0.5, 0.1, 0.01, 1e-3])
def test_rice_mean_length_on_geometric_values(oracle_mod, p):
    """The mean code length of geometric values equals k + 1 + t/(1-t),
    t = (1-p)^(2^k), within 5 standard errors (numpy's geometric sampler as
    the source)."""
    from paper_2308_09561_amd import rice
    rng = np.random.default_rng(int(1 / p))
    L = 20000
    values = (rng.geometric(p, size=L) - 1).astype(np.uint64)
    kk = rice.optimal_k(p)
    k = np.zeros(65, np.uint8)
    k[1] = kk
    offs = np.arange(L + 1, dtype=np.uint64)
    rc, _, _, _, bits = oracle_mod.rice_encode(values, offs, k)
    lengths = kk + 1 + (values >> np.uint64(kk)).astype(np.float64)
    assert rc == 0 and sum(bits) == int(lengths.sum())
    mean, se = lengths.mean(), lengths.std() / math.sqrt(L)
    assert abs(mean - rice.expected_length(kk, p)) < 5 * se + 1e-9


# -------------------------------------------------- Rice parameter helper ----

@pytest.mark.parametrize("n", [2, 3, 5, 8, 13, 24, 40, 48])
def test_helper_success_probability_matches_closed_form(n):
    from paper_2308_09561_amd import rice
    assert rice.success_probability(n) == pytest.approx(float(T.p_accept(n)), rel=1e-12)


@pytest.mark.parametrize("p", [0.9, 0.5, 0.2, 0.05, 1e-2, 1e-4, 1e-6, 2.3e-6, 1e-8])
def test_optimal_rice_is_within_one_bit_of_entropy(p):
    """Golomb codes are optimal prefix codes for geometric sources (Gallager
    and Van Voorhis 1975), hence within one bit of the entropy; Rice codes
    (power-of-two divisors) lose only a small fraction of a bit more.  Also
    checks the chosen k is a minimum by brute force over all k."""
    from paper_2308_09561_amd import rice
    k = rice.optimal_k(p)
    e = rice.expected_length(k, p)
    h = rice.geometric_entropy(p)
    assert h - 1e-9 <= e <= h + 1.0
    assert all(rice.expected_length(j, p) >= e - 1e-12 for j in range(0, 57))


def test_seed_code_grows_by_0_44_bits_per_key():
    """Section 4: the Golomb-Rice coded seed takes 0.44n + o(n) bits.  With
    the exact per-seed success probability of the plain search, the expected
    code length grows by log2(e/2) = 0.4427 bits per key, less the
    derivative of the polynomial factor (the mean seed is ~ (e/2)^n / sqrt(n)
    by Section 5's measurements, i.e. -0.5 / (n ln 2) bits per key)."""
    from paper_2308_09561_amd import rice
    lens = {n: rice.expected_length(rice.optimal_k(float(T.p_accept(n))), float(T.p_accept(n)))
            for n in (24, 32, 40, 48, 56, 64)}
    for a, b in ((24, 40), (32, 48), (48, 64)):
        slope = (lens[b] - lens[a]) / (b - a)
        mid = (a + b) / 2
        assert abs(slope - (math.log2(math.e / 2) - 0.5 / (mid * math.log(2)))) < 0.02, (a, b, slope)
    # and a code is about the entropy of the seed plus at most one bit
    for n, e in lens.items():
        p = float(T.p_accept(n))
        assert rice.geometric_entropy(p) <= e <= rice.geometric_entropy(p) + 1


def test_real_seed_codes_match_the_expected_length(oracle_mod):
    """The whole chain: the oracle's seeds of 20-key leaves are geometric with
    the exact success probability, so their Rice codes average the expected
    length within 5 standard errors."""
    from paper_2308_09561_amd import rice
    n, L = 20, 4000
    keys, offs = fixed_leaves(L, n, 808)
    rc, s, _ = oracle_mod.leaf_search(keys, offs)
    table = rice.plain_table()
    k = np.array(table, np.uint8)
    rc, _, _, _, bits = oracle_mod.rice_encode(s, offs, k)
    lengths = table[n] + 1 + (s >> np.uint64(table[n])).astype(np.float64)
    p = float(T.p_accept(n))
    assert rc == 0 and sum(bits) == int(lengths.sum())
    assert abs(lengths.mean() - rice.expected_length(table[n], p)) < 5 * lengths.std() / math.sqrt(L)
