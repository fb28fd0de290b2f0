"""CPU oracle for the ShockHash leaf seed search -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The GPU library never imports, links or calls it.  The C
source (shock_oracle.c, definitions in shock_oracle.h) is compiled with gcc
into liboracle.so next to this file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("shock_oracle.c", "shock_oracle_mphf.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
EINVAL = -1
ENOTFOUND = -2
NOT_FOUND_SEED = np.uint64(0xFFFFFFFFFFFFFFFF)
DEFAULT_MAX_SEED = 1 << 32

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation flags)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def build_sanitized(path: str) -> str:
    """The same sources built with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only; any report aborts the process).  Loading it needs the
    ASan runtime preloaded; tests/test_oracle_sanitized.py does that in a
    child process and points SHOCK_ORACLE_LIB at this file."""
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           "-o", path, *_SRCS, "-lm"])
    return path


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("SHOCK_ORACLE_LIB") or _LIB
        if path == _LIB and (not os.path.exists(_LIB) or
                             max(os.path.getmtime(f) for f in _SRCS + [os.path.join(_HERE, "shock_oracle.h")])
                             > os.path.getmtime(_LIB)):
            build(force=True)  # missing, or older than its sources
        L = ctypes.CDLL(path)
        L.shock_oracle_fmix64.restype = ctypes.c_uint64
        L.shock_oracle_fmix64.argtypes = [ctypes.c_uint64]
        L.shock_oracle_slots.restype = None
        L.shock_oracle_slots.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, _u32p, _u32p]
        L.shock_oracle_is_pseudoforest.restype = ctypes.c_int
        L.shock_oracle_is_pseudoforest.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _u32p, _u32p]
        L.shock_oracle_orientation.restype = ctypes.c_int
        L.shock_oracle_orientation.argtypes = [ctypes.c_uint32, _u32p, _u32p, _u64p]
        L.shock_oracle_leaf_search.restype = ctypes.c_int
        L.shock_oracle_leaf_search.argtypes = [_u64p, _u64p, ctypes.c_uint64, _u64p, _u64p,
                                               ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int]
        L.shock_oracle_verify.restype = ctypes.c_int
        L.shock_oracle_verify.argtypes = [_u64p, _u64p, ctypes.c_uint64, _u64p, _u64p, ctypes.c_uint64,
                                          ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint8)]
        L.shock_oracle_side.restype = ctypes.c_int
        L.shock_oracle_side.argtypes = [ctypes.c_uint64]
        L.shock_oracle_rf_slots.restype = None
        L.shock_oracle_rf_slots.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_uint32, _u32p, _u32p]
        L.shock_oracle_rf_leaf_search.restype = ctypes.c_int
        L.shock_oracle_rf_leaf_search.argtypes = [_u64p, _u64p, ctypes.c_uint64, _u64p, _u32p, _u64p,
                                                  ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int]
        L.shock_oracle_leaf_query.restype = ctypes.c_int
        L.shock_oracle_leaf_query.argtypes = [_u64p, _u64p, ctypes.c_uint64, _u64p, _u64p, _u64p]
        L.shock_oracle_rf_leaf_query.restype = ctypes.c_int
        L.shock_oracle_rf_leaf_query.argtypes = [_u64p, _u64p, ctypes.c_uint64, _u64p, _u32p, _u64p,
                                                 ctypes.c_uint32, _u64p]
        L.shock_oracle_rice_encode.restype = ctypes.c_int
        L.shock_oracle_rice_encode.argtypes = [_u64p, _u64p, ctypes.c_uint64, _u8p, _u64p, ctypes.c_uint64, _u64p,
                                               ctypes.c_uint64, _u64p, _u64p]
        L.shock_oracle_rice_decode.restype = ctypes.c_int
        L.shock_oracle_rice_decode.argtypes = [_u64p, _u64p, _u64p, ctypes.c_uint64, _u8p, _u64p]
        L.shock_oracle_mphf_split.restype = ctypes.c_int
        L.shock_oracle_mphf_split.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                              ctypes.c_uint32, ctypes.c_uint64, _u64p, _u64p, _u32p, _u8p,
                                              ctypes.c_uint64, _u64p, _u64p, _u64p]
        L.shock_oracle_xor_segment.restype = ctypes.c_uint64
        L.shock_oracle_xor_segment.argtypes = [ctypes.c_uint64]
        L.shock_oracle_xor_build.restype = ctypes.c_int
        L.shock_oracle_xor_build.argtypes = [_u64p, _u8p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, _u64p,
                                             _u8p]
        L.shock_oracle_xor_get.restype = ctypes.c_int
        L.shock_oracle_xor_get.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint64, _u8p, _u8p]
        L.shock_oracle_leaf_size_base.restype = ctypes.c_uint32
        L.shock_oracle_leaf_size_base.argtypes = [ctypes.c_uint64, ctypes.c_uint32]
        L.shock_oracle_gf2_solve.restype = ctypes.c_int
        L.shock_oracle_gf2_solve.argtypes = [_u64p, _u8p, ctypes.c_uint64, ctypes.c_uint64, _u8p]
        L.shock_oracle_ribbon_cols.restype = ctypes.c_uint64
        L.shock_oracle_ribbon_cols.argtypes = [ctypes.c_uint64]
        L.shock_oracle_ribbon_row.restype = None
        L.shock_oracle_ribbon_row.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, _u64p, _u64p]
        L.shock_oracle_ribbon_build.restype = ctypes.c_int
        L.shock_oracle_ribbon_build.argtypes = [_u64p, _u8p, ctypes.c_uint64, ctypes.c_uint32,
                                                ctypes.POINTER(ctypes.c_uint32), _u8p]
        L.shock_oracle_ribbon_get.restype = ctypes.c_uint8
        L.shock_oracle_ribbon_get.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, _u8p]
        L.shock_oracle_mphf_ribbon.restype = ctypes.c_int
        L.shock_oracle_mphf_ribbon.argtypes = [_u64p, _u8p, ctypes.c_uint64, _u64p, ctypes.c_uint32, _u8p, _u64p, _u8p]
        L.shock_oracle_mphf_query.restype = ctypes.c_int
        L.shock_oracle_mphf_query.argtypes = [_u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                              ctypes.c_uint64, _u64p, _u64p, _u32p, _u8p, _u64p, ctypes.c_int,
                                              ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64, _u8p, _u64p, _u8p,
                                              _u64p]
        L.shock_oracle_bip_pair_rank.restype = ctypes.c_uint64
        L.shock_oracle_bip_pair_rank.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.shock_oracle_bip_slots.restype = None
        L.shock_oracle_bip_slots.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, _u32p, _u32p]
        L.shock_oracle_bip_leaf_search.restype = ctypes.c_int
        L.shock_oracle_bip_leaf_search.argtypes = [_u64p, _u64p, ctypes.c_uint64, _u64p, _u64p, _u64p,
                                                   ctypes.c_uint64, ctypes.c_int]
        L.shock_oracle_seed_stats.restype = None
        L.shock_oracle_seed_stats.argtypes = [_u64p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                              _u64p, _u64p, _u64p]
        _lib = L
    return _lib


def _p64(a: np.ndarray):
    return a.ctypes.data_as(_u64p)


def _p32(a: np.ndarray):
    return a.ctypes.data_as(_u32p)


def fmix64(k: int) -> int:
    return int(lib().shock_oracle_fmix64(k & 0xFFFFFFFFFFFFFFFF))


def slots(key: int, seed: int, n: int) -> tuple[int, int]:
    a = ctypes.c_uint32()
    b = ctypes.c_uint32()
    lib().shock_oracle_slots(key & 0xFFFFFFFFFFFFFFFF, seed & 0xFFFFFFFFFFFFFFFF, n,
                             ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def leaf_slots(keys, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """h0, h1 arrays of one leaf under one seed."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    n = len(keys)
    h = [slots(int(x), seed, n) for x in keys]
    return (np.array([p[0] for p in h], dtype=np.uint32), np.array([p[1] for p in h], dtype=np.uint32))


def is_pseudoforest(n: int, h0, h1) -> bool:
    h0 = np.ascontiguousarray(h0, dtype=np.uint32)
    h1 = np.ascontiguousarray(h1, dtype=np.uint32)
    return bool(lib().shock_oracle_is_pseudoforest(n, len(h0), _p32(h0), _p32(h1)))


def orientation(n: int, h0, h1):
    """Canonical orientation mask, or None if the graph is not a pseudoforest."""
    h0 = np.ascontiguousarray(h0, dtype=np.uint32)
    h1 = np.ascontiguousarray(h1, dtype=np.uint32)
    f = ctypes.c_uint64()
    rc = lib().shock_oracle_orientation(n, _p32(h0), _p32(h1), ctypes.byref(f))
    return None if rc != OK else int(f.value)


def leaf_search(keys, offsets, start_seed: int = 0, max_seed: int = DEFAULT_MAX_SEED, use_filter: bool = True):
    """(status, seeds uint64[L], orient uint64[L]) for a CSR batch (host arrays)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    L = max(len(offsets) - 1, 0)
    seeds = np.zeros(L, dtype=np.uint64)
    orient = np.zeros(L, dtype=np.uint64)
    rc = lib().shock_oracle_leaf_search(_p64(keys) if keys.size else None, _p64(offsets) if offsets.size else None,
                                        L, _p64(seeds), _p64(orient), start_seed, max_seed, int(use_filter))
    return rc, seeds, orient


def verify(keys, offsets, seeds, orient, start_seed: int = 0, window: int = 64):
    """Per-leaf flags (see shock_oracle_verify): 0 = claimed seed qualifies, its
    orientation is canonical and no seed in the window below it qualifies."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    orient = np.ascontiguousarray(orient, dtype=np.uint64)
    L = len(offsets) - 1
    flags = np.zeros(max(L, 1), dtype=np.uint8)
    rc = lib().shock_oracle_verify(_p64(keys), _p64(offsets), L, _p64(seeds), _p64(orient), start_seed, window,
                                   flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc != OK:
        raise ValueError("malformed batch")
    return flags[:L]


def _leaf_chunks(offsets, parts):
    L = len(offsets) - 1
    step = max(1, (L + parts - 1) // parts)
    return [(a, min(a + step, L)) for a in range(0, L, step)]


def parallel(fn, keys, offsets, *per_leaf, threads: int | None = None, **kw):
    """Run a per-leaf oracle function over leaf ranges on several host threads.
    Each leaf is still processed by the single-threaded oracle code; the
    driver only partitions the batch (ctypes releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    threads = threads or min(16, os.cpu_count() or 1)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    chunks = _leaf_chunks(offsets, threads * 4)

    def run(ab):
        a, b = ab
        sub_off = offsets[a:b + 1]
        args = [x[a:b] for x in per_leaf]
        return fn(keys, sub_off, *args, **kw)

    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(run, chunks))


def seed_stats(keys, s0: int, count: int):
    """(cover, pseudoforest, h0_bijective) counts over seeds s0 .. s0+count-1 of one leaf."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    lib().shock_oracle_seed_stats(_p64(keys), len(keys), s0, count, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def side(key: int) -> int:
    return int(lib().shock_oracle_side(key & 0xFFFFFFFFFFFFFFFF))


def rf_slots(key: int, seed: int, rot: int, k: int, n: int) -> tuple[int, int]:
    a = ctypes.c_uint32()
    b = ctypes.c_uint32()
    lib().shock_oracle_rf_slots(key & 0xFFFFFFFFFFFFFFFF, seed & 0xFFFFFFFFFFFFFFFF, rot, k, n,
                                ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def rf_leaf_search(keys, offsets, start_seed: int = 0, max_seed: int = DEFAULT_MAX_SEED, partial_k: int = 0,
                   use_filter: bool = True):
    """(status, seeds uint64[L], rot uint32[L], orient uint64[L]) of the rotation-fitting search."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    L = max(len(offsets) - 1, 0)
    seeds = np.zeros(L, dtype=np.uint64)
    rot = np.zeros(L, dtype=np.uint32)
    orient = np.zeros(L, dtype=np.uint64)
    rc = lib().shock_oracle_rf_leaf_search(_p64(keys) if keys.size else None, _p64(offsets) if offsets.size else None,
                                           L, _p64(seeds), _p32(rot), _p64(orient), start_seed, max_seed,
                                           partial_k, int(use_filter))
    return rc, seeds, rot, orient


def leaf_query(keys, offsets, seeds, orient):
    """(status, positions uint64[N]): the MPHF value of every key (Section 4's query)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    orient = np.ascontiguousarray(orient, dtype=np.uint64)
    L = max(len(offsets) - 1, 0)
    pos = np.zeros(max(int(offsets[-1]) if len(offsets) else 0, 1), dtype=np.uint64)
    rc = lib().shock_oracle_leaf_query(_p64(keys) if keys.size else None, _p64(offsets), L, _p64(seeds),
                                       _p64(orient), _p64(pos))
    return rc, pos[:int(offsets[-1]) if len(offsets) else 0]


def rf_leaf_query(keys, offsets, seeds, rot, orient, partial_k: int = 0):
    """(status, positions uint64[N]) under rotation fitting."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    rot = np.ascontiguousarray(rot, dtype=np.uint32)
    orient = np.ascontiguousarray(orient, dtype=np.uint64)
    L = max(len(offsets) - 1, 0)
    pos = np.zeros(max(int(offsets[-1]) if len(offsets) else 0, 1), dtype=np.uint64)
    rc = lib().shock_oracle_rf_leaf_query(_p64(keys) if keys.size else None, _p64(offsets), L, _p64(seeds),
                                          _p32(rot), _p64(orient), partial_k, _p64(pos))
    return rc, pos[:int(offsets[-1]) if len(offsets) else 0]


def rice_encode(values, offsets, k_by_n, fixed_words=None, unary_words=None):
    """(status, fixed uint64[], unary uint64[], index uint64[], (fixed_bits, unary_bits)).

    Without explicit capacities the streams are sized from a first call."""
    values = np.ascontiguousarray(values, dtype=np.uint64)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    k = np.ascontiguousarray(k_by_n, dtype=np.uint8)
    assert k.size == 65
    L = max(len(offsets) - 1, 0)
    bits = np.zeros(2, dtype=np.uint64)
    if fixed_words is None or unary_words is None:
        rc = lib().shock_oracle_rice_encode(_p64(values) if values.size else None, _p64(offsets), L,
                                            k.ctypes.data_as(_u8p), None, 0, None, 0, None, _p64(bits))
        fixed_words = int((bits[0] + 63) // 64)
        unary_words = int((bits[1] + 63) // 64)
    fixed = np.zeros(max(fixed_words, 1), dtype=np.uint64)
    unary = np.zeros(max(unary_words, 1), dtype=np.uint64)
    index = np.zeros(2 * ((L + 63) // 64 + 1), dtype=np.uint64)
    rc = lib().shock_oracle_rice_encode(_p64(values) if values.size else None, _p64(offsets), L,
                                        k.ctypes.data_as(_u8p), _p64(fixed), fixed_words, _p64(unary), unary_words,
                                        _p64(index), _p64(bits))
    return rc, fixed[:fixed_words], unary[:unary_words], index, (int(bits[0]), int(bits[1]))


def rice_decode(fixed, unary, offsets, k_by_n):
    """(status, values uint64[L]) decoded from the two streams alone."""
    fixed = np.ascontiguousarray(fixed, dtype=np.uint64)
    unary = np.ascontiguousarray(unary, dtype=np.uint64)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    k = np.ascontiguousarray(k_by_n, dtype=np.uint8)
    L = max(len(offsets) - 1, 0)
    values = np.zeros(max(L, 1), dtype=np.uint64)
    f = fixed if fixed.size else np.zeros(1, dtype=np.uint64)
    rc = lib().shock_oracle_rice_decode(_p64(f), _p64(unary) if unary.size else None, _p64(offsets), L,
                                        k.ctypes.data_as(_u8p), _p64(values))
    return rc, values[:L]


# ---- flat ShockHash MPHF ------------------------------------------------------

def _p8(a: np.ndarray):
    return a.ctypes.data_as(_u8p)


def mphf_buckets(n_keys: int, bucket_size: int) -> int:
    return 1 if n_keys == 0 or bucket_size == 0 else -(-n_keys // bucket_size)


def mphf_split(keys, bucket_size: int = 3000, leaf_target: int = 40, leaf_max: int = 56):
    """(status, dict) of the bucket/leaf layout: bucket_offset, leaf_base,
    sigma, leaf_sizes, leaf_keys, key_index, leaf_offsets (global key offsets)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    N = keys.size
    B = mphf_buckets(N, bucket_size)
    cap = B + N // max(leaf_target, 1) + 1
    bo = np.zeros(B + 1, np.uint64)
    lb = np.zeros(B + 1, np.uint64)
    sg = np.zeros(B, np.uint32)
    sz = np.zeros(max(cap, 1), np.uint8)
    lk = np.zeros(max(N, 1), np.uint64)
    ki = np.zeros(max(N, 1), np.uint64)
    nl = ctypes.c_uint64()
    rc = lib().shock_oracle_mphf_split(_p64(keys) if N else None, N, bucket_size, leaf_target, leaf_max, B,
                                       _p64(bo), _p64(lb), _p32(sg), _p8(sz), cap, _p64(lk), _p64(ki),
                                       ctypes.byref(nl))
    L = int(nl.value)
    sizes = sz[:L]
    offs = np.zeros(L + 1, np.uint64)
    np.cumsum(sizes.astype(np.uint64), out=offs[1:])
    return rc, {"n_buckets": B, "bucket_offset": bo, "leaf_base": lb, "sigma": sg, "leaf_sizes": sizes,
                "leaf_keys": lk[:N], "key_index": ki[:N], "leaf_offsets": offs, "n_leaves": L}


RETRIEVAL_RIBBON = 0
RETRIEVAL_XOR = 1
RIBBON_MAX_SEEDS = 256


def leaf_size_base(m: int, n_leaves: int) -> int:
    return int(lib().shock_oracle_leaf_size_base(m, n_leaves))


def gf2_solve(rows, b, cols: int):
    """(solvable, z uint8[cols]) of the system rows (uint64[m][ceil(cols/64)],
    bit c = column c) x = b, z the canonical solution (non-pivot columns 0)."""
    rows = np.ascontiguousarray(rows, dtype=np.uint64)
    m = rows.shape[0] if rows.ndim == 2 else 0
    b = np.ascontiguousarray(b, dtype=np.uint8)
    z = np.zeros(max(cols, 1), np.uint8)
    ok = lib().shock_oracle_gf2_solve(_p64(rows.reshape(-1)) if m else None, _p8(b) if m else None, m, cols, _p8(z))
    if ok < 0:
        raise MemoryError("gf2_solve")
    return bool(ok), z[:cols]


def ribbon_cols(m: int) -> int:
    return int(lib().shock_oracle_ribbon_cols(m))


def ribbon_row(key: int, rseed: int, cols: int) -> tuple[int, int]:
    s, c = ctypes.c_uint64(), ctypes.c_uint64()
    lib().shock_oracle_ribbon_row(key & 0xFFFFFFFFFFFFFFFF, rseed, cols, ctypes.byref(s), ctypes.byref(c))
    return s.value, c.value


def ribbon_build(keys, values, max_seeds: int = RIBBON_MAX_SEEDS):
    """(status, rseed, z uint8[cols]) of one bucket's ribbon system."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    values = np.ascontiguousarray(values, dtype=np.uint8)
    m = keys.size
    z = np.zeros(max(ribbon_cols(m), 1), np.uint8)
    r = ctypes.c_uint32()
    rc = lib().shock_oracle_ribbon_build(_p64(keys) if m else None, _p8(values) if m else None, m, max_seeds,
                                         ctypes.byref(r), _p8(z))
    return rc, int(r.value), z[:ribbon_cols(m)]


def ribbon_get(key: int, rseed: int, cols: int, z) -> int:
    return int(lib().shock_oracle_ribbon_get(key & 0xFFFFFFFFFFFFFFFF, rseed, cols,
                                             _p8(np.ascontiguousarray(z, np.uint8))))


def mphf_ribbon(leaf_keys, values, bucket_offset, max_seeds: int = RIBBON_MAX_SEEDS):
    """(status, rseed uint8[B], bit_offset uint64[B+1], z uint8[total]) of every bucket's system."""
    lk = np.ascontiguousarray(leaf_keys, dtype=np.uint64)
    v = np.ascontiguousarray(values, dtype=np.uint8)
    bo = np.ascontiguousarray(bucket_offset, dtype=np.uint64)
    B = bo.size - 1
    total = sum(ribbon_cols(int(bo[b + 1] - bo[b])) for b in range(B))
    rseed = np.zeros(max(B, 1), np.uint8)
    boff = np.zeros(B + 1, np.uint64)
    z = np.zeros(max(total, 1), np.uint8)
    rc = lib().shock_oracle_mphf_ribbon(_p64(lk) if lk.size else None, _p8(v) if v.size else None, B, _p64(bo),
                                        max_seeds, _p8(rseed), _p64(boff), _p8(z))
    return rc, rseed[:B], boff, z[:total]


def xor_segment(n_keys: int) -> int:
    return int(lib().shock_oracle_xor_segment(n_keys))


def xor_build(keys, values, rho_start: int = 0, max_tries: int = 64):
    """(status, rho, z uint8[3 * seg])."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    values = np.ascontiguousarray(values, dtype=np.uint8)
    N = keys.size
    z = np.zeros(3 * xor_segment(N), np.uint8)
    rho = ctypes.c_uint64()
    rc = lib().shock_oracle_xor_build(_p64(keys) if N else None, _p8(values) if N else None, N, rho_start,
                                      max_tries, ctypes.byref(rho), _p8(z))
    return rc, int(rho.value), z


def xor_get(keys, rho: int, z):
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    out = np.zeros(max(keys.size, 1), np.uint8)
    lib().shock_oracle_xor_get(_p64(keys), keys.size, rho, _p8(np.ascontiguousarray(z, np.uint8)), _p8(out))
    return out[:keys.size]


def mphf_build(keys, bucket_size: int = 3000, leaf_target: int = 40, leaf_max: int = 56, rf: bool = False,
               partial_k: int = 0, bip: bool = False, retrieval: int = RETRIEVAL_RIBBON):
    """The whole flat MPHF: layout, leaf seeds and orientations (the leaf
    search, rotation fitting with values s * n + r, or with bip the bipartite
    search with values the rank of the pair (a, b) in its search order), the
    retrieval of each key's choice (per-bucket ribbon systems, or the XOR
    system), and every key's position (index i of the input keys ->
    positions[i]).  With bip the positions come from the oracle's own query
    (shock_oracle_mphf_query) over the built structure."""
    rc, lay = mphf_split(keys, bucket_size, leaf_target, leaf_max)
    if rc != OK:
        return rc, None
    lk, offs = lay["leaf_keys"], lay["leaf_offsets"]
    if bip:
        rc, pa, pb, orient = bip_leaf_search(lk, offs)
        seeds = np.array([bip_pair_rank(int(x), int(y)) for x, y in zip(pa, pb)], dtype=np.uint64)
    elif rf:
        rc, s_rf, rot, orient = rf_leaf_search(lk, offs, partial_k=partial_k)
        sizes_u = lay["leaf_sizes"].astype(np.uint64)
        seeds = np.where(sizes_u >= 2, s_rf * sizes_u + rot.astype(np.uint64), s_rf)
    else:
        rc, seeds, orient = leaf_search(lk, offs)
    if rc != OK:
        return rc, None
    sizes = lay["leaf_sizes"].astype(np.int64)
    leaf_of_key = np.repeat(np.arange(lay["n_leaves"]), sizes)
    idx_in_leaf = np.arange(lk.size) - offs[:-1].astype(np.int64)[leaf_of_key] if lk.size else np.zeros(0, np.int64)
    f = ((orient[leaf_of_key] >> idx_in_leaf.astype(np.uint64)) & np.uint64(1)).astype(np.uint8) if lk.size \
        else np.zeros(0, np.uint8)
    rseed, rbit = np.zeros(0, np.uint8), np.zeros(1, np.uint64)
    rho = 0
    if retrieval == RETRIEVAL_RIBBON:
        rc, rseed, rbit, z = mphf_ribbon(lk, f, lay["bucket_offset"])
    else:
        rc, rho, z = xor_build(lk, f)
    if rc != OK:
        return rc, None
    lay.update({"seeds": seeds, "orient": orient, "choice": f, "rho": rho, "z": z, "retrieval": retrieval,
                "rseed": rseed, "rbit_offset": rbit,
                "leaf_target": leaf_target, "leaf_max": leaf_max, "bucket_size": bucket_size, "rf": bool(rf),
                "partial_k": partial_k, "bip": bool(bip)})
    positions = np.zeros(lk.size, np.uint64)
    if bip:
        rc, pos_leaf_order = mphf_query(lay, lk)
        if rc != OK:
            return rc, None
    elif rf:
        _, pos_leaf_order = rf_leaf_query(lk, offs, s_rf, rot, orient, partial_k=partial_k)
    else:
        _, pos_leaf_order = leaf_query(lk, offs, seeds, orient)
    positions[lay["key_index"].astype(np.int64)] = pos_leaf_order
    lay["positions"] = positions
    return OK, lay


def mphf_query(lay, queries):
    """(status, positions) of query keys through the stored structure."""
    q = np.ascontiguousarray(queries, dtype=np.uint64)
    out = np.zeros(max(q.size, 1), np.uint64)
    N = lay["leaf_keys"].size
    rc = lib().shock_oracle_mphf_query(_p64(q), q.size, N, lay["leaf_target"], lay["n_buckets"],
                                       _p64(lay["bucket_offset"]), _p64(lay["leaf_base"]), _p32(lay["sigma"]),
                                       _p8(np.ascontiguousarray(lay["leaf_sizes"])),
                                       _p64(np.ascontiguousarray(lay["seeds"], dtype=np.uint64)),
                                       2 if lay.get("bip", False) else int(lay.get("rf", False)),
                                       lay.get("partial_k", 0), int(lay.get("retrieval", RETRIEVAL_XOR)),
                                       lay["rho"], _p8(np.ascontiguousarray(lay.get("rseed", np.zeros(1, np.uint8)),
                                                                            dtype=np.uint8)),
                                       _p64(np.ascontiguousarray(lay.get("rbit_offset", np.zeros(1, np.uint64)),
                                                                 dtype=np.uint64)),
                                       _p8(np.ascontiguousarray(lay["z"], dtype=np.uint8)), _p64(out))
    return rc, out[:q.size]


# ---- bipartite ShockHash ---------------------------------------------------------

def bip_slots(key: int, seed: int, n: int) -> tuple[int, int]:
    a, b = ctypes.c_uint32(), ctypes.c_uint32()
    lib().shock_oracle_bip_slots(key & 0xFFFFFFFFFFFFFFFF, seed & 0xFFFFFFFFFFFFFFFF, n, ctypes.byref(a),
                                 ctypes.byref(b))
    return a.value, b.value


def bip_pair_rank(a: int, b: int) -> int:
    """Rank of the seed pair (a, b) in the bipartite search order."""
    return int(lib().shock_oracle_bip_pair_rank(a, b))


def bip_leaf_search(keys, offsets, max_seed: int = 1 << 22, use_filter: bool = True):
    """(status, a uint64[L], b uint64[L], orient uint64[L]) of bipartite ShockHash."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
    L = max(len(offsets) - 1, 0)
    a = np.zeros(max(L, 1), np.uint64)
    b = np.zeros(max(L, 1), np.uint64)
    f = np.zeros(max(L, 1), np.uint64)
    rc = lib().shock_oracle_bip_leaf_search(_p64(keys) if keys.size else None, _p64(offsets), L, _p64(a), _p64(b),
                                            _p64(f), max_seed, int(use_filter))
    return rc, a[:L], b[:L], f[:L]

