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
_SRC = os.path.join(_HERE, "shock_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
EINVAL = -1
ENOTFOUND = -2
NOT_FOUND_SEED = np.uint64(0xFFFFFFFFFFFFFFFF)
DEFAULT_MAX_SEED = 1 << 32

_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation flags)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
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
