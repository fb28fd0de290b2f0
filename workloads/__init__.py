"""Seeded synthetic inputs for the ShockHash leaf seed search.

This module is shared by the tests, the benchmark and the oracle checks.  It
holds none of the method's arithmetic: only pseudo-random key streams
(splitmix64, Steele/Lea/Flood 2014, written from its public definition) and
the CSR leaf layouts of the workloads.

Keys are uniform 64-bit values.  The paper hashes string keys to a 64-bit
master hash code first and evaluates every later hash function on that code
(Section 8, experimental setup), so uniform 64-bit keys stand in for its
random-string inputs.

Layout of a batch of leaves (CSR):
    keys    : uint64[sum n_j], leaf j = keys[offsets[j] : offsets[j+1]]
    offsets : uint64[L + 1], nondecreasing, offsets[0] = 0
All arrays are numpy uint64 (torch carries the same bits as int64).
"""
from __future__ import annotations

import hashlib

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """Outputs start .. start+count-1 of splitmix64 seeded with `seed`.

    The generator's state starts at `seed` and advances by the golden-ratio
    increment before every output; output k is the finaliser applied to
    seed + (k + 1) * gamma (mod 2^64).
    """
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def fixed_leaves(n_leaves: int, n: int, seed: int):
    """n_leaves leaves of exactly n keys each, keys from splitmix64(seed)."""
    keys = splitmix64(seed, n_leaves * n)
    offsets = np.arange(n_leaves + 1, dtype=np.uint64) * np.uint64(n)
    return keys, offsets


def uneven_sizes(n_leaves: int, n_min: int, n_max: int, size_seed: int) -> np.ndarray:
    """Leaf sizes uniform in [n_min, n_max] (inclusive): n = n_min + floor(hi32(u) * span / 2^32)."""
    u = splitmix64(size_seed, n_leaves)
    span = np.uint64(n_max - n_min + 1)
    return (np.uint64(n_min) + (((u >> np.uint64(32)) * span) >> np.uint64(32))).astype(np.uint64)


def uneven_leaves(n_leaves: int, n_min: int, n_max: int, key_seed: int, size_seed: int):
    """Leaves of uneven size (a batch of bucket splits); keys from splitmix64(key_seed) in CSR order."""
    sizes = uneven_sizes(n_leaves, n_min, n_max, size_seed)
    offsets = np.zeros(n_leaves + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    keys = splitmix64(key_seed, int(offsets[-1]))
    return keys, offsets


def chunk_offsets(n_keys: int, leaf_size: int) -> np.ndarray:
    """Split n_keys keys in input order into leaves of leaf_size plus one remainder leaf."""
    full = n_keys // leaf_size
    offs = list(range(0, full * leaf_size + 1, leaf_size))
    if n_keys % leaf_size:
        offs.append(n_keys)
    return np.asarray(offs, dtype=np.uint64)


# Named workloads.  The sizes follow the batch shapes this library targets:
# fixed leaf size, uneven leaf sizes from bucket splits, hard leaves near the
# 64-key register limit, and a stream of build requests cut into 48-key leaves.
WORKLOADS = {
    # 4096 leaves x 24 keys, searched one leaf per launch.
    "plain24": dict(kind="fixed", n_leaves=4096, n=24, seed=1),
    # 65536 leaves x 40 keys, one launch over all leaves.
    "fixed40": dict(kind="fixed", n_leaves=65536, n=40, seed=2),
    # 200000 leaves, n uniform in [32, 56].
    "uneven32_56": dict(kind="uneven", n_leaves=200000, n_min=32, n_max=56, seed=3, size_seed=1003),
    # 2048 leaves x 60 keys (hard leaves, split across workgroups).
    "hard60": dict(kind="fixed", n_leaves=2048, n=60, seed=4),
    # 16384 leaves x 48 keys: the leaf size of the serving stream.
    "fixed48": dict(kind="fixed", n_leaves=16384, n=48, seed=48),
    # 32 leaves x 64 keys: the full 64-bit coverage register.
    "full64": dict(kind="fixed", n_leaves=32, n=64, seed=64),
}


def inputs_digest(keys: np.ndarray, offsets: np.ndarray) -> str:
    """SHA-256 of a CSR batch, naming the inputs that stored results belong to."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(keys, dtype=np.uint64).tobytes())
    h.update(np.ascontiguousarray(offsets, dtype=np.uint64).tobytes())
    return h.hexdigest()


def make_workload(name: str, n_leaves: int | None = None):
    """Keys and offsets of a named workload, optionally truncated to its first n_leaves leaves."""
    w = WORKLOADS[name]
    L = w["n_leaves"] if n_leaves is None else min(n_leaves, w["n_leaves"])
    if w["kind"] == "fixed":
        return fixed_leaves(L, w["n"], w["seed"])
    sizes = uneven_sizes(w["n_leaves"], w["n_min"], w["n_max"], w["size_seed"])[:L]
    offsets = np.zeros(L + 1, dtype=np.uint64)
    np.cumsum(sizes, out=offsets[1:])
    keys = splitmix64(w["seed"], int(offsets[-1]))
    return keys, offsets


def serving_requests(n_requests: int = 1000, rate_per_s: float = 200.0, seed: int = 5,
                     min_keys: int = 1000, max_keys: int = 1_000_000):
    """A Poisson stream of MPHF-build requests.

    Returns a list of (arrival_time_s, n_keys, key_seed).  Gaps are exponential
    with the given rate; key counts are log-uniform in [min_keys, max_keys].
    Both use 53-bit uniforms from splitmix64(seed) (two outputs per request).
    Request r draws its keys from splitmix64(seed * 2^32 + r).
    """
    u = splitmix64(seed, 2 * n_requests)
    unif = (u >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    gaps = -np.log1p(-unif[0::2]) / rate_per_s
    arrivals = np.cumsum(gaps)
    lo, hi = np.log(min_keys), np.log(max_keys)
    counts = np.floor(np.exp(lo + unif[1::2] * (hi - lo))).astype(np.int64)
    counts = np.clip(counts, min_keys, max_keys)
    return [(float(arrivals[r]), int(counts[r]), seed * (1 << 32) + r) for r in range(n_requests)]
