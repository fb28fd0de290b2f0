"""Write the oracle's per-leaf results for every full-size workload.

Calls only `oracle/` (the plain CPU search, leaf ranges spread over host
threads by `oracle.parallel`) and `workloads/` (the seeded inputs).  Nothing
here comes from the GPU library.  Each workload becomes one compressed file
`oracle_<name>.npz` next to this script with:

  seeds   uint32[L]  the smallest qualifying seed (Section 4); every seed of
                     these workloads is below the default cap of 2^32
  orient  uint64[L]  the canonical orientation (smallest valid mask, Section 5)
  rot     uint32[L]  (rotation fitting only) the rotation of the candidate
  inputs  str        SHA-256 of the keys and offsets the results belong to
  kind    str        "plain" or "rf"

The long workloads are cut into chunks; finished chunks are kept under
`--cache` so an interrupted run resumes where it stopped.

    python tests/golden/make_oracle_outputs.py [--threads 8] [name ...]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import inputs_digest, make_workload  # noqa: E402

# (file name, workload, search kind)
TARGETS = [
    ("plain24", "plain24", "plain"),
    ("fixed40", "fixed40", "plain"),
    ("fixed48", "fixed48", "plain"),
    ("full64", "full64", "plain"),
    ("rf_full64", "full64", "rf"),
    ("rf_fixed48", "fixed48", "rf"),
    ("hard60", "hard60", "plain"),
    ("uneven32_56", "uneven32_56", "plain"),
]

CHUNK = 4096


def golden_path(name: str) -> str:
    return os.path.join(HERE, f"oracle_{name}.npz")


def _search(kind, keys, offsets, threads):
    if kind == "plain":
        parts = oracle.parallel(oracle.leaf_search, keys, offsets, threads=threads)
        rc = [p[0] for p in parts]
        seeds = np.concatenate([p[1] for p in parts])
        orient = np.concatenate([p[2] for p in parts])
        rot = None
    else:
        parts = oracle.parallel(oracle.rf_leaf_search, keys, offsets, threads=threads)
        rc = [p[0] for p in parts]
        seeds = np.concatenate([p[1] for p in parts])
        rot = np.concatenate([p[2] for p in parts])
        orient = np.concatenate([p[3] for p in parts])
    if any(r != oracle.OK for r in rc):
        raise RuntimeError(f"oracle returned {rc}")
    return seeds, rot, orient


def make(name: str, workload: str, kind: str, threads: int, cache: str) -> None:
    keys, offsets = make_workload(workload)
    L = len(offsets) - 1
    digest = inputs_digest(keys, offsets)
    os.makedirs(cache, exist_ok=True)
    seeds, rots, orients = [], [], []
    t0 = time.time()
    for a in range(0, L, CHUNK):
        b = min(a + CHUNK, L)
        part = os.path.join(cache, f"{name}_{digest[:16]}_{a}_{b}.npz")
        if os.path.exists(part):
            z = np.load(part)
            s, f = z["seeds"], z["orient"]
            r = z["rot"] if kind == "rf" else None
        else:
            sub = offsets[a:b + 1]
            base = int(sub[0])
            s, r, f = _search(kind, keys[base:int(sub[-1])], sub - np.uint64(base), threads)
            extra = {"rot": r} if kind == "rf" else {}
            np.savez(part + ".tmp.npz", seeds=s, orient=f, **extra)
            os.replace(part + ".tmp.npz", part)
        seeds.append(s)
        orients.append(f)
        if kind == "rf":
            rots.append(r)
        print(f"{name}: leaves {b}/{L}  {time.time() - t0:.0f} s", flush=True)
    seeds = np.concatenate(seeds)
    if (seeds >= np.uint64(1 << 32)).any():
        raise RuntimeError("a seed does not fit 32 bits")
    out = dict(seeds=seeds.astype(np.uint32), orient=np.concatenate(orients), inputs=np.array(digest),
               kind=np.array(kind))
    if kind == "rf":
        out["rot"] = np.concatenate(rots).astype(np.uint32)
    tmp = golden_path(name) + ".tmp.npz"
    np.savez_compressed(tmp, **out)
    os.replace(tmp, golden_path(name))
    print(f"{name}: wrote {golden_path(name)} in {time.time() - t0:.0f} s", flush=True)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", help="subset of: " + ", ".join(t[0] for t in TARGETS))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--cache", default=os.path.join(HERE, ".oracle_cache"))
    ap.add_argument("--force", action="store_true", help="rewrite files that already exist")
    args = ap.parse_args()
    oracle.build(force=False)
    for name, workload, kind in TARGETS:
        if args.names and name not in args.names:
            continue
        if os.path.exists(golden_path(name)) and not args.force:
            print(f"{name}: exists, skipped", flush=True)
            continue
        make(name, workload, kind, args.threads, args.cache)


if __name__ == "__main__":
    main()
