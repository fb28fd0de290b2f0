"""Autotuner for the persistent leaf-search kernel.

It chooses, by timing the kernel on this device, for each leaf size n in a
list, the best of every combination of:

* seeds per lane (`spl`, the ILP width of the hash loop: 1, 2 or 4),
* waves per workgroup (the waves that share each fresh leaf: 1, 2, 4 or 8),
* the claim size: how many 64*spl-seed units a worker takes from a leaf at
  once (`block_iters_by_n`).  Small claims keep the speculative work beyond a
  leaf's answer low; large ones amortise the claim atomic.

One launch runs one (spl, waves per workgroup) pair, so a batch of mixed leaf
sizes needs one pair for all of them: the record's `spl` and `waves_per_wg`
are the pair with the least total time over the tuned sizes (each size's time
relative to its own best), and `per_n` keeps every size's own best pair and
how much slower the shared pair is there.

Each trial searches a synthetic batch of n-key leaves (uniform 64-bit keys)
and is timed with the library's HIP-event kernel time.  The table covers
every n in [0, 64] by taking the nearest tuned size.  Results are cached as
JSON keyed by the device name under paper_2308_09561_amd/tuning/.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
TUNING_DIR = os.path.join(_HERE, "tuning")


def expected_seeds(n: int) -> float:
    """Rough seeds per leaf (the construction bound (e/2)^n e/sqrt(pi) of
    ShockHash's analysis, shrunk by 1.5 sqrt(n)); used only to size trials."""
    if n < 2:
        return 1.0
    return (math.e / 2) ** n * math.e / math.sqrt(math.pi) / (1.5 * math.sqrt(n))


def _device_name():
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0] + "-" + p.name.replace(" ", "_")


def _batch(n: int, leaves: int, seed: int):
    from workloads import fixed_leaves
    import torch
    keys, offs = fixed_leaves(leaves, n, seed)
    k = torch.from_numpy(keys.view(np.int64)).cuda()
    o = torch.from_numpy(offs.view(np.int64)).cuda()
    return k, o


def _trial(k, o, **opts) -> float:
    from . import binding as B
    rc, _, _ = B.leaf_search(k, o, **opts)
    if rc != B.SHOCK_OK:
        raise RuntimeError(f"trial failed: {rc}")
    return B.shock_last_stats()["kernel_ms"]


def leaves_for(n: int, target_s: float = 0.1, evals_per_s: float = 2.6e12, lo: int = 256, hi: int = 65536) -> int:
    return int(min(hi, max(lo, target_s * evals_per_s / (expected_seeds(n) * max(n, 1)))))


def pick_units(res, tolerance: float = 0.01) -> int:
    """The largest claim size within `tolerance` of the fastest: timings of
    near-equal claim sizes differ by run-to-run noise, and larger claims make
    fewer atomics on the leaf's claim word."""
    best = min(ms for ms, _ in res)
    return max(u for ms, u in res if ms <= best * (1.0 + tolerance))


HEAVY_UNITS = (8, 16, 32, 64)  # claim sizes tried above 44 keys (smaller ones lose there by far)


def tune(sizes=(16, 24, 32, 40, 48, 56, 64), units=(1, 2, 4, 8, 16, 32, 64), spls=(1, 2, 4), wpws=(1, 2, 4, 8),
         repeats: int = 2, log=print) -> dict:
    """Run the sweep; returns the tuning record (also usable as search opts).

    Every leaf size n is timed on its own batch (about 0.1 s of work: 65536
    light leaves down to 256 of 64 keys) for every (spl, waves per workgroup,
    claim size); the best time of `repeats` runs counts."""
    t0 = time.time()
    per_n = {}
    for n in sizes:
        k, o = _batch(n, leaves_for(n), 7100 + n)
        _trial(k, o)  # warm
        grid = {}
        for spl in spls:
            for wpw in wpws:
                res = []
                for u in (units if n <= 44 else HEAVY_UNITS):
                    ms = min(_trial(k, o, spl=spl, waves_per_wg=wpw, block_iters=u) for _ in range(repeats))
                    res.append((ms, u))
                grid[(spl, wpw)] = res
                log(f"[tune] n={n} spl={spl} wpw={wpw}: best {min(res)[0]:.3f} ms")
        best_pair = min(grid, key=lambda p: min(grid[p])[0])
        per_n[n] = {"leaves": int(o.numel() - 1), "grid": grid, "best_pair": best_pair,
                    "best_ms": min(grid[best_pair])[0]}
    # one pair for every size: least sum of (time / that size's best)
    pairs = list(per_n[sizes[0]]["grid"])
    cost = {p: sum(min(per_n[n]["grid"][p])[0] / per_n[n]["best_ms"] for n in sizes) for p in pairs}
    spl, wpw = min(pairs, key=lambda p: cost[p])
    table = [0] * 65
    out_n = {}
    for n in sizes:
        g = per_n[n]["grid"]
        out_n[str(n)] = {
            "leaves": per_n[n]["leaves"],
            "best": {"spl": per_n[n]["best_pair"][0], "waves_per_wg": per_n[n]["best_pair"][1],
                     "units": pick_units(g[per_n[n]["best_pair"]]), "ms": per_n[n]["best_ms"]},
            "units": pick_units(g[(spl, wpw)]),
            "shared_pair_ms": min(g[(spl, wpw)])[0],
            "shared_pair_slowdown": min(g[(spl, wpw)])[0] / per_n[n]["best_ms"] - 1.0,
            "ms": {f"spl{p[0]}_wpw{p[1]}": {str(u): m for m, u in g[p]} for p in g},
        }
    tuned = sorted(per_n)
    for n in range(65):
        near = min(tuned, key=lambda t: (abs(t - n), t))
        table[n] = out_n[str(near)]["units"]
    rec = {"device": _device_name(), "spl": spl, "waves_per_wg": wpw, "block_iters_by_n": table,
           "spl_by_n": [out_n[str(min(tuned, key=lambda t: (abs(t - n), t)))]["best"]["spl"] for n in range(65)],
           "waves_per_wg_by_n": [out_n[str(min(tuned, key=lambda t: (abs(t - n), t)))]["best"]["waves_per_wg"]
                                 for n in range(65)],
           "pair_cost": {f"spl{p[0]}_wpw{p[1]}": c for p, c in cost.items()},
           "per_n": out_n, "seconds": time.time() - t0}
    return rec


def _nearest(tuned, n):
    return min(tuned, key=lambda t: (abs(t - n), t))


def opts_for_sizes(sizes, rec: dict | None = None) -> dict:
    """Search options for a batch with these leaf sizes (host array): the
    (spl, waves per workgroup) pair with the least expected time, the sum over
    the batch's leaves of the tuned time per leaf of the nearest tuned size,
    with that pair's best claim size per leaf size.  {} without a record."""
    rec = rec if rec is not None else load()
    if not rec or "pair_cost" not in rec:  # records without per-size pairs
        return {}
    tuned = sorted(int(n) for n in rec["per_n"])
    counts = np.bincount(np.asarray(sizes, dtype=np.int64), minlength=65)
    pairs = list(rec["per_n"][str(tuned[0])]["ms"])
    best, best_t = None, None
    for p in pairs:
        t = 0.0
        for n in np.nonzero(counts)[0]:
            e = rec["per_n"][str(_nearest(tuned, int(n)))]
            t += counts[n] * min(e["ms"][p].values()) / e["leaves"]
        if best_t is None or t < best_t:
            best, best_t = p, t
    spl, wpw = (int(x) for x in best[3:].split("_wpw"))
    table = []
    for n in range(65):
        res = rec["per_n"][str(_nearest(tuned, n))]["ms"][best]
        table.append(pick_units([(m, int(u)) for u, m in res.items()]))
    return {"spl": spl, "waves_per_wg": wpw, "block_iters_by_n": table}


def cache_path(device: str | None = None) -> str:
    return os.path.join(TUNING_DIR, f"{device or _device_name()}.json")


def save(rec: dict, path: str | None = None) -> str:
    path = path or cache_path(rec["device"])
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return path


def load(device: str | None = None) -> dict | None:
    """The cached record for this device, or None.  Falls back to a record of
    the same architecture when the marketing name differs (it can, between
    driver stacks and under profilers)."""
    try:
        device = device or _device_name()
    except Exception:
        return None
    path = cache_path(device)
    if not os.path.exists(path):
        arch = device.split("-", 1)[0]
        same = sorted(f for f in os.listdir(TUNING_DIR) if f.startswith(arch + "-")) if os.path.isdir(TUNING_DIR) else []
        if not same:
            return None
        path = os.path.join(TUNING_DIR, same[0])
    with open(path) as fh:
        return json.load(fh)


def tuned_opts(device: str | None = None, sizes=None) -> dict:
    """Search options from the cache ({} if this device was never tuned): for
    a batch with the given leaf sizes (opts_for_sizes), else the pair shared
    by all tuned sizes."""
    rec = load(device)
    if not rec:
        return {}
    if sizes is not None and "pair_cost" in rec:
        return opts_for_sizes(sizes, rec)
    return {"spl": rec["spl"], "waves_per_wg": rec["waves_per_wg"], "block_iters_by_n": rec["block_iters_by_n"]}


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="tune the leaf-search kernel on this GPU")
    ap.add_argument("--out", default=None, help="JSON path (default: the package's tuning cache)")
    args = ap.parse_args()
    r = tune()
    print(save(r, args.out))
    print(json.dumps({k: v for k, v in r.items() if k != "per_n"}))
