"""Autotuner for the persistent leaf-search kernel.

It chooses, by timing the kernel on this device:

* seeds per lane (`spl`, the ILP width of the hash loop) and waves per
  workgroup (the number of leaves a workgroup works on at once), once, on a
  representative leaf size;
* for each leaf size n in a list, the claim size: how many 64*spl-seed units
  a worker takes from a leaf at once (`block_iters_by_n`).  Small claims keep
  the speculative work beyond a leaf's answer low; large ones amortise the
  claim atomic.

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


def leaves_for(n: int, target_s: float = 0.04, evals_per_s: float = 2.6e12, lo: int = 256, hi: int = 65536) -> int:
    return int(min(hi, max(lo, target_s * evals_per_s / (expected_seeds(n) * max(n, 1)))))


def pick_units(res, tolerance: float = 0.01) -> int:
    """The largest claim size within `tolerance` of the fastest: timings of
    near-equal claim sizes differ by run-to-run noise, and larger claims make
    fewer atomics on the leaf's claim word."""
    best = min(ms for ms, _ in res)
    return max(u for ms, u in res if ms <= best * (1.0 + tolerance))


def tune(sizes=(16, 24, 32, 40, 48, 56, 64), units=(1, 2, 4, 8, 16, 32, 64), spls=(1, 2, 4), wpws=(2, 4, 8),
         rep_n: int = 48, rep_leaves: int = 16384, rep_units=(16, 64), repeats: int = 3, log=print) -> dict:
    """Run the sweep; returns the tuning record (also usable as search opts).

    Seeds per lane and waves per workgroup are chosen on a batch of the
    serving stream's shape (rep_leaves leaves of rep_n keys: a batch too small
    favours wide teams that only shorten its tail), each at its better claim
    size of rep_units; then the claim size per leaf size."""
    t0 = time.time()
    k, o = _batch(rep_n, rep_leaves, 7001)
    _trial(k, o)  # warm
    best = None
    for spl in spls:
        for wpw in wpws:
            ms = min(_trial(k, o, spl=spl, waves_per_wg=wpw, block_iters=u) for u in rep_units for _ in range(repeats))
            log(f"[tune] n={rep_n} spl={spl} wpw={wpw}: {ms:.2f} ms")
            if best is None or ms < best[0]:
                best = (ms, spl, wpw)
    _, spl, wpw = best
    per_n = {}
    for n in sizes:
        k, o = _batch(n, leaves_for(n), 7100 + n)
        _trial(k, o, spl=spl, waves_per_wg=wpw)
        res = []
        for u in units:
            ms = min(_trial(k, o, spl=spl, waves_per_wg=wpw, block_iters=u) for _ in range(repeats))
            res.append((ms, u))
            log(f"[tune] n={n} units={u}: {ms:.2f} ms")
        per_n[n] = {"units": pick_units(res), "ms": {str(u): m for m, u in res}, "leaves": int(o.numel() - 1)}
    table = [0] * 65
    tuned = sorted(per_n)
    for n in range(65):
        near = min(tuned, key=lambda t: (abs(t - n), t))
        table[n] = per_n[near]["units"]
    rec = {"device": _device_name(), "spl": spl, "waves_per_wg": wpw, "block_iters_by_n": table,
           "per_n": per_n, "seconds": time.time() - t0}
    return rec


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


def tuned_opts(device: str | None = None) -> dict:
    """Search options from the cache ({} if this device was never tuned)."""
    rec = load(device)
    if not rec:
        return {}
    return {"spl": rec["spl"], "waves_per_wg": rec["waves_per_wg"], "block_iters_by_n": rec["block_iters_by_n"]}


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="tune the leaf-search kernel on this GPU")
    ap.add_argument("--out", default=None, help="JSON path (default: the package's tuning cache)")
    args = ap.parse_args()
    r = tune()
    print(save(r, args.out))
    print(json.dumps({k: v for k, v in r.items() if k != "per_n"}))
