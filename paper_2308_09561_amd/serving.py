"""Serving loop: continuous batching of MPHF-build requests on one GPU.

A request carries N keys.  It is cut into leaves of `leaf_size` keys in input
order, plus one remainder leaf, and its build is done when every leaf has its
smallest seed and orientation.

LeafServer drives the library's native request queue (shock_queue in
include/shockleaf.h).  This module only turns arrivals into submissions and
completions into latencies; admission, batching and launches happen in the
library's dispatcher thread:

* Requests that arrive while others are on the GPU wait in a FIFO queue.
* A free slot takes as many queued requests, in order, as the queue's device
  arena (the HBM budget) and the slot's capacity allow.
* The slot uploads their keys from pinned staging, enqueues one asynchronous
  persistent search over all of them, and moves on.  Batches on different
  streams run concurrently: a persistent kernel's idle workers leave once
  nothing is open in their batch, and a newer batch's workgroups take their
  place.
* When a slot's search completes, its results are copied into each request's
  host buffers, its arena block is freed and the next requests are admitted.

Latency of a request = completion time (the dispatcher's clock) - arrival
time.  The device memory a batch holds while admitted (keys, offsets, outputs
and search scratch) is one block of the budget.  A request alone larger than
the budget is rejected; a request still queued past its deadline is
withdrawn (timeout).

MphfServer serves the same requests with complete minimal perfect hash
functions (the flat ShockHash MPHF of include/shockmphf.h): each request is
one build on one of `slots` worker threads, each with its own HIP stream, so
builds overlap on the GPU; admission follows the same budget and queue rules
with the build's device footprint.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait
from dataclasses import dataclass, field

import numpy as np

from .binding import MPHF, SHOCK_ECANCELED, SHOCK_ENOMEM, SHOCK_OK, RequestQueue, queue_batch_bytes

SCRATCH_BYTES_PER_LEAF = 600  # premixed keys, claim word, best seed, counters (MPHF build estimate)


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    keys: np.ndarray        # uint64 keys (host)
    deadline: float | None = None  # seconds after arrival; None = no deadline
    # filled in by the server
    offsets: np.ndarray | None = None
    admitted: float | None = None
    completed: float | None = None
    status: str = "queued"
    seeds: np.ndarray | None = None
    orient: np.ndarray | None = None
    info: dict | None = None  # MPHF build figures (MphfServer)

    @property
    def n_leaves(self) -> int:
        if self.offsets is None:
            return int(self.info["n_leaves"]) if self.info else 0
        return len(self.offsets) - 1

    def latency(self) -> float | None:
        return None if self.completed is None else self.completed - self.arrival


def leaf_offsets(n_keys: int, leaf_size: int) -> np.ndarray:
    full = n_keys // leaf_size
    offs = np.arange(full + 1, dtype=np.uint64) * np.uint64(leaf_size)
    if n_keys % leaf_size:
        offs = np.append(offs, np.uint64(n_keys))
    return offs


def footprint(n_keys: int, n_leaves: int) -> int:
    """Device bytes a request alone holds while admitted (one batch)."""
    return queue_batch_bytes(n_leaves, n_keys)


@dataclass
class ServeReport:
    requests: list
    makespan_s: float
    max_bytes_in_flight: int
    max_batches_in_flight: int
    batches: int
    extra: dict = field(default_factory=dict)

    def summary(self) -> dict:
        done = [r for r in self.requests if r.status == "done"]
        lat = np.array([r.latency() for r in done], dtype=np.float64)
        keys = float(sum(len(r.keys) for r in done))
        leaves = float(sum(r.n_leaves for r in done))
        infos = [r.info for r in done if r.info]
        if infos:
            self.extra.setdefault("bits_per_key", float(sum(i["bits_total"] for i in infos) /
                                                        max(sum(i["n_keys"] for i in infos), 1)))
        return {
            "requests": len(self.requests), "completed": len(done),
            "timed_out": sum(r.status == "timeout" for r in self.requests),
            "rejected": sum(r.status == "rejected" for r in self.requests),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "mean_ms": float(lat.mean() * 1e3) if lat.size else None,
            "keys_per_s": keys / self.makespan_s if self.makespan_s > 0 else None,
            "leaves_per_s": leaves / self.makespan_s if self.makespan_s > 0 else None,
            "makespan_s": self.makespan_s, "batches": self.batches,
            "max_bytes_in_flight": self.max_bytes_in_flight,
            "max_batches_in_flight": self.max_batches_in_flight, **self.extra,
        }


class LeafServer:
    def __init__(self, hbm_budget_bytes: int = 256 << 20, slots: int = 4, leaf_size: int = 48,
                 max_batch_leaves: int = 1 << 16, search_opts: dict | None = None, device: str = "cuda:0"):
        import torch

        if leaf_size < 1 or leaf_size > 64:
            raise ValueError("leaf_size must be in [1, 64]")
        self.device = torch.device(device)
        self.budget = int(hbm_budget_bytes)
        self.slots = slots
        self.leaf_size = leaf_size
        self.max_batch_leaves = max_batch_leaves
        self.opts = dict(search_opts or {})
        self.opts.pop("leaf_size_hint", None)

    def close(self):
        pass

    def run(self, requests: list, realtime: bool = True) -> ServeReport:
        """Serve requests (sorted by arrival).  With realtime=False every
        request is treated as having arrived at time 0 (a backlog)."""
        for r in requests:
            r.offsets = leaf_offsets(len(r.keys), self.leaf_size)
            r.status = "queued"
            r.admitted = r.completed = None
            r.seeds = r.orient = None
        q = RequestQueue(device=self.device.index or 0, hbm_budget_bytes=self.budget, slots=self.slots,
                         max_batch_leaves=self.max_batch_leaves,
                         max_batch_keys=self.max_batch_leaves * self.leaf_size, **self.opts)
        try:
            pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
            inflight = {}
            t0 = time.perf_counter_ns()
            now = lambda: (time.perf_counter_ns() - t0) * 1e-9  # noqa: E731 (same clock as the library's)
            while pending or inflight:
                t = now()
                while pending and (not realtime or pending[0].arrival <= t):
                    r = pending.popleft()
                    rc, ticket = q.submit(r.keys, r.offsets)
                    if rc == SHOCK_ENOMEM:
                        r.status = "rejected"
                        continue
                    if rc != SHOCK_OK:
                        raise RuntimeError(f"submit failed with status {rc}")
                    inflight[ticket] = r
                for ticket, r in list(inflight.items()):
                    done, rc, info, seeds, orient = q.poll(ticket)
                    if not done:
                        if r.deadline is not None and now() - r.arrival > r.deadline:
                            r.deadline = None  # withdrawn now, or already running and left to finish
                            q.cancel(ticket)
                        continue
                    del inflight[ticket]
                    if rc == SHOCK_ECANCELED:
                        r.status = "timeout"
                        continue
                    r.admitted = (info["admit_ns"] - t0) * 1e-9
                    r.completed = (info["done_ns"] - t0) * 1e-9
                    r.seeds, r.orient = seeds, orient
                    r.status = "done" if rc == SHOCK_OK else f"error {rc}"
                if inflight:
                    time.sleep(0.0001)
                elif pending:
                    time.sleep(max(0.0, min(0.001, pending[0].arrival - now())))
            makespan = now()
            st = q.stats()
        finally:
            q.close()
        return ServeReport(requests=list(requests), makespan_s=makespan, max_bytes_in_flight=st["max_bytes_in_flight"],
                           max_batches_in_flight=st["max_batches_in_flight"], batches=st["batches"])


def synthetic_stream(n_requests: int, rate_per_s: float, seed: int = 5, min_keys: int = 1000,
                     max_keys: int = 1_000_000, deadline: float | None = None) -> list:
    """Requests of the serving workload: Poisson arrivals, log-uniform key
    counts, keys from splitmix64 per request (see workloads.serving_requests)."""
    from workloads import serving_requests, splitmix64

    out = []
    for rid, (arr, n, kseed) in enumerate(serving_requests(n_requests, rate_per_s, seed, min_keys, max_keys)):
        out.append(Request(rid=rid, arrival=arr, keys=splitmix64(kseed, n), deadline=deadline))
    return out


def _ribbon_cols(m: int) -> int:
    return 0 if m == 0 else max(64, m + (m + 49) // 50)


def mphf_footprint(n_keys: int, bucket_size: int = 2000, leaf_target: int = 40, bipartite: bool = False) -> int:
    """Device bytes an MPHF build of n_keys (ribbon retrieval) holds at its
    peak: the keys; the build's scratch arena (a bucket-ordered and a
    leaf-ordered copy of the keys, the choices, per-leaf and per-bucket
    tables, and the ribbon region: the larger of the walk's slots, about 9.5
    bytes per key, and the block solver's pivot rows, two waves of 16 bytes
    per column for each bucket it runs at once, sized for buckets of 9/8 of
    bucket_size plus 256 keys), grown by an eighth; and the leaf search
    outputs and scratch (bipartite: also the second pass's leaf list, kept by
    the device).  The arena stays cached by the building thread after the
    build."""
    N = int(n_keys)
    B = max(1, -(-N // bucket_size))
    L = B + -(-N // leaf_target)
    rib_max = N + N // 50 + 65 * B
    slot = 8 * (rib_max + rib_max // 8 + 2 * (rib_max // 64) + 3 * B + 64)
    m_est = min(bucket_size + bucket_size // 8 + 256, 16384)
    W = -(-_ribbon_cols(m_est) // 64)
    piv = B * 2 * (-(-16 * 64 * W // 256) * 256)
    arena = 18 * N + 31 * L + 49 * B + max(slot, piv) + 8448 + (16 * L if bipartite else 0)
    arena += arena // 8  # the arena grows by an eighth over a reservation
    return 8 * N + arena + (16 + SCRATCH_BYTES_PER_LEAF + (4 if bipartite else 0)) * L + (1 << 20)


class MphfServer:
    """Requests served as complete MPHF builds (see the module docstring)."""

    def __init__(self, hbm_budget_bytes: int = 1 << 30, slots: int = 2, bucket_size: int = 2000,
                 leaf_target: int = 40, leaf_max: int = 56, rice_table=None, verify: bool = False,
                 rotation_fitting: bool = False, bipartite: bool = False, device: str = "cuda:0"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(hbm_budget_bytes)
        self.slots = slots
        self.params = dict(bucket_size=bucket_size, leaf_target=leaf_target, leaf_max=leaf_max, rice_table=rice_table,
                           rotation_fitting=rotation_fitting, bipartite=bipartite)
        self.verify = verify
        self._local = threading.local()
        self.pool = ThreadPoolExecutor(max_workers=slots)

    def close(self):
        self.pool.shutdown(wait=True)

    def _stream(self):
        st = getattr(self._local, "stream", None)
        if st is None:
            st = self._local.stream = self.torch.cuda.Stream(device=self.device)
        return st

    def _build(self, r: Request, now_fn):
        torch = self.torch
        stream = self._stream()
        with torch.cuda.stream(stream):
            kh = torch.from_numpy(np.ascontiguousarray(r.keys).view(np.int64)).pin_memory()
            kd = kh.to(self.device, non_blocking=True)
            m = MPHF(kd, stream=stream.cuda_stream, **self.params)
            try:
                r.info = m.info()
                if self.verify:
                    pos = m.query(kd, stream=stream.cuda_stream)
                    srt, _ = torch.sort(pos)
                    ok = bool(torch.equal(srt, torch.arange(len(r.keys), device=self.device, dtype=torch.int64)))
                    r.info["bijection"] = ok
            finally:
                m.close()
            stream.synchronize()
        r.completed = now_fn()
        r.status = "done" if (not self.verify or r.info.get("bijection")) else "error bijection"
        return r

    def run(self, requests: list, realtime: bool = True) -> ServeReport:
        for r in requests:
            r.offsets = None
            r.status = "queued"
            r.admitted = r.completed = None
            r.info = None
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        inflight = {}
        bytes_in_flight = max_bytes = max_batches = n_batches = 0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        while pending or queue or inflight:
            t = now()
            while pending and (not realtime or pending[0].arrival <= t):
                queue.append(pending.popleft())
            for fut in [f for f in inflight if f.done()]:
                fut.result()  # re-raise build errors
                bytes_in_flight -= inflight.pop(fut)
            t = now()
            queue = collections.deque(r for r in queue if not self._expired(r, t))
            while queue and len(inflight) < self.slots:
                r = queue[0]
                fb = mphf_footprint(len(r.keys), self.params["bucket_size"], self.params["leaf_target"],
                                    bool(self.params["bipartite"]))
                if fb > self.budget:
                    queue.popleft()
                    r.status = "rejected"
                    continue
                if bytes_in_flight + fb > self.budget:
                    break
                queue.popleft()
                r.admitted = now()
                r.status = "running"
                inflight[self.pool.submit(self._build, r, now)] = fb
                bytes_in_flight += fb
                n_batches += 1
                max_bytes = max(max_bytes, bytes_in_flight)
                max_batches = max(max_batches, len(inflight))
            if inflight:
                wait(list(inflight), timeout=0.0005, return_when=FIRST_COMPLETED)
            elif pending:
                time.sleep(max(0.0, min(0.001, pending[0].arrival - now())))
        return ServeReport(requests=list(requests), makespan_s=now(), max_bytes_in_flight=max_bytes,
                           max_batches_in_flight=max_batches, batches=n_batches)

    @staticmethod
    def _expired(r: Request, t: float) -> bool:
        if r.deadline is not None and t - r.arrival > r.deadline:
            r.status = "timeout"
            r.completed = None
            return True
        return False

