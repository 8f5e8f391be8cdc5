"""Continuous-batching request loop over a dlrtrt batch.

Requests arrive at given times; each asks for n_steps DLR steps of one problem.
Arrived requests are admitted in arrival order as soon as their device footprint
fits in what the batch budget has left (first-in first-out: a request that does
not fit holds back the ones behind it).  Every pass advances all admitted
requests by one step together; finished requests are read back, released, and
their time-to-solution (result on the host minus arrival) recorded.  The batch
library does the work; this module only schedules.
"""
from __future__ import annotations

import collections
import time

import numpy as np

from . import dlrtrt


def serve(requests, hbm_budget=0, max_wall_s=None, progress=None):
    """requests: iterable of (t_arrival_s, problem, n_steps), sorted by arrival; problem is
    a problem dict or a callable that builds it (called when the request reaches the head of
    the admission queue, so its build time counts in its latency).

    Returns a dict with per-request latency (s), completion order, the
    cell-angle updates done, wall time and how many requests were left when
    max_wall_s stopped the loop (requests not yet finished are not counted), split
    into admitted-but-unfinished and still queued."""
    pending = collections.deque(requests)
    waiting = collections.deque()
    inflight = {}
    latency = {}
    failed = {}
    ca = 0
    passes = 0
    t0 = time.perf_counter()
    with dlrtrt.Batch(hbm_budget=hbm_budget) as batch:
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            if max_wall_s is not None and now > max_wall_s:
                break
            while pending and pending[0][0] <= now:
                waiting.append(pending.popleft())
            while waiting:
                t_arr, prob, nsteps = waiting[0]
                if callable(prob):
                    prob = prob()
                    waiting[0] = (t_arr, prob, nsteps)
                slot = batch.admit(prob, nsteps)
                if slot is None:
                    if not inflight:
                        raise RuntimeError(f"request {prob.get('name')} does not fit in an empty batch")
                    break
                waiting.popleft()
                inflight[slot] = (t_arr, prob)
            if not inflight:
                if pending:
                    time.sleep(max(0.0, pending[0][0] - (time.perf_counter() - t0)))
                continue
            batch.advance()
            passes += 1
            for slot, (t_arr, prob) in inflight.items():
                try:
                    st = batch.read_stats(slot)
                    ca += int(st["si_iters"]) * int(prob["nx"]) * int(prob["ny"]) * int(prob["rank"])
                except dlrtrt.DlrError:
                    pass
            for slot in batch.poll():
                t_arr, prob = inflight.pop(slot)
                try:
                    batch.read(slot)
                    latency[prob.get("name", str(slot))] = time.perf_counter() - t0 - t_arr
                except dlrtrt.DlrError as err:
                    failed[prob.get("name", str(slot))] = err.status
                batch.release(slot)
            if progress is not None:
                progress(passes, len(latency), len(inflight), len(waiting) + len(pending))
    wall = time.perf_counter() - t0
    lat = np.array(list(latency.values()))
    return {
        "completed": len(latency),
        "failed": failed,
        "unfinished": len(inflight) + len(waiting) + len(pending),
        "unfinished_admitted": len(inflight),
        "unfinished_queued": len(waiting) + len(pending),
        "arrived": len(latency) + len(failed) + len(inflight) + len(waiting),
        "wall_s": wall,
        "passes": passes,
        "cell_angle_updates": ca,
        "ca_per_s": ca / wall if wall > 0 else 0.0,
        "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
        "latency": latency,
    }
