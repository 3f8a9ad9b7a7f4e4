"""Continuous-batching request loop over a Pool (serving form).

Requests arrive on a clock; each one is admitted into the pool as soon as it
has arrived AND the pool has a free slot and enough contiguous workspace
bytes (FIFO: a request that does not fit blocks the ones behind it).  Every
iteration advances all active simulations by one pool step (one graph
replay); simulations that have taken their steps are read out and retired,
which frees their memory for the queue.  Per-step latency of a simulation is
the duration of the pool step that advanced it (HIP events).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class RequestRecord:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    steps: int = 0
    dofs: int = 0
    step_ms: List[float] = dataclasses.field(default_factory=list)
    result: Optional[object] = None


def serve(pool, requests, setup: Callable, steps_of: Callable, dofs_of: Callable,
          keep_results: bool = False, clock=time.perf_counter, max_wall: float = 600.0):
    """Run the request stream to completion.

    requests: objects with ``rid``, ``arrival`` (seconds after start) and
    ``cfg``; setup(sim, cfg) configures a freshly admitted slot (initial
    state, load, factor); steps_of(req) / dofs_of(req) give the step count
    and the DOFs counted by the throughput metric.  Returns (records, stats).
    """
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    recs = {r.rid: RequestRecord(r.rid, r.arrival) for r in requests}
    active = {}                      # slot -> [req, sim, steps_done]
    t0 = clock()
    busy = 0.0
    dof_steps = 0
    while pending or active:
        now = clock() - t0
        if now > max_wall:
            raise TimeoutError("serving loop exceeded its wall-clock budget")
        while pending and pending[0].arrival <= now:
            req = pending[0]
            sim = pool.admit(req.cfg)
            if sim is None:
                break
            pending.popleft()
            setup(sim, req.cfg)
            pool.activate(sim)
            active[sim.slot] = [req, sim, 0]
            recs[req.rid].admitted = clock() - t0
        if not active:
            if pending:
                time.sleep(max(0.0, min(0.01, pending[0].arrival - (clock() - t0))))
            continue
        pool.step(1)
        dt = float(pool.step_times()[-1])          # synchronizes
        busy += dt * 1e-3
        for slot in list(active):
            ent = active[slot]
            req, sim = ent[0], ent[1]
            ent[2] += 1
            rec = recs[req.rid]
            rec.step_ms.append(dt)
            dof_steps += dofs_of(req)
            if ent[2] >= steps_of(req):
                if keep_results:
                    rec.result = [t.cpu().numpy() if t is not None else None for t in sim.get_state()]
                rec.steps = ent[2]
                rec.dofs = dofs_of(req)
                pool.retire(sim)
                del active[slot]
                rec.finished = clock() - t0
    wall = clock() - t0
    lat = np.concatenate([np.asarray(r.step_ms) for r in recs.values()]) if recs else np.zeros(0)
    req_lat = np.array([r.finished - r.arrival for r in recs.values()])
    stats = {
        "requests": len(recs),
        "wall_s": wall,
        "gpu_busy_s": busy,
        "dof_steps": int(dof_steps),
        "dof_steps_per_s": dof_steps / wall if wall > 0 else 0.0,
        "step_ms_p50": float(np.percentile(lat, 50)) if lat.size else None,
        "step_ms_p99": float(np.percentile(lat, 99)) if lat.size else None,
        "request_s_p50": float(np.percentile(req_lat, 50)) if req_lat.size else None,
        "request_s_p99": float(np.percentile(req_lat, 99)) if req_lat.size else None,
    }
    return list(recs.values()), stats
