"""Continuous-batching request loop over a Pool (serving form).

Requests arrive on a clock; each one is admitted into the pool as soon as it
has arrived AND the pool has a free slot and enough contiguous workspace
bytes (FIFO: a request that does not fit blocks the ones behind it).  Every
iteration advances all active simulations by one pool step (one graph
replay); simulations that have taken their steps are read out and retired,
which frees their memory for the queue.  Per-step latency of a simulation is
the duration of the pool step that advanced it (HIP events).

Failure handling (every request ends with a status):
  done       all steps taken;
  rejected   the pool refuses the parameters (ADS_EINVAL), or the request
             does not fit even in an empty pool (it could never be admitted);
  cancelled  the request's ``cancel_at`` time (seconds after the start)
             passed while it was queued or running;
  failed     the periodic health check (every ``check_every`` steps) found a
             non-finite state: the slot is retired, the others continue.
"""
from __future__ import annotations

import collections
import dataclasses
import json
import time
from typing import Callable, List, Optional

import numpy as np

from .binding import AdsError

ADS_ENUMERIC = -5


@dataclasses.dataclass
class RequestRecord:
    rid: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    steps: int = 0
    dofs: int = 0
    status: str = "queued"
    error: str = ""
    step_ms: List[float] = dataclasses.field(default_factory=list)
    result: Optional[object] = None

    def as_json(self) -> dict:
        """Per-request metrics record: times in seconds after the start of
        the loop, per-step latency percentiles in ms, DOF-steps served."""
        def num(x):
            return None if x is None or x != x else float(x)
        ms = np.asarray(self.step_ms)
        return {"rid": self.rid, "status": self.status, "error": self.error,
                "arrival_s": num(self.arrival), "admitted_s": num(self.admitted),
                "finished_s": num(self.finished), "steps": self.steps,
                "dof_steps": int(self.steps * self.dofs),
                "step_ms_p50": float(np.percentile(ms, 50)) if ms.size else None,
                "step_ms_p99": float(np.percentile(ms, 99)) if ms.size else None}


def serve(pool, requests, setup: Callable, steps_of: Callable, dofs_of: Callable,
          keep_results: bool = False, clock=time.perf_counter, max_wall: float = 600.0,
          check_every: int = 0, sleep=time.sleep, records_path: Optional[str] = None):
    """Run the request stream to completion.

    requests: objects with ``rid``, ``arrival`` (seconds after start), ``cfg``
    and optionally ``cancel_at``; setup(sim, cfg) configures a freshly
    admitted slot (initial state, load, factor); steps_of(req) / dofs_of(req)
    give the step count and the DOFs counted by the throughput metric.
    check_every > 0: every that many steps of a simulation its state is
    checked for non-finite values.  records_path: one JSON line per request
    (RequestRecord.as_json) is written there at the end.  Returns
    (records, stats).
    """
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    recs = {r.rid: RequestRecord(r.rid, r.arrival) for r in requests}
    active = {}                      # slot -> [req, sim, steps_done]
    t0 = clock()
    busy = 0.0
    dof_steps = 0

    def cancelled(req, now):
        c = getattr(req, "cancel_at", None)
        return c is not None and now >= c

    def finish(slot, status, error=""):
        req, sim, n = active.pop(slot)
        rec = recs[req.rid]
        if keep_results and status == "done":
            rec.result = [t.cpu().numpy() if t is not None else None for t in sim.get_state()]
        rec.steps = n
        rec.dofs = dofs_of(req)
        rec.status = status
        rec.error = error
        pool.retire(sim)
        rec.finished = clock() - t0

    while pending or active:
        now = clock() - t0
        if now > max_wall:
            raise TimeoutError("serving loop exceeded its wall-clock budget")
        # running requests whose cancellation time has passed
        for slot in [s for s, ent in active.items() if cancelled(ent[0], now)]:
            finish(slot, "cancelled")
        # admission, first come first served
        while pending and pending[0].arrival <= now:
            req = pending[0]
            rec = recs[req.rid]
            if cancelled(req, now):
                pending.popleft()
                rec.status, rec.finished = "cancelled", now
                continue
            try:
                sim = pool.admit(req.cfg)
            except AdsError as e:            # parameters this pool cannot take
                pending.popleft()
                rec.status, rec.error, rec.finished = "rejected", str(e), now
                continue
            if sim is None:
                if not active:               # nothing left to free: it never fits
                    pending.popleft()
                    rec.status, rec.error, rec.finished = "rejected", "larger than the empty pool", now
                    continue
                break
            pending.popleft()
            setup(sim, req.cfg)
            pool.activate(sim)
            active[sim.slot] = [req, sim, 0]
            rec.admitted = clock() - t0
            rec.status = "running"
        if not active:
            if pending:
                sleep(max(0.0, min(0.01, pending[0].arrival - (clock() - t0))))
            continue
        pool.step(1)
        dt = float(pool.step_times()[-1])          # synchronizes
        busy += dt * 1e-3
        for slot in list(active):
            ent = active[slot]
            req, sim = ent[0], ent[1]
            ent[2] += 1
            recs[req.rid].step_ms.append(dt)
            dof_steps += dofs_of(req)
            if check_every > 0 and ent[2] % check_every == 0:
                try:
                    sim.check_finite()
                except AdsError as e:
                    if e.status != ADS_ENUMERIC:
                        raise
                    finish(slot, "failed", "non-finite state")
                    continue
            if ent[2] >= steps_of(req):
                finish(slot, "done")
    wall = clock() - t0
    done = [r for r in recs.values() if r.status == "done"]
    lat = np.concatenate([np.asarray(r.step_ms) for r in recs.values()] or [np.zeros(0)])
    req_lat = np.array([r.finished - r.arrival for r in done])
    counts = collections.Counter(r.status for r in recs.values())
    stats = {
        "requests": len(recs),
        "status": dict(counts),
        "wall_s": wall,
        "gpu_busy_s": busy,
        "dof_steps": int(dof_steps),
        "dof_steps_per_s": dof_steps / wall if wall > 0 else 0.0,
        "step_ms_p50": float(np.percentile(lat, 50)) if lat.size else None,
        "step_ms_p99": float(np.percentile(lat, 99)) if lat.size else None,
        "request_s_p50": float(np.percentile(req_lat, 50)) if req_lat.size else None,
        "request_s_p99": float(np.percentile(req_lat, 99)) if req_lat.size else None,
    }
    if records_path is not None:
        with open(records_path, "w") as fh:
            for r in recs.values():
                fh.write(json.dumps(r.as_json()) + "\n")
    return list(recs.values()), stats
