"""The serving loop's scheduling logic on the CPU, against a fake pool with
the same interface as paper_1911_08158_amd.Pool (admission by bytes and
slots, one step for every active simulation, retirement frees memory) and a
deterministic clock: FIFO admission and head-of-line blocking, a request
that can never fit, parameters the pool refuses, cancellation while queued
and while running, and eviction of a simulation whose state turns
non-finite while the others run to completion."""
import dataclasses

import pytest

from paper_1911_08158_amd.binding import AdsError
from paper_1911_08158_amd.serve import serve


@dataclasses.dataclass
class Cfg:
    size: int                 # workspace bytes
    steps: int
    nan_at: int = 0           # state turns non-finite after this many steps (0: never)
    invalid: bool = False     # parameters the pool refuses


@dataclasses.dataclass
class Req:
    rid: int
    arrival: float
    cfg: Cfg
    cancel_at: float = None


class FakeSim:
    def __init__(self, slot, cfg):
        self.slot, self.cfg, self.steps = slot, cfg, 0
        self.active = False

    def check_finite(self):
        if self.cfg.nan_at and self.steps >= self.cfg.nan_at:
            raise AdsError(-5, "non-finite state")

    def get_state(self):
        return [None]


class FakePool:
    def __init__(self, nbytes, slots):
        self.nbytes, self.free_slots = nbytes, list(range(slots))
        self.used = 0
        self.sims = {}
        self.admitted = []           # ids of the admitted configurations, in admission order
        self.max_used = 0

    def admit(self, cfg):
        if cfg.invalid:
            raise AdsError(-1, "bad parameters")
        if not self.free_slots or self.used + cfg.size > self.nbytes:
            return None
        slot = self.free_slots.pop(0)
        self.used += cfg.size
        self.max_used = max(self.max_used, self.used)
        s = FakeSim(slot, cfg)
        self.sims[slot] = s
        self.admitted.append(id(cfg))
        return s

    def activate(self, sim):
        sim.active = True

    def step(self, n):
        for s in self.sims.values():
            if s.active:
                s.steps += n

    def step_times(self):
        return [1.0]

    def retire(self, sim):
        del self.sims[sim.slot]
        self.used -= sim.cfg.size
        self.free_slots.append(sim.slot)


class Clock:
    """Advances 1 ms per reading; sleeping advances it by the time slept."""

    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


def run(pool, reqs, check_every=0):
    clk = Clock()
    recs, stats = serve(pool, reqs, setup=lambda sim, cfg: None, steps_of=lambda r: r.cfg.steps,
                        dofs_of=lambda r: 1, clock=clk, sleep=clk.sleep, max_wall=1e4,
                        check_every=check_every)
    return {r.rid: r for r in recs}, stats


def test_fifo_admission_and_head_of_line_blocking():
    # room for one 60-byte request at a time: admission follows arrival order
    cfgs = [Cfg(60, 3), Cfg(60, 2), Cfg(30, 1), Cfg(30, 1)]
    reqs = [Req(i, 0.001 * i, c) for i, c in enumerate(cfgs)]
    pool = FakePool(100, 8)
    recs, stats = run(pool, reqs)
    assert pool.admitted == [id(c) for c in cfgs]
    # request 2 (30 bytes) would fit beside request 0 at once, but waits
    # behind request 1 (60 bytes), which waits for request 0 to retire
    assert recs[2].admitted >= recs[0].finished
    assert recs[2].admitted >= recs[1].admitted
    assert all(r.status == "done" for r in recs.values())
    assert stats["status"] == {"done": 4}
    assert pool.used == 0 and not pool.sims


def test_head_of_line_blocks_until_memory_frees():
    big, small = Cfg(80, 2), Cfg(10, 1)
    reqs = [Req(0, 0.0, Cfg(50, 5)), Req(1, 0.001, big), Req(2, 0.002, small)]
    pool = FakePool(100, 8)
    recs, _ = run(pool, reqs)
    # the small request fits at once but queues behind the big one (FIFO)
    assert recs[1].admitted >= recs[0].finished
    assert recs[2].admitted >= recs[1].admitted
    assert all(r.status == "done" for r in recs.values())


def test_request_larger_than_the_pool_is_rejected_not_stalled():
    reqs = [Req(0, 0.0, Cfg(40, 2)), Req(1, 0.001, Cfg(500, 2)), Req(2, 0.002, Cfg(40, 2))]
    pool = FakePool(100, 8)
    recs, stats = run(pool, reqs)
    assert recs[1].status == "rejected" and "empty pool" in recs[1].error
    assert recs[0].status == "done" and recs[2].status == "done"
    assert stats["status"] == {"done": 2, "rejected": 1}


def test_parameters_the_pool_refuses_are_rejected():
    reqs = [Req(0, 0.0, Cfg(10, 2, invalid=True)), Req(1, 0.0, Cfg(10, 3))]
    recs, _ = run(FakePool(100, 8), reqs)
    assert recs[0].status == "rejected" and "bad parameters" in recs[0].error
    assert recs[1].status == "done" and recs[1].steps == 3


def test_cancellation_queued_and_running():
    pool = FakePool(100, 8)
    reqs = [Req(0, 0.0, Cfg(90, 1000), cancel_at=0.05),    # cancelled while running
            Req(1, 0.001, Cfg(90, 5), cancel_at=0.02),      # cancelled while queued behind 0
            Req(2, 0.002, Cfg(90, 4))]
    recs, stats = run(pool, reqs)
    assert recs[0].status == "cancelled" and 0 < recs[0].steps < 1000
    assert recs[1].status == "cancelled" and recs[1].steps == 0
    assert recs[2].status == "done" and recs[2].steps == 4
    assert pool.used == 0


def test_nonfinite_simulation_is_evicted_others_continue():
    pool = FakePool(1000, 8)
    reqs = [Req(0, 0.0, Cfg(10, 30)), Req(1, 0.0, Cfg(10, 30, nan_at=7)), Req(2, 0.0, Cfg(10, 30))]
    recs, stats = run(pool, reqs, check_every=5)
    assert recs[1].status == "failed" and recs[1].steps == 10   # found at the first check after step 7
    assert recs[0].status == "done" and recs[0].steps == 30
    assert recs[2].status == "done" and recs[2].steps == 30
    assert stats["status"] == {"done": 2, "failed": 1}
    # the throughput counts every step taken, the failed simulation's too
    assert stats["dof_steps"] == 30 + 10 + 30


def test_slots_bound_the_batch():
    pool = FakePool(10 ** 6, 2)
    reqs = [Req(i, 0.0, Cfg(1, 3)) for i in range(5)]
    recs, _ = run(pool, reqs)
    assert all(r.status == "done" for r in recs.values())
    # at most two in flight: the third starts after one of the first two ends
    assert recs[2].admitted >= min(recs[0].finished, recs[1].finished)


def test_per_request_records(tmp_path):
    import json
    path = str(tmp_path / "records.jsonl")
    pool = FakePool(100, 8)
    reqs = [Req(0, 0.0, Cfg(40, 3)), Req(1, 0.001, Cfg(500, 2)), Req(2, 0.002, Cfg(40, 2))]
    clk = Clock()
    recs, _ = serve(pool, reqs, setup=lambda sim, cfg: None, steps_of=lambda r: r.cfg.steps,
                    dofs_of=lambda r: 10, clock=clk, sleep=clk.sleep, max_wall=1e4, records_path=path)
    lines = [json.loads(x) for x in open(path)]
    assert [x["rid"] for x in lines] == [0, 1, 2]
    assert [x["status"] for x in lines] == ["done", "rejected", "done"]
    assert lines[0]["dof_steps"] == 30 and lines[0]["steps"] == 3 and lines[0]["step_ms_p99"] == 1.0
    assert lines[1]["admitted_s"] is None and lines[1]["dof_steps"] == 0
