"""Batched pool (serving form): every result is bitwise the same alone and in
the mix, with simulations of different problems, meshes, degrees and
precisions joining and leaving the batch; graph replay equals direct
launches; admission is by workspace bytes."""
import numpy as np
import pytest

import workloads as W
from runners import gpu_sim, oracle_pwave, rel_l2

pytestmark = pytest.mark.gpu


def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


MIX = [
    W.C1.with_(nelem=(20, 17, 23), tau=0.01),
    W.C1.with_(nelem=(13, 11, 9), p=3, q=4, tau=0.01),
    W.C1.with_(nelem=(24, 16, 20), tau=0.005, precision="mixed_fp32"),
    W.C4.with_(nelem=(9, 8, 10), tau=0.01),
    W.C4.with_(nelem=(6, 7, 5), p=3, q=4, tau=0.02, lam=2.0, mu=0.5),
    W.C4.with_(nelem=(11, 7, 9), tau=0.01, precision="mixed_fp32"),
    W.C2.with_(nelem=(16, 18, 14), steps=100),           # P-wave p=3 with a point source
]


def _setup(sim, cfg):
    import torch
    xs = [sim.quad_points(d) for d in range(3)]
    u0 = sim.project(torch.from_numpy(np.ascontiguousarray(W.initial_values(cfg, *xs))).to("cuda"))
    sim.set_state(u0, None, None, 0)
    if cfg.load == "ricker_point":
        sim.set_point_load(W.source_point(cfg.seed), W.load_amplitudes(cfg))
    sim.factor()


def _alone(cfg, nsteps):
    sim, _ = gpu_sim(cfg, precision=cfg.precision)
    sim.factor()
    sim.step(nsteps)
    out = [t.cpu().numpy() for t in sim.get_state() if t is not None]
    sim.close()
    return out


@pytest.mark.parametrize("use_graph,branches", [(True, 2), (False, 2), (True, 1), (False, 1)])
def test_alone_equals_mix_with_staggered_joins(use_graph, branches):
    """Two concurrent branches (the default) or one; a profiled step (one
    branch, direct launches) in the middle of the run."""
    _cuda()
    from paper_1911_08158_amd import Pool
    nsteps = 6
    ref = [_alone(c, nsteps) for c in MIX]
    pool = Pool(512 << 20, max_slots=16, use_graph=use_graph)
    pool.set_branches(branches)
    sims = []
    done = {}
    # first half joins at step 0, second half after two pool steps
    for c in MIX[:3]:
        s = pool.admit(c)
        _setup(s, c)
        pool.activate(s)
        sims.append((s, c, 0))
    pool.step(2)
    for c in MIX[3:]:
        s = pool.admit(c)
        _setup(s, c)
        pool.activate(s)
        sims.append((s, c, 2))
    for k in range(2, 2 + nsteps):
        if k == 3:
            pool.profile(True)
            pool.step(1)
            pool.profile_read()
            pool.profile(False)
        else:
            pool.step(1)
        for s, c, t0 in sims:
            if s.slot in done:
                continue
            if k + 1 - t0 == nsteps:
                done[s.slot] = [t.cpu().numpy() for t in s.get_state() if t is not None]
                assert s.step_index() == nsteps
                pool.retire(s)
    assert len(done) == len(MIX)
    for (s, c, _), r in zip(sims, ref):
        out = done[s.slot]
        for x, y in zip(out, r):
            assert np.array_equal(x, y), c
    times = pool.step_times()
    assert len(times) == 2 + nsteps and np.all(times > 0)
    pool.close()


def test_pool_matches_oracle_and_mixed_error():
    """A pooled FP64 run matches the oracle; a pooled mixed run stays within
    1e-6 of it."""
    _cuda()
    from paper_1911_08158_amd import Pool
    cfg = W.C1.with_(nelem=(18, 20, 16), tau=0.01, steps=10)
    pw, u0, (ur, vr, ar) = oracle_pwave(cfg, cfg.steps)
    pool = Pool(256 << 20, max_slots=4)
    sims = []
    for prec in ("fp64", "mixed_fp32"):
        s = pool.admit(cfg, precision=prec)
        import torch
        s.set_state(torch.from_numpy(pw.to_full(u0)).cuda(), None, None, 0)
        s.factor()
        pool.activate(s)
        sims.append(s)
    pool.step(cfg.steps)
    e64 = rel_l2(sims[0].get_state()[0].cpu().numpy(), pw.to_full(ur))
    e32 = rel_l2(sims[1].get_state()[0].cpu().numpy(), pw.to_full(ur))
    assert e64 <= 1e-12 and e32 <= 1e-6, (e64, e32)
    pool.close()


@pytest.mark.parametrize("cfg", [W.C1.with_(nelem=(14, 12, 10), tau=0.01, steps=6),
                                 W.C4.with_(nelem=(7, 6, 8), tau=0.02, steps=4)], ids=["pwave", "elastic"])
def test_admit_with_fields_and_retire_with_state(cfg):
    """ads_pool_admit takes the initial coefficients and ads_pool_retire
    hands back the final state: bitwise the run of the same fields alone
    (ads_create with them); the P-wave also against the oracle; the freed
    memory takes the next admission."""
    _cuda()
    import torch
    from paper_1911_08158_amd import Pool, Sim
    if cfg.problem == "pwave":
        pw, u0r, (ur, vr, ar) = oracle_pwave(cfg, cfg.steps)
        u0 = torch.from_numpy(pw.to_full(u0r)).cuda()
        v0 = torch.zeros_like(u0)
    else:
        from paper_1911_08158_amd.binding import Params
        n = Params.of(cfg).full_numel
        g = np.random.default_rng(7)
        u0 = torch.from_numpy(g.uniform(-1, 1, n)).cuda()
        v0 = torch.from_numpy(g.uniform(-1, 1, n)).cuda()
    alone = Sim(cfg, device="cuda", u0=u0, v0=v0)
    alone.factor()
    alone.step(cfg.steps)
    ref = [t.cpu().numpy() for t in alone.get_state() if t is not None]
    alone.close()
    pool = Pool(128 << 20, max_slots=4)
    s = pool.admit(cfg, u0=u0, v0=v0)
    slot = s.slot
    s.factor()
    pool.activate(s)
    pool.step(cfg.steps)
    got = [t.cpu().numpy() for t in pool.retire(s, state=True) if t is not None]
    assert len(got) == len(ref)
    for x, y in zip(got, ref):
        assert np.array_equal(x, y)
    if cfg.problem == "pwave":
        for x, r in zip(got, (ur, vr, ar)):
            assert rel_l2(x, pw.to_full(r)) <= 1e-12
    nxt = pool.admit(cfg)
    assert nxt is not None and nxt.slot == slot
    assert pool.retire(nxt) is None
    pool.close()


def test_admission_by_memory():
    _cuda()
    from paper_1911_08158_amd import Pool
    from paper_1911_08158_amd.binding import Params, workspace_bytes
    cfg = W.C1.with_(nelem=(48, 48, 48))
    need = workspace_bytes(Params.of(cfg))
    assert need > (4 << 20)
    # job tables (< 1 MiB for 8 slots) + room for 3.5 simulations
    pool = Pool((1 << 20) + int(3.5 * need), max_slots=8)
    got = [pool.admit(cfg) for _ in range(4)]
    assert all(g is not None for g in got[:3]) and got[3] is None
    info = pool.info()
    assert info["used_bytes"] >= 3 * need
    pool.retire(got[1])
    again = pool.admit(cfg)
    assert again is not None and again.slot == got[1].slot
    pool.close()


def test_benchmark_batch_full_size():
    """The configuration the benchmark times: four 128^3 p=2 simulations with
    the mixed-precision right-hand side in one pool, one graph replay per
    step.  They start from different seeded fields; each equals its run
    alone bitwise, and the first stays within 1e-6 of the FP64 oracle
    (started from the oracle's projection)."""
    _cuda()
    import torch
    from paper_1911_08158_amd import Pool
    from paper_1911_08158_amd.binding import Params, workspace_bytes
    nsteps = 10
    cfgs = [W.C3.with_(steps=nsteps)] + [W.C3.with_(steps=nsteps, init=f"gauss1:{k}") for k in (11, 12, 13)]
    pw, u0, (ur, _, _) = oracle_pwave(cfgs[0], nsteps)
    starts = [pw.to_full(u0), None, None, None]
    need = workspace_bytes(Params.of(cfgs[0], precision="mixed_fp32"))
    pool = Pool((8 << 20) + 4 * (need + 4096), max_slots=4, use_graph=True)
    sims = []
    for c, u in zip(cfgs, starts):
        s = pool.admit(c, precision="mixed_fp32")
        if u is None:
            _setup(s, c)
        else:
            s.set_state(torch.from_numpy(u).cuda(), None, None, 0)
            s.factor()
        pool.activate(s)
        sims.append(s)
    pool.step(nsteps)
    outs = [[t.cpu().numpy() for t in s.get_state() if t is not None] for s in sims]
    pool.close()
    e = rel_l2(outs[0][0], pw.to_full(ur))
    print(f"batched 4 x 128^3 mixed, {nsteps} steps: rel L2 u {e:.3e}", flush=True)
    assert e <= 1e-6, e
    for c, u, out in zip(cfgs, starts, outs):
        sim, _ = gpu_sim(c, precision="mixed_fp32", u0_full=u)
        sim.factor()
        sim.step(nsteps)
        ref = [t.cpu().numpy() for t in sim.get_state() if t is not None]
        sim.close()
        for x, y in zip(out, ref):
            assert np.array_equal(x, y), c.init


def test_tune_refused_for_pooled_sim_and_pool_matches_oracle():
    """ads_tune on a pooled simulation is refused (ADS_ESTATE): the pool fixes
    its launch classes, and a changed right-hand-side variant would match no
    class and leave the simulation without a right-hand side.  The pooled
    run that follows is checked against the oracle, as is a simulation whose
    load is replaced while it is in the batch (the pool gathers its jobs
    again)."""
    _cuda()
    import torch
    from paper_1911_08158_amd import Pool
    from paper_1911_08158_amd.binding import AdsError
    cfg = W.C2.with_(nelem=(12, 10, 14), steps=8)
    pw, u0_ref, (_, hist) = oracle_pwave(cfg, cfg.steps, history=True)
    pool = Pool(256 << 20, max_slots=4)
    s = pool.admit(cfg)
    s.set_state(torch.from_numpy(np.ascontiguousarray(pw.to_full(u0_ref))).to("cuda"), None, None, 0)
    s.set_point_load(W.source_point(cfg.seed), W.load_amplitudes(cfg))
    s.factor()
    with pytest.raises(AdsError) as e:
        s.tune()
    assert e.value.status == -4
    pool.activate(s)
    pool.step(4)
    # the same load again, set while the simulation is in the batch
    s.set_point_load(W.source_point(cfg.seed), W.load_amplitudes(cfg))
    pool.step(cfg.steps - 4)
    u, v, a = s.get_state()
    for x, r in zip((u, v, a), hist[cfg.steps]):
        assert rel_l2(x.cpu().numpy(), pw.to_full(r)) <= 1e-12
    pool.retire(s)
    pool.close()


def test_serve_evicts_nonfinite_and_rejects_what_never_fits():
    """The serving loop on the real pool: a simulation whose initial state is
    NaN is evicted at its first health check while the others run on; a
    request larger than the empty pool and one the pool refuses (more than
    128 free coefficients per direction) are rejected instead of stalling
    the queue; every completed result is bitwise the simulation run alone."""
    _cuda()
    import dataclasses

    import torch
    from paper_1911_08158_amd import Pool
    from paper_1911_08158_amd.serve import serve

    cfgs = [W.C1.with_(name="ok0", nelem=(20, 17, 23), tau=0.01, steps=6, precision="mixed_fp32"),
            W.C1.with_(name="nan", nelem=(12, 11, 9), tau=0.01, steps=6),
            W.C4.with_(name="big", nelem=(96, 96, 96), tau=0.01, steps=6),
            W.C1.with_(name="ok1", nelem=(9, 8, 10), p=3, q=4, tau=0.01, steps=6),
            W.C1.with_(name="wide", nelem=(200, 4, 4), tau=0.01, steps=6),
            W.C4.with_(name="ok2", nelem=(7, 6, 8), tau=0.02, steps=6, precision="mixed_fp32")]

    @dataclasses.dataclass
    class Req:
        rid: int
        arrival: float
        cfg: object

    def setup(sim, cfg):
        xs = [sim.quad_points(d) for d in range(3)]
        u0 = sim.project(torch.from_numpy(np.ascontiguousarray(W.initial_values(cfg, *xs))).to("cuda"))
        if cfg.name == "nan":
            u0 = u0 * float("nan")
        sim.set_state(u0, None, None, 0)
        sim.factor()

    pool = Pool(64 << 20, max_slots=8)
    recs, stats = serve(pool, [Req(i, 0.0, c) for i, c in enumerate(cfgs)], setup,
                        steps_of=lambda r: r.cfg.steps, dofs_of=lambda r: r.cfg.dofs(),
                        keep_results=True, check_every=2)
    pool.close()
    st = {cfgs[r.rid].name: r for r in recs}
    print({k: (v.status, v.steps, v.error) for k, v in st.items()}, flush=True)
    assert st["nan"].status == "failed" and st["nan"].steps == 2
    assert st["big"].status == "rejected" and st["wide"].status == "rejected"
    for name in ("ok0", "ok1", "ok2"):
        r = st[name]
        assert r.status == "done" and r.steps == 6
        cfg = cfgs[r.rid]
        ref = _alone(cfg, 6)
        got = [x for x in r.result if x is not None]
        for x, y in zip(got, ref):
            assert np.array_equal(x, y), name


def test_pool_tune_keeps_results_and_caches():
    """ads_pool_tune times the right-hand-side variants and the sweep tile
    widths on the batch, keeps the fastest per class, and the tuned batch
    still matches the oracle (FP64 bar); a second call on the same batch
    shape takes the cached choices and changes nothing."""
    _cuda()
    import torch
    from paper_1911_08158_amd import Pool
    cfgs = [W.C1.with_(nelem=(20, 17, 23), tau=0.01, steps=5),
            W.C1.with_(nelem=(13, 11, 9), p=3, q=4, tau=0.01, steps=5)]
    refs = [oracle_pwave(c, c.steps, history=True) for c in cfgs]
    pool = Pool(128 << 20, max_slots=4)
    sims = []
    for c, (pw, u0, _) in zip(cfgs, refs):
        s = pool.admit(c)
        s.set_state(torch.from_numpy(pw.to_full(u0)).cuda(), None, None, 0)
        s.factor()
        pool.activate(s)
        sims.append(s)
    n1, shapes = pool.tune()
    launched = shapes[shapes >= 0]
    print(f"tuned shapes {launched.tolist()}, {n1} changed", flush=True)
    assert launched.size >= 4
    n2, shapes2 = pool.tune()
    assert n2 == 0 and np.array_equal(shapes, shapes2)
    pool.step(5)
    for s, c, (pw, _, (_, hist)) in zip(sims, cfgs, refs):
        u, v, a = (t.cpu().numpy() for t in s.get_state())
        for x, r in zip((u, v, a), hist[5]):
            assert rel_l2(x, pw.to_full(r)) <= 1e-12
    pool.close()


def test_pool_tune_with_field_in_mixed_mode():
    """The pool's tuner on a class of mixed-mode simulations with a
    wave-speed field (its candidates include the MFMA x-stage, variant 4):
    the tuned batch stays within the mixed bar of the FP64 oracle."""
    _cuda()
    import torch
    from oracle import pwave
    from runners import oracle_bc
    from paper_1911_08158_amd import Pool
    cfgs = [W.C1.with_(nelem=(12, 10, 9), tau=0.01, steps=6),
            W.C1.with_(nelem=(11, 9, 10), p=3, q=4, tau=0.01, steps=6)]
    pool = Pool(128 << 20, max_slots=4)
    runs = []
    for c in cfgs:
        base = pwave.PWave(c.nelem, c.p, c.q, c.tau, bc=oracle_bc(c))
        xs = [base.quad_points(d) for d in range(3)]
        c2 = W.wave_speed_field(*xs)
        pw = pwave.PWave(c.nelem, c.p, c.q, c.tau, bc=oracle_bc(c), coef=c2, c2ref=1.5)
        u0 = pw.project(W.initial_values(c, *xs))
        _, hist = pw.run(u0, None, c.steps, history=True)
        s = pool.admit(c, precision="mixed_fp32", u0=torch.from_numpy(pw.to_full(u0)).cuda())
        s.set_coefficient(torch.from_numpy(c2).cuda(), 1.5)
        s.factor()
        pool.activate(s)
        runs.append((s, pw, hist))
    n, shapes = pool.tune()
    print(f"tuned shapes {shapes[shapes >= 0].tolist()}", flush=True)
    pool.step(cfgs[0].steps)
    for s, pw, hist in runs:
        u = s.get_state()[0].cpu().numpy()
        e = rel_l2(u, pw.to_full(hist[-1][0]))
        assert 0 < e <= 1e-6, e
    pool.close()


def test_pool_tune_chooses_coupling_form_bitwise_with_alone():
    """The pool's tuner times the two forms of the elasticity couplings on
    the batch (its in-plane launches hold the planes of every simulation)
    and applies its choice to every pooled elasticity simulation; each then
    runs bitwise as the same simulation alone that switches to that form
    after ads_factor (the start, computed there, used the default form, as
    in the pool), and the two elasticity runs stay within 1e-12 of the
    oracle."""
    _cuda()
    import torch
    from paper_1911_08158_amd import Pool
    from runners import oracle_elastic
    # the third elasticity mesh has planes of 82 x 72 unknowns, too large
    # for the in-plane stage: it keeps separate launches, and its in-plane
    # jobs share the launch class of the others' coupled ones
    cfgs = [W.C4.with_(nelem=(6, 5, 40), tau=0.02, steps=4),
            W.C4.with_(nelem=(5, 6, 30), p=3, q=4, tau=0.02, steps=4, lam=2.0, mu=0.5),
            W.C1.with_(nelem=(9, 8, 7), tau=0.01, steps=4),
            W.C4.with_(nelem=(80, 70, 3), tau=0.01, steps=4, bc="natural")]
    pool = Pool(128 << 20, max_slots=4)
    sims, refs = [], []
    for c in cfgs:
        s = pool.admit(c)
        _setup(s, c)
        pool.activate(s)
        sims.append(s)
    n, _ = pool.tune()
    forms = [s.coupling_fused for s in sims]
    print(f"pool coupling form: {'in-plane' if forms[0] else 'separate'} ({n} changed)", flush=True)
    assert forms[0] == forms[1] and not forms[2] and not forms[3]
    n2, _ = pool.tune()
    assert n2 == 0
    pool.step(4)
    pooled = [[t.cpu().numpy() for t in s.get_state() if t is not None] for s in sims]
    pool.close()
    for c, fused, got in zip(cfgs, forms, pooled):
        sim, _ = gpu_sim(c)
        sim.factor()
        if c.problem == "elastic":
            sim.set_coupling(fused)
        sim.step(4)
        want = [t.cpu().numpy() for t in sim.get_state() if t is not None]
        sim.close()
        for x, y in zip(got, want):
            assert np.array_equal(x, y)
        if c.problem == "elastic":
            el, U0, (_, hist) = oracle_elastic(c, c.steps, history=True)
            sim, _ = gpu_sim(c, u0_full=el.to_full(U0), coupling=fused)
            sim.factor()
            sim.step(4)
            u, v, _ = sim.get_state()
            assert max(rel_l2(u.cpu().numpy(), el.to_full(hist[4][0])),
                       rel_l2(v.cpu().numpy(), el.to_full(hist[4][1]))) <= 1e-12
            sim.close()
