"""Shared drivers for the parity tests: the same seeded workload run through
the HIP library (via the C-ABI binding) and through the CPU oracle.  The two
runs share only the input recipes of ``workloads``."""
from __future__ import annotations

import numpy as np

import workloads as W


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    nr = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (nr if nr > 0 else 1.0))


# ---------------------------------------------------------------- oracle side
def oracle_bc(cfg: W.SimConfig) -> str:
    """The oracle's name of the configuration's boundary condition."""
    return {"dirichlet": "dirichlet", "natural": "neumann"}[cfg.bc]


def oracle_pwave(cfg: W.SimConfig, nsteps: int, history: bool = False):
    from oracle import pwave
    pw = pwave.PWave(cfg.nelem, cfg.p, cfg.q, cfg.tau, bc=oracle_bc(cfg))
    xs = [pw.quad_points(d) for d in range(3)]
    u0 = pw.project(W.initial_values(cfg, *xs))
    b = amps = None
    if cfg.load == "ricker_point":
        b = pw.point_load(W.source_point(cfg.seed))
        amps = W.load_amplitudes(cfg, nsteps)
    res = pw.run(u0, None, nsteps, b, amps, history=history)
    return pw, u0, res


def oracle_elastic(cfg: W.SimConfig, nsteps: int, history: bool = False):
    from oracle import elastic
    el = elastic.Elastic(cfg.nelem, cfg.p, cfg.q, cfg.tau, rho=cfg.rho, lam=cfg.lam, mu=cfg.mu, bc=oracle_bc(cfg))
    xs = [el.b1[d].x for d in range(3)]
    vals = W.initial_values(cfg, *xs)
    from oracle import pwave
    # component-wise L2 projection with the same 1D structure
    pw = pwave.PWave(cfg.nelem, cfg.p, cfg.q, cfg.tau, bc=oracle_bc(cfg))
    U0 = np.stack([pw.project(vals[c]) for c in range(3)])
    res = el.run(U0, None, nsteps, history=history)
    return el, U0, res


# ------------------------------------------------------------------- GPU side
def gpu_sim(cfg: W.SimConfig, device="cuda", precision=None, u0_full=None, rhs_var=None, rhs_tz=None,
            coupling=None):
    """Create the GPU simulation.  Without ``u0_full`` the initial field is
    the library's own L2 projection of the seeded data; with it (a full
    coefficient array, e.g. the oracle's projection) both implementations
    start the time integration from identical coefficients, so that the
    parity of the stepping is not blurred by the rounding noise of two
    independent projections (u'' = G^{-1}(-K u) amplifies high-frequency
    differences of u by the stiffness).  rhs_var / rhs_tz: right-hand-side
    variant and z-tile depth set through ads_set_launch_shape; coupling
    (elasticity): True / False = the couplings in the in-plane sweeps or by
    separate launches (ads_set_coupling)."""
    import torch
    from paper_1911_08158_amd import Sim
    kw = {} if precision is None else {"precision": precision}
    sim = Sim(cfg, device=device, **kw)
    if rhs_var is not None or rhs_tz is not None:
        sim.set_launch_shape(-1 if rhs_var is None else rhs_var, -1 if rhs_tz is None else rhs_tz)
    if coupling is not None:
        sim.set_coupling(coupling)
    if u0_full is None:
        xs = [sim.quad_points(d) for d in range(3)]
        vals = torch.from_numpy(np.ascontiguousarray(W.initial_values(cfg, *xs))).to(device)
        u0 = sim.project(vals)
    else:
        u0 = torch.from_numpy(np.ascontiguousarray(u0_full)).to(device)
    sim.set_state(u0, None, None, 0)
    if cfg.load == "ricker_point":
        sim.set_point_load(W.source_point(cfg.seed), W.load_amplitudes(cfg))
    return sim, u0


def oracle_pwave_at(cfg: W.SimConfig, steps):
    """The oracle's P-wave run with the states (u, v, a) kept only after the
    steps listed in ``steps`` (a 128^3 history of every step would not fit
    comfortably in host memory).  Returns (pw, u0, {k: (u, v, a)})."""
    from oracle import pwave
    pw = pwave.PWave(cfg.nelem, cfg.p, cfg.q, cfg.tau, bc=oracle_bc(cfg))
    xs = [pw.quad_points(d) for d in range(3)]
    u0 = pw.project(W.initial_values(cfg, *xs))
    last = max(steps)
    F = lambda k: None
    if cfg.load == "ricker_point":
        b = pw.point_load(W.source_point(cfg.seed))
        amps = W.load_amplitudes(cfg, last)
        F = lambda k: amps[k] * b
    u, v = u0, np.zeros_like(u0)
    a = pw.initial_accel(u0, F(0))
    keep = {0: (u, v, a)} if 0 in steps else {}
    for k in range(1, last + 1):
        u, v, a = pw.step(u, v, a, F(k))
        if k in steps:
            keep[k] = (u, v, a)
    return pw, u0, keep


def oracle_elastic_at(cfg: W.SimConfig, steps):
    """The oracle's elasticity run with (U^n, U^{n-1}) kept only after the
    listed steps.  Returns (el, U0, {k: (U^k, U^{k-1})})."""
    from oracle import elastic, pwave
    el = elastic.Elastic(cfg.nelem, cfg.p, cfg.q, cfg.tau, rho=cfg.rho, lam=cfg.lam, mu=cfg.mu, bc=oracle_bc(cfg))
    vals = W.initial_values(cfg, *[el.b1[d].x for d in range(3)])
    pw = pwave.PWave(cfg.nelem, cfg.p, cfg.q, cfg.tau, bc=oracle_bc(cfg))
    U0 = np.stack([pw.project(vals[c]) for c in range(3)])
    keep = {}
    Un, Unm1 = U0, el.start(U0, None)
    for k in range(1, max(steps) + 1):
        Un, Unm1 = el.step(Un, Unm1), Un
        if k in steps:
            keep[k] = (Un, Unm1)
    return el, U0, keep
