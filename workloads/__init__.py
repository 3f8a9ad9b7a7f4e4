"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds NO arithmetic of the solver method: it only names the
workload presets (element counts, spline degree, time step, step count) and
evaluates the analytic initial data / load time profiles at points that the
caller supplies.  Each side (oracle, HIP library) computes its own Gauss
points and basis functions and feeds them here, so the two implementations
share no code beyond these input recipes.

Workloads (the paper gives mesh size and time step only, Sections 4 and 7;
everything else is a stated synthetic recipe):

* ``C1``  P-wave, 16^3 elements, p=2, q=3, tau=1e-2, 10 steps, FP64,
          u0 = exp(-200 |x - 0.5|^2), v0 = 0, f = 0.
* ``C2``  P-wave, 64^3 elements, p=3, q=4, tau=5e-3, 100 steps, FP64,
          u0 = sum of 8 seeded Gaussians, Ricker point source (10 Hz).
* ``C3``  P-wave, 128^3 elements, p=2, q=3, tau=2e-3, 100 steps,
          u0 = C1's bump, f = 0 (mixed-precision RHS variants).
* ``C4``  elasticity, 64^3 elements, p=2, lambda=mu=rho=1, tau=5e-3,
          100 steps, U0 = curl-free + divergence-free Gaussian pulse.
* ``C5``  serving mix: Poisson arrivals of P-wave / elasticity requests.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

MASTER_SEED = 20191118


@dataclasses.dataclass(frozen=True)
class SimConfig:
    name: str
    problem: str            # "pwave" | "elastic"
    nelem: tuple            # elements per direction (x, y, z)
    p: int                  # spline degree
    q: int                  # Gauss points per element per direction
    tau: float
    steps: int
    precision: str = "fp64"  # "fp64" | "mixed_fp32" | "mixed_bf16"
    rho: float = 1.0
    lam: float = 1.0
    mu: float = 1.0
    init: str = "bump"      # "bump" | "gauss8" | "elastic_pulse" | "noise" | "gauss1:<seed>"
    load: str = "none"      # "none" | "ricker_point"
    seed: int = MASTER_SEED
    bc: str = "dirichlet"   # "dirichlet" (zero) | "natural" (zero normal derivative / traction-free)

    @property
    def n(self):
        """Basis functions per direction (open knots, maximal continuity);
        nelem[2] = 0 is the two-dimensional problem (one z-layer)."""
        return tuple(1 if (d == 2 and e == 0) else e + self.p for d, e in enumerate(self.nelem))

    @property
    def comps(self):
        return 3 if self.problem == "elastic" else 1

    def dofs(self):
        """DOF count used by the throughput metric: all n^3 coefficients per
        component, boundary ones included."""
        nx, ny, nz = self.n
        return nx * ny * nz * self.comps

    def with_(self, **kw):
        return dataclasses.replace(self, **kw)


C1 = SimConfig("C1", "pwave", (16, 16, 16), 2, 3, 1e-2, 10)
C2 = SimConfig("C2", "pwave", (64, 64, 64), 3, 4, 5e-3, 100,
               init="gauss8", load="ricker_point")
C3 = SimConfig("C3", "pwave", (128, 128, 128), 2, 3, 2e-3, 100,
               precision="mixed_fp32")
C4 = SimConfig("C4", "elastic", (64, 64, 64), 2, 3, 5e-3, 100,
               init="elastic_pulse")
PRESETS = {c.name: c for c in (C1, C2, C3, C4)}


# ---------------------------------------------------------------------------
# analytic initial data
# ---------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class GaussianSum:
    centres: np.ndarray   # (k, 3) in (x, y, z)
    widths: np.ndarray    # (k,) standard deviations
    amps: np.ndarray      # (k,)


def bump() -> GaussianSum:
    """exp(-200 |x - 0.5|^2): one Gaussian with 2 w^2 = 1/200."""
    return GaussianSum(np.array([[0.5, 0.5, 0.5]]), np.array([math.sqrt(1.0 / 400.0)]),
                       np.array([1.0]))


def gauss8(seed: int = MASTER_SEED) -> GaussianSum:
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.2, 0.8, size=(8, 3))
    widths = rng.uniform(0.02, 0.08, size=8)
    return GaussianSum(centres, widths, np.ones(8))


def eval_gaussian_sum(g: GaussianSum, xs, ys, zs) -> np.ndarray:
    """Values of sum_k A_k exp(-|x-c_k|^2 / (2 w_k^2)) on the tensor grid
    xs x ys x zs, returned as an array indexed [z, y, x]."""
    xs, ys, zs = (np.asarray(a, dtype=np.float64) for a in (xs, ys, zs))
    out = np.zeros((zs.size, ys.size, xs.size))
    for c, w, a in zip(g.centres, g.widths, g.amps):
        s = 1.0 / (2.0 * w * w)
        fx = np.exp(-s * (xs - c[0]) ** 2)
        fy = np.exp(-s * (ys - c[1]) ** 2)
        fz = np.exp(-s * (zs - c[2]) ** 2)
        out += a * fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    return out


@dataclasses.dataclass(frozen=True)
class ElasticPulse:
    c_phi: np.ndarray     # centre of the scalar potential Gaussian
    c_psi: np.ndarray     # centre of the vector potential Gaussian
    width: float
    axis: np.ndarray      # unit vector of the vector potential


def elastic_pulse(seed: int = MASTER_SEED) -> ElasticPulse:
    rng = np.random.default_rng(seed + 4)
    c1 = rng.uniform(0.3, 0.7, size=3)
    c2 = rng.uniform(0.3, 0.7, size=3)
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    return ElasticPulse(c1, c2, 0.05, a)


def eval_elastic_pulse(ep: ElasticPulse, xs, ys, zs) -> np.ndarray:
    """w * (grad phi + curl(psi a)) with Gaussian phi, psi of width w,
    on the grid xs x ys x zs; returns [3, z, y, x] (components x, y, z).
    The factor w makes the amplitude O(1)."""
    xs, ys, zs = (np.asarray(a, dtype=np.float64) for a in (xs, ys, zs))
    w = ep.width
    s = 1.0 / (2.0 * w * w)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    d1 = [X - ep.c_phi[0], Y - ep.c_phi[1], Z - ep.c_phi[2]]
    d2 = [X - ep.c_psi[0], Y - ep.c_psi[1], Z - ep.c_psi[2]]
    phi = np.exp(-s * (d1[0] ** 2 + d1[1] ** 2 + d1[2] ** 2))
    psi = np.exp(-s * (d2[0] ** 2 + d2[1] ** 2 + d2[2] ** 2))
    gphi = [-2.0 * s * d * phi for d in d1]
    gpsi = [-2.0 * s * d * psi for d in d2]
    a = ep.axis
    curl = [gpsi[1] * a[2] - gpsi[2] * a[1],
            gpsi[2] * a[0] - gpsi[0] * a[2],
            gpsi[0] * a[1] - gpsi[1] * a[0]]
    return w * np.stack([gphi[i] + curl[i] for i in range(3)])


def initial_values(cfg: SimConfig, xs, ys, zs) -> np.ndarray:
    """Initial displacement sampled at the tensor grid of points; [z,y,x] for
    the P-wave, [3,z,y,x] for elasticity."""
    if cfg.init == "bump":
        return eval_gaussian_sum(bump(), xs, ys, zs)
    if cfg.init == "gauss8":
        return eval_gaussian_sum(gauss8(cfg.seed), xs, ys, zs)
    if cfg.init == "elastic_pulse":
        return eval_elastic_pulse(elastic_pulse(cfg.seed), xs, ys, zs)
    if cfg.init == "noise":
        # seeded white noise at the points (broad spectrum; indexed by point
        # order, so both sides see the same values at their own points)
        rng = np.random.default_rng(cfg.seed + 3)
        shape = (len(zs), len(ys), len(xs))
        v = rng.uniform(-1.0, 1.0, size=((3,) if cfg.problem == "elastic" else ()) + shape)
        return v
    if cfg.init.startswith("gauss1:"):
        # single seeded bump used by the serving mix: "gauss1:<seed>"
        s = int(cfg.init.split(":")[1])
        rng = np.random.default_rng(s)
        g = GaussianSum(rng.uniform(0.3, 0.7, size=(1, 3)),
                        rng.uniform(0.03, 0.08, size=1), np.ones(1))
        v = eval_gaussian_sum(g, xs, ys, zs)
        return np.stack([v, 0.5 * v, -0.25 * v]) if cfg.problem == "elastic" else v
    raise ValueError(cfg.init)


def greville_abscissae(E: int, p: int) -> np.ndarray:
    """Averages of p consecutive interior knots of the open uniform knot
    vector with E elements (where a spline coefficient 'sits')."""
    t = np.concatenate([np.zeros(p + 1), np.arange(1, E) / E, np.ones(p + 1)])
    return np.array([t[i + 1:i + p + 1].mean() for i in range(E + p)])


def initial_coefficients(cfg: SimConfig) -> np.ndarray:
    """Cheap initial coefficients for the serving mix: the initial function
    sampled at the Greville abscissae (boundary coefficients set to 0, the
    zero-Dirichlet value).  Full layout [z, y, x] or [3, z, y, x]."""
    xs, ys, zs = (greville_abscissae(cfg.nelem[d], cfg.p) for d in range(3))
    c = np.array(initial_values(cfg, xs, ys, zs))
    if cfg.bc != "dirichlet":
        return np.ascontiguousarray(c)
    c[..., 0, :, :] = 0
    c[..., -1, :, :] = 0
    c[..., :, 0, :] = 0
    c[..., :, -1, :] = 0
    c[..., :, :, 0] = 0
    c[..., :, :, -1] = 0
    return np.ascontiguousarray(c)


def wave_speed_field(xs, ys, zs, amp: float = 0.5) -> np.ndarray:
    """Smooth squared wave speed c^2 = 1 + amp sin(2 pi x) cos(2 pi y) sin(2 pi z + 0.3)
    on the tensor grid of the given points, [z, y, x] (values in [1 - amp, 1 + amp])."""
    xs, ys, zs = (np.asarray(v, dtype=np.float64) for v in (xs, ys, zs))
    return 1.0 + amp * (np.sin(2 * np.pi * zs + 0.3)[:, None, None] * np.cos(2 * np.pi * ys)[None, :, None]
                        * np.sin(2 * np.pi * xs)[None, None, :])


# ---------------------------------------------------------------------------
# loads
# ---------------------------------------------------------------------------
RICKER_F0 = 10.0
RICKER_T0 = 0.1


def ricker(t, f0: float = RICKER_F0, t0: float = RICKER_T0):
    """Ricker wavelet (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2)."""
    a = (math.pi * f0 * (np.asarray(t, dtype=np.float64) - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def source_point(seed: int = MASTER_SEED) -> np.ndarray:
    rng = np.random.default_rng(seed + 1)
    return rng.uniform(0.2, 0.8, size=3)


def load_amplitudes(cfg: SimConfig, nsteps: Optional[int] = None) -> np.ndarray:
    """Amplitude r(t_k) of the load at t_k = k tau, k = 0..nsteps."""
    ns = cfg.steps if nsteps is None else nsteps
    t = cfg.tau * np.arange(ns + 1)
    if cfg.load == "ricker_point":
        return ricker(t)
    return np.zeros(ns + 1)


# ---------------------------------------------------------------------------
# serving mix
# ---------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    arrival: float          # seconds after the stream starts
    cfg: SimConfig


def serving_mix(nreq: int = 200, rate: float = 1.0, seed: int = MASTER_SEED,
                sizes: Sequence[int] = (32, 48, 64, 96), degrees=(2, 3),
                taus=(1e-3, 5e-3), steps: int = 50, elastic_frac: float = 0.5,
                precision: str = "mixed_fp32") -> List[Request]:
    """Poisson stream of requests with per-direction element counts drawn
    independently from ``sizes``."""
    rng = np.random.default_rng(seed + 2)
    t = 0.0
    out = []
    for i in range(nreq):
        t += rng.exponential(1.0 / rate)
        prob = "elastic" if rng.uniform() < elastic_frac else "pwave"
        ne = tuple(int(rng.choice(sizes)) for _ in range(3))
        p = int(rng.choice(degrees))
        tau = float(rng.choice(taus))
        cfg = SimConfig(f"req{i}", prob, ne, p, p + 1, tau, steps, precision=precision,
                        init=f"gauss1:{seed + 1000 + i}")
        out.append(Request(i, t, cfg))
    return out
