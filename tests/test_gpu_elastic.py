"""GPU parity of the elasticity (alternating-triangular) hot path against the
CPU oracle, through the C-ABI.  Bar: relative L2 <= 1e-12 (FP64)."""
import numpy as np
import pytest

import workloads as W
from runners import gpu_sim, oracle_elastic, oracle_elastic_at, rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("cfg", [
    W.C4.with_(nelem=(6, 5, 7), steps=4, tau=0.02, lam=0.8, mu=0.6, rho=1.3),
    W.C4.with_(nelem=(17, 9, 11), steps=3, tau=0.01),
    W.C4.with_(nelem=(5, 6, 4), p=3, q=4, steps=3, tau=0.02, lam=2.0, mu=0.5, rho=0.9),
    W.C4.with_(nelem=(1, 2, 3), steps=2, tau=0.1, init="noise"),
    W.C4.with_(nelem=(8, 8, 8), steps=3, tau=2.0),
    W.C4.with_(nelem=(7, 5, 6), steps=4, tau=0.02, lam=0.8, mu=0.6, rho=1.3, bc="natural"),   # traction-free
    W.C4.with_(nelem=(4, 6, 5), p=3, q=4, steps=3, tau=0.02, lam=2.0, mu=0.5, bc="natural"),
], ids=lambda c: f"{c.nelem}-p{c.p}-tau{c.tau}-{c.bc}")
@pytest.mark.parametrize("form", ["band", "quadrature"])
def test_elastic_matches_oracle(cfg, form):
    """Both right-hand-side forms (Kronecker band passes, sum-factorized
    quadrature) against the oracle, step by step."""
    _cuda()
    var = 3 if form == "band" else 0
    el, U0_ref, (_, hist) = oracle_elastic(cfg, cfg.steps, history=True)
    sim, U0 = gpu_sim(cfg, rhs_var=var)
    assert rel_l2(U0.cpu().numpy(), el.to_full(U0_ref)) <= TOL
    sim.close()
    sim, _ = gpu_sim(cfg, u0_full=el.to_full(U0_ref), rhs_var=var)
    sim.factor()
    u, v, _ = sim.get_state()
    assert rel_l2(v.cpu().numpy(), el.to_full(hist[0][1])) <= TOL   # U^{-1}
    for k in range(1, cfg.steps + 1):
        sim.step(1)
        u, v, _ = sim.get_state()
        eu = rel_l2(u.cpu().numpy(), el.to_full(hist[k][0]))
        ev = rel_l2(v.cpu().numpy(), el.to_full(hist[k][1]))
        assert max(eu, ev) <= TOL, (k, eu, ev)
    sim.close()


@pytest.mark.parametrize("cfg,fits", [
    (W.C4.with_(nelem=(6, 5, 7), steps=4, tau=0.02, lam=0.8, mu=0.6, rho=1.3), True),
    (W.C4.with_(nelem=(5, 6, 4), p=3, q=4, steps=3, tau=0.02, lam=2.0, mu=0.5, rho=0.9), True),
    (W.C4.with_(nelem=(7, 5, 6), steps=4, tau=0.02, lam=0.8, mu=0.6, rho=1.3, bc="natural"), True),
    (W.C4.with_(nelem=(9, 7, 5), p=4, q=5, steps=3, tau=0.02), True),
    # 82 x 72 unknowns per plane: above the 4,608 the in-plane stage takes
    (W.C4.with_(nelem=(80, 70, 3), steps=3, tau=0.01, bc="natural"), False),
], ids=lambda c: f"{c.nelem}-p{c.p}-{c.bc}" if hasattr(c, "nelem") else str(c))
def test_coupling_forms(cfg, fits):
    """The couplings of the two stages (eq. pre, eq. corr) applied in the
    input stage of the in-plane sweeps and by separate launches: each
    against the oracle at every step (1e-12), the two forms within
    rounding of each other; the library reports the form that ran (the
    in-plane one only where the plane takes it)."""
    _cuda()
    el, U0_ref, (_, hist) = oracle_elastic(cfg, cfg.steps, history=True)
    runs = {}
    for fused in (True, False):
        sim, _ = gpu_sim(cfg, u0_full=el.to_full(U0_ref), coupling=fused)
        assert sim.coupling_fused == (fused and fits)
        sim.factor()
        for k in range(1, cfg.steps + 1):
            sim.step(1)
            u, v, _ = sim.get_state()
            eu = rel_l2(u.cpu().numpy(), el.to_full(hist[k][0]))
            ev = rel_l2(v.cpu().numpy(), el.to_full(hist[k][1]))
            assert max(eu, ev) <= TOL, (fused, k, eu, ev)
        runs[fused] = u.cpu().numpy()
        sim.close()
    assert rel_l2(runs[True], runs[False]) <= TOL


def test_tuned_coupling_form_matches_oracle():
    """ads_tune times both coupling forms on the mesh (a tall one with small
    planes, where the in-plane form has many workgroups) and keeps one; the
    step then matches the oracle (1e-12)."""
    _cuda()
    cfg = W.C4.with_(nelem=(6, 5, 40), steps=3, tau=0.02)
    el, U0_ref, (_, hist) = oracle_elastic(cfg, cfg.steps, history=True)
    sim, _ = gpu_sim(cfg, u0_full=el.to_full(U0_ref))
    assert not sim.coupling_fused   # default: separate launches
    sim.factor()
    sim.tune()
    print(f"tuned coupling form: {'in-plane' if sim.coupling_fused else 'separate'}", flush=True)
    for k in range(1, cfg.steps + 1):
        sim.step(1)
        u, v, _ = sim.get_state()
        assert max(rel_l2(u.cpu().numpy(), el.to_full(hist[k][0])),
                   rel_l2(v.cpu().numpy(), el.to_full(hist[k][1]))) <= TOL, k
    sim.close()


def test_coupling_form_refused_for_pwave():
    _cuda()
    from paper_1911_08158_amd import AdsError
    sim, _ = gpu_sim(W.C1.with_(nelem=(4, 4, 4), steps=1))
    with pytest.raises(AdsError):
        sim.set_coupling(False)
    assert not sim.coupling_fused
    sim.close()


# Mixed mode (FP32 stiffness-type passes on FP64 differences, FP64 mass
# channels, z-pass and update): relative L2 error of U^n against the FP64
# oracle after the 100 steps of C4.
MIXED_TOL = 1e-6


def test_elastic_c4_steps():
    """C4 (64^3, p=2, lambda = mu = rho = 1, tau = 5e-3): the full 100 steps;
    U^n and U^{n-1} compared in full at steps 1, 10, 50 and 100, in FP64
    (bar 1e-12) and in mixed mode (error stated, bar 1e-6 at step 100)."""
    _cuda()
    cfg = W.C4
    marks = (1, 10, 50, 100)
    el, U0_ref, keep = oracle_elastic_at(cfg, set(marks))
    for prec in ("fp64", "mixed_fp32"):
        sim, _ = gpu_sim(cfg, precision=prec, u0_full=el.to_full(U0_ref))
        sim.factor()
        done = 0
        for k in marks:
            sim.step(k - done)
            done = k
            u, v, _ = sim.get_state()
            eu = rel_l2(u.cpu().numpy(), el.to_full(keep[k][0]))
            ev = rel_l2(v.cpu().numpy(), el.to_full(keep[k][1]))
            print(f"C4 {prec} step {k}: rel L2 U^n {eu:.2e} U^(n-1) {ev:.2e}", flush=True)
            if prec == "fp64":
                assert max(eu, ev) <= TOL, (k, eu, ev)
        if prec == "mixed_fp32":
            assert max(eu, ev) <= MIXED_TOL, (eu, ev)
        sim.close()


@pytest.mark.parametrize("cfg", [
    W.C4.with_(nelem=(6, 5, 7), steps=6, tau=0.02, lam=0.8, mu=0.6, rho=1.3),
    W.C4.with_(nelem=(5, 6, 4), p=3, q=4, steps=5, tau=0.02, lam=2.0, mu=0.5, rho=0.9, bc="natural"),
], ids=lambda c: f"{c.nelem}-p{c.p}-{c.bc}")
def test_elastic_mixed_small(cfg):
    """Mixed mode on small meshes (ragged tiles, p = 3, traction-free):
    within the mixed bar of the oracle (the start is FP64)."""
    _cuda()
    el, U0_ref, (_, hist) = oracle_elastic(cfg, cfg.steps, history=True)
    sim, _ = gpu_sim(cfg, precision="mixed_fp32", u0_full=el.to_full(U0_ref))
    sim.factor()
    u, v, _ = sim.get_state()
    assert rel_l2(v.cpu().numpy(), el.to_full(hist[0][1])) <= TOL
    sim.step(cfg.steps)
    u, v, _ = sim.get_state()
    eu = rel_l2(u.cpu().numpy(), el.to_full(hist[cfg.steps][0]))
    print(f"mixed elasticity {cfg.nelem} p={cfg.p}: rel L2 U^n {eu:.2e}", flush=True)
    assert 0 < eu <= MIXED_TOL, eu
    sim.close()


def test_elastic_energy_on_gpu():
    _cuda()
    cfg = W.C4.with_(nelem=(6, 6, 6), steps=20, tau=0.5)
    from oracle import elastic
    el = elastic.Elastic(cfg.nelem, cfg.p, cfg.q, cfg.tau)
    sim, _ = gpu_sim(cfg)
    sim.factor()
    E = []
    prev = sim.get_state()[0].cpu().numpy()
    for k in range(cfg.steps):
        sim.step(1)
        cur = sim.get_state()[0].cpu().numpy()
        E.append(el.energy(el.to_free(cur), el.to_free(prev)))
        prev = cur
    E = np.array(E)
    assert np.all(np.abs(E / E[0] - 1) < 1e-10)
    sim.close()


@pytest.mark.parametrize("cfg", [
    W.C4.with_(nelem=(6, 7, 5), steps=3, tau=0.02, lam=0.8, mu=0.6, rho=1.3),
    W.C4.with_(nelem=(5, 4, 6), p=3, q=4, steps=3, tau=0.05, lam=2.0, mu=0.5, bc="natural"),
], ids=lambda c: f"{c.nelem}-p{c.p}-{c.bc}")
def test_device_energy_matches_oracle(cfg):
    """ads_energy (three-level energy with the alternating-triangular
    operator, on the device) equals the oracle's energy of the same states."""
    _cuda()
    el, U0_ref, _ = oracle_elastic(cfg, 0)
    sim, _ = gpu_sim(cfg, u0_full=el.to_full(U0_ref))
    sim.factor()
    for k in range(cfg.steps):
        sim.step(1)
        u, v, _ = sim.get_state()
        ref = el.energy(el.to_free(u.cpu().numpy()), el.to_free(v.cpu().numpy()))
        e = sim.energy()
        assert abs(e - ref) <= 1e-12 * abs(ref), (k, e, ref)
    sim.close()


@pytest.mark.parametrize("bc", ["dirichlet", "natural"])
def test_device_energy_conserved(bc):
    """The paper's elasticity run (Section 7: 32^3 elements, tau = 1e-2):
    the device energy is constant over 100 steps."""
    _cuda()
    cfg = W.C4.with_(nelem=(32, 32, 32), tau=1e-2, steps=100, bc=bc)
    sim, _ = gpu_sim(cfg)
    sim.factor()
    E = []
    for k in range(cfg.steps):
        sim.step(1)
        E.append(sim.energy())
    E = np.array(E)
    print(f"elasticity 32^3 {bc}: E = {E[0]:.12e}, max |E/E1 - 1| = {np.abs(E / E[0] - 1).max():.2e}", flush=True)
    assert E[0] > 0 and np.all(np.abs(E / E[0] - 1) < 1e-11)
    sim.close()
