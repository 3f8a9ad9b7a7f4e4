"""GPU parity of the two-dimensional P-wave (nelem[2] = 0, the setting of
Section 2) against the 2D oracle, through the C-ABI.  Bar: relative L2
<= 1e-12 (FP64), 1e-6 with FP32 contractions."""
import numpy as np
import pytest

from runners import rel_l2

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bump2d(x, y):
    return np.exp(-200.0 * ((y[:, None] - 0.5) ** 2 + (x[None, :] - 0.47) ** 2))


def _case(E, p, tau, bc="dirichlet", precision="fp64"):
    import torch
    from oracle import pwave2d
    from paper_1911_08158_amd import Sim
    pw = pwave2d.PWave2D(E, p, tau=tau, bc={"dirichlet": "dirichlet", "natural": "neumann"}[bc])
    sim = Sim(None, device="cuda", problem="pwave", nelem=(E[0], E[1], 0), p=p, tau=tau, bc=bc,
              precision=precision)
    return pw, sim, torch


@pytest.mark.parametrize("E,p,tau,bc", [((14, 11), 2, 0.02, "dirichlet"), ((9, 12), 3, 0.05, "natural"),
                                        ((1, 3), 2, 0.1, "dirichlet")])
def test_pwave2d_matches_oracle(E, p, tau, bc):
    _cuda()
    pw, sim, torch = _case(E, p, tau, bc)
    x, y = pw.quad_points(0), pw.quad_points(1)
    vals = _bump2d(x, y)
    u0 = pw.project(vals)
    # projection of data constant along the flat direction
    q = p + 1
    v3 = np.ascontiguousarray(np.broadcast_to(vals[None], (q,) + vals.shape))
    u0g = sim.project(torch.from_numpy(v3).cuda())
    assert u0g.shape == (1,) + pw.full_shape
    assert rel_l2(u0g.cpu().numpy()[0], pw.to_full(u0)) <= TOL
    # time integration from identical coefficients
    sim.set_state(torch.from_numpy(pw.to_full(u0)[None]).cuda(), None, None, 0)
    sim.factor()
    _, hist = pw.run(u0, nsteps=6, history=True)
    assert rel_l2(sim.get_state()[2].cpu().numpy()[0], pw.to_full(hist[0][2])) <= TOL
    for k in range(1, 7):
        sim.step(1)
        u, v, a = (t.cpu().numpy()[0] for t in sim.get_state())
        errs = [rel_l2(g, pw.to_full(r)) for g, r in zip((u, v, a), hist[k])]
        assert max(errs) <= TOL, (k, errs)
        e, ref = sim.energy(), pw.energy(*hist[k][:2])
        assert abs(e - ref) <= 1e-12 * abs(ref), (k, e, ref)
    sim.close()


def test_pwave2d_mixed_precision():
    _cuda()
    pw, sim, torch = _case((40, 36), 2, 0.01, precision="mixed_fp32")
    u0 = pw.project(_bump2d(pw.quad_points(0), pw.quad_points(1)))
    sim.set_state(torch.from_numpy(pw.to_full(u0)[None]).cuda(), None, None, 0)
    sim.factor()
    (u_ref, _, _) = pw.run(u0, nsteps=30)
    sim.step(30)
    e = rel_l2(sim.get_state()[0].cpu().numpy()[0], pw.to_full(u_ref))
    assert e <= 1e-6, e
    sim.close()
