"""Mixed-precision right-hand side (FP32 stiffness passes on FP64
differences or FP32 quadrature contractions; FP64 predictor, mass channel,
z-accumulation, assembly, factors, sweeps and update), in both forms
(Kronecker band passes and quadrature), against the FP64 oracle: relative
L2 error of u, u' and u'' reported per step; target <= 1e-6 for u and u'
after 100 steps on C3 (128^3 elements, p = 2).  The BF16-input mode
(predictor rounded to BF16, then a correction pass on the FP64 remainder)
is held to the same bars."""
import numpy as np
import pytest

import workloads as W
from runners import gpu_sim, oracle_pwave, oracle_pwave_at, rel_l2

pytestmark = pytest.mark.gpu


def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("cfg", [W.C1.with_(nelem=(20, 17, 23), tau=0.01, steps=20),
                                 W.C1.with_(nelem=(13, 11, 9), p=3, q=4, tau=0.01, steps=20)],
                         ids=["p2", "p3"])
@pytest.mark.parametrize("form", ["band", "quadrature"])
def test_mixed_small_meshes(cfg, form):
    _cuda()
    pw, u0, (_, hist) = oracle_pwave(cfg, cfg.steps, history=True)
    sim, _ = gpu_sim(cfg, precision="mixed_fp32", u0_full=pw.to_full(u0), rhs_var=3 if form == "band" else 0)
    sim.factor()
    for k in range(1, cfg.steps + 1):
        sim.step(1)
        u, _, _ = sim.get_state()
        ref = pw.to_full(hist[k][0])
        e = rel_l2(u.cpu().numpy(), ref)
        # pointwise as well: these meshes end in ragged tiles (20 x 17 x 23
        # against 32 x 8 and 14 x 14 columns), where a localized error would
        # hide in the global norm
        m = max_rel(u.cpu().numpy(), ref)
        assert e <= 1e-6 and m <= 1e-5, (k, e, m)
    sim.close()


@pytest.mark.parametrize("cfg", [W.C1.with_(nelem=(20, 17, 23), tau=0.01, steps=20),
                                 W.C1.with_(nelem=(13, 11, 9), p=3, q=4, tau=0.01, steps=20)],
                         ids=["p2", "p3"])
@pytest.mark.parametrize("form", ["band", "quadrature"])
def test_bf16_inputs_small_meshes(cfg, form):
    _cuda()
    pw, u0, (_, hist) = oracle_pwave(cfg, cfg.steps, history=True)
    sim, _ = gpu_sim(cfg, precision="mixed_bf16", u0_full=pw.to_full(u0), rhs_var=3 if form == "band" else 0)
    sim.factor()
    for k in range(1, cfg.steps + 1):
        sim.step(1)
        u, _, _ = sim.get_state()
        e = rel_l2(u.cpu().numpy(), pw.to_full(hist[k][0]))
        assert e <= 1e-6, (k, e)
    sim.close()


def test_bf16_inputs_not_pooled():
    _cuda()
    from paper_1911_08158_amd import Pool
    from paper_1911_08158_amd.binding import AdsError
    pool = Pool(64 << 20, max_slots=2)
    with pytest.raises(AdsError) as e:
        pool.admit(W.C1, precision="mixed_bf16")
    assert e.value.status == -1
    pool.close()


def max_rel(x, ref):
    """Largest pointwise error relative to the largest reference entry: an
    error confined to a few lines or tiles, which a global L2 norm over 2.2 M
    coefficients would dilute, shows here."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(x - ref).max() / np.abs(ref).max())


@pytest.mark.parametrize("precision", ["mixed_fp32", "mixed_bf16"])
def test_mixed_c3_error_per_step(precision):
    """C3, 100 steps: the error of u, u' and u'' against the FP64 oracle at
    steps 1, 10, 20, ..., 100 (relative L2 over all coefficients, and the
    pointwise maximum relative to the largest entry).  Bars after 100 steps:
    u and u' 1e-6 in L2 (1e-5 pointwise); u'' 1e-5 in L2 (1e-4 pointwise).
    u'' = G^{-1}(F - K w) carries the high-frequency part of the accumulated
    error of u amplified by the stiffness (its error grows about linearly
    with the step count from 8e-7 at step 1), so an FP32 stiffness action
    cannot hold it to 1e-6 over 100 steps; the measured values are printed
    per step."""
    _cuda()
    cfg = W.C3
    marks = [1] + list(range(10, cfg.steps + 1, 10))
    pw, u0, keep = oracle_pwave_at(cfg, set(marks))
    sim, _ = gpu_sim(cfg, precision=precision, u0_full=pw.to_full(u0))
    sim.factor()
    errs = []
    done = 0
    for k in marks:
        sim.step(k - done)
        done = k
        st = [t.cpu().numpy() for t in sim.get_state()]
        ref = [pw.to_full(r) for r in keep[k]]
        e = [rel_l2(x, r) for x, r in zip(st, ref)]
        m = [max_rel(x, r) for x, r in zip(st, ref)]
        errs.append((k, e, m))
        print(f"C3 {precision} step {k}: rel L2 u {e[0]:.3e} v {e[1]:.3e} a {e[2]:.3e}; "
              f"max u {m[0]:.3e} v {m[1]:.3e} a {m[2]:.3e}", flush=True)
    sim.close()
    k, e, m = errs[-1]
    assert max(e[0], e[1]) <= 1e-6 and e[2] <= 1e-5, errs
    assert max(m[0], m[1]) <= 1e-5 and m[2] <= 1e-4, errs
