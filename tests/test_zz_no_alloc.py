"""ads_project_static (the projection on the library's static staging
memory, for callers that cannot allocate) against ads_project on the same
simulation: identical kernels on identical inputs, so the outputs agree
bitwise.  Two calls in a row on one GPU, the second on a smaller mesh (the
static array keeps the first call's contents), plus the size limit."""
import dataclasses

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _case(nelem, p, problem="pwave", seed=7):
    base = W.C4 if problem == "elastic" else W.C1
    return dataclasses.replace(base, name="noalloc", nelem=nelem, p=p, q=p + 1, init="noise", seed=seed,
                               bc="dirichlet")


def _both(cfg):
    import torch
    from paper_1911_08158_amd import Sim
    sim = Sim(cfg, device="cuda")
    xs = [sim.quad_points(d) for d in range(3)]
    vals = torch.from_numpy(np.ascontiguousarray(W.initial_values(cfg, *xs))).to("cuda")
    print(f"no-alloc case {cfg.problem} nelem={cfg.nelem} p={cfg.p}", flush=True)
    ref = sim.project(vals)
    got = sim.project_static(vals)
    torch.cuda.synchronize()
    sim.close()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_static_projection_matches_two_calls_then_smaller():
    for cfg in (_case((40, 36, 32), 3), _case((12, 9, 7), 2)):
        ref, got = _both(cfg)
        assert np.isfinite(ref).all() and np.abs(ref).max() > 0
        assert np.array_equal(ref, got), (cfg.nelem, float(np.abs(ref - got).max()))


def test_static_projection_elastic_then_pwave():
    for cfg in (_case((20, 18, 16), 2, problem="elastic"), _case((6, 5, 4), 3)):
        ref, got = _both(cfg)
        assert np.array_equal(ref, got), (cfg.nelem, float(np.abs(ref - got).max()))


def test_static_projection_rejects_meshes_beyond_the_buffer():
    import torch
    from paper_1911_08158_amd import Sim
    from paper_1911_08158_amd.binding import AdsError
    cfg = _case((96, 96, 96), 2)
    sim = Sim(cfg, device="cuda")
    vals = torch.zeros(sim.prm.gauss_numel, dtype=torch.float64, device="cuda")
    with pytest.raises(AdsError) as ei:
        sim.project_static(vals)
    assert ei.value.status == -2 and "static buffer" in str(ei.value)
    sim.close()
