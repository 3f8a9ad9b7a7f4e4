"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function declared in include/ads.h, validates parameters, sizes the
workspace, and its host Gauss rule / layout helpers agree with independent
references."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1911_08158_amd import binding
    if not os.path.exists(binding.lib_path()):
        from paper_1911_08158_amd import build
        build.build(verbose=False)
    return binding.load_library()


def test_exports_every_declared_symbol(lib):
    hdr = open(os.path.join(ROOT, "include", "ads.h")).read()
    names = set(re.findall(r"^\s*(?:ads_status|const char\*|int32_t)\s+(ads_\w+)\s*\(", hdr, re.M))
    assert len(names) >= 14 and "ads_coupling_fused" in names
    for n in sorted(names):
        assert hasattr(lib, n), n


def _params(**kw):
    from paper_1911_08158_amd.binding import Params
    d = dict(problem="pwave", nelem=(4, 5, 6), p=2, tau=0.01)
    d.update(kw)
    return Params.of(**d)


@pytest.mark.parametrize("bad", [dict(p=0), dict(p=6), dict(q=2), dict(q=6), dict(tau=0.0), dict(tau=-1.0), dict(nelem=(0, 4, 4)),
                                 dict(problem="elastic", mu=0.0), dict(problem="elastic", rho=-1.0),
                                 dict(problem="elastic", precision="mixed_bf16"),
                                 dict(nelem=(600, 4, 4)), dict(bc=2), dict(bc=-1),
                                 dict(nelem=(511, 4, 4), bc="natural"),
                                 dict(problem="elastic", nelem=(4, 0, 4)), dict(nelem=(0, 4, 4))])
def test_invalid_params_rejected(lib, bad):
    from paper_1911_08158_amd import binding
    with pytest.raises(binding.AdsError) as e:
        binding.workspace_bytes(_params(**bad))
    assert e.value.status == -1


def test_precision_modes_accepted(lib):
    from paper_1911_08158_amd import binding
    sizes = {m: binding.workspace_bytes(_params(precision=m)) for m in ("fp64", "mixed_fp32", "mixed_bf16")}
    assert len(set(sizes.values())) == 1, sizes   # same fields and tables in every mode


def test_workspace_scales_linearly(lib):
    from paper_1911_08158_amd import binding
    b1 = binding.workspace_bytes(_params(nelem=(30, 30, 30)))
    b2 = binding.workspace_bytes(_params(nelem=(60, 60, 60)))
    nf1, nf2 = 30 ** 3, 60 ** 3
    # 8 FP64 fields (u, v, a, R, X, load, the predictor w, the half-step velocity b) plus O(n) tables
    assert 6 * 8 * nf1 < b1 < 12 * 8 * nf1
    assert 6 * 8 * nf2 < b2 < 12 * 8 * nf2
    be = binding.workspace_bytes(_params(problem="elastic", nelem=(30, 30, 30)))
    assert be > 2.2 * b1   # elasticity: 20 FP64 fields (3 components of u, v, R, load, Y, Z; X, T) against 8


def test_two_dimensional_elasticity_accepted(lib):
    """nelem[2] = 0 is accepted for elasticity too (plane strain with the
    antiplane component): 20 component fields of (E + p - 2)^2 coefficients."""
    from paper_1911_08158_amd import binding
    b2 = binding.workspace_bytes(_params(problem="elastic", nelem=(30, 20, 0)))
    assert 20 * 8 * 30 * 20 < b2 < 20 * 8 * 30 * 20 + (4 << 20)   # 20 component fields


def test_two_dimensional_layout(lib):
    """nelem[2] = 0: one z-layer; the workspace holds (E + p - 2)^2 coefficients
    per field, and the z Gauss weights of the flat direction sum to one."""
    from paper_1911_08158_amd import binding
    prm = _params(nelem=(30, 20, 0))
    assert prm.n == (32, 22, 1) and prm.full_shape == (1, 22, 32)
    b2 = binding.workspace_bytes(prm)
    assert 6 * 8 * 30 * 20 < b2 < 6 * 8 * 30 * 20 + (4 << 20)
    z = binding.quad_points(prm, 2)
    assert z.shape == (3,) and np.all((z > 0) & (z < 1))


def test_natural_bc_keeps_every_coefficient(lib):
    """Natural conditions eliminate no basis function: the fields hold
    (E + p)^3 coefficients instead of (E + p - 2)^3."""
    from paper_1911_08158_amd import binding
    bd = binding.workspace_bytes(_params(nelem=(40, 40, 40)))
    bn = binding.workspace_bytes(_params(nelem=(40, 40, 40), bc="natural"))
    grow = 6 * 8 * (42 ** 3 - 40 ** 3)
    assert 0.8 * grow < bn - bd < 1.5 * grow
    assert binding.workspace_bytes(_params(nelem=(510, 4, 4), bc="natural")) > 0   # 512 coefficients


@pytest.mark.parametrize("p", [2, 3])
def test_host_gauss_points(lib, p):
    from numpy.polynomial.legendre import leggauss
    from paper_1911_08158_amd import binding
    prm = _params(p=p, nelem=(7, 3, 5))
    for d, E in enumerate((7, 3, 5)):
        x = binding.quad_points(prm, d)
        xi, _ = leggauss(p + 1)
        ref = ((np.arange(E)[:, None] + 0.5) + 0.5 * xi[None, :]) / E
        np.testing.assert_allclose(x, ref.ravel(), atol=1e-15)


def test_library_has_no_cpu_fallback_symbols(lib):
    """The product path has exactly one implementation: the HIP kernels."""
    from paper_1911_08158_amd import binding
    src = open(binding.__file__).read()
    assert "oracle" not in src.replace("no fallback", "")


def test_binding_rejects_bad_tensors():
    """The binding refuses anything but an FP64 contiguous device tensor
    (here: host tensors and wrong dtypes) with ValueError, and knows the
    sizes the library will read (full layout and Gauss-point grid)."""
    import torch
    from paper_1911_08158_amd import binding
    for t in (torch.zeros(8, dtype=torch.float64), torch.zeros(8, dtype=torch.float32), np.zeros(8)):
        with pytest.raises(ValueError):
            binding._ptr(t, 8, "x")
    assert binding._ptr(None, 8) is None
    p = _params(nelem=(4, 5, 6), p=2)
    assert p.full_numel == 6 * 7 * 8 and p.gauss_numel == 12 * 15 * 18
    e = _params(problem="elastic", nelem=(4, 5, 6), p=3)
    assert e.full_numel == 3 * 7 * 8 * 9
    f = _params(nelem=(4, 5, 0), p=2)
    assert f.full_numel == 6 * 7 and f.gauss_numel == 12 * 15 * 3


def test_gauss_rules_above_p_plus_one_accepted(lib):
    """nquad in [p+1, p+3] is accepted; the projection data grid and the
    workspace follow the rule."""
    from paper_1911_08158_amd import binding
    a = _params(q=3)
    b = _params(q=5)
    assert b.gauss_numel * 27 == a.gauss_numel * 125
    assert binding.workspace_bytes(b) > binding.workspace_bytes(a)
    xs = binding.quad_points(b, 0)
    assert xs.size == 4 * 5 and np.all(np.diff(xs) > 0)


def test_coupling_form_host_checks(lib):
    """ads_set_coupling refuses a NULL simulation; ads_coupling_fused of a
    NULL simulation is 0 (host logic only, no device call)."""
    lib.ads_set_coupling.restype = ctypes.c_int32
    lib.ads_set_coupling.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.ads_coupling_fused.restype = ctypes.c_int32
    lib.ads_coupling_fused.argtypes = [ctypes.c_void_p]
    assert lib.ads_set_coupling(None, 1) != 0
    assert lib.ads_coupling_fused(None) == 0
