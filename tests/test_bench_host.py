"""Host logic of bench.py (no GPU): the algorithmic counts its roofline
uses and its refusal of more than one GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _count_sumfact_fmas(P, q):
    """FMAs per element of the tile-shared sum factorization, counted stage
    by stage: forward z (value and derivative of a shared column at q
    points), forward y (value, y- and z-derivative rows), forward x (three
    gradient components at q^3 points), the pointwise weights, and the
    transposed backward stages."""
    fwd_z = 2 * q * P            # per coefficient column (one per element in a tile's interior)
    fwd_y = 3 * q * P * q        # per x-column and z Gauss point: 3 outputs at q y-points
    fwd_x = 3 * q * P * q * q    # per Gauss row (q^2 of them): 3 components at q x-points
    point = 3 * q ** 3
    return 2 * (fwd_z + fwd_y + fwd_x) + point


def test_rhs_flop_count():
    # 765 / 2,176 FMAs per element for p = 2 / 3 (q = p + 1)
    assert _count_sumfact_fmas(3, 3) == 765 and _count_sumfact_fmas(4, 4) == 2176
    for p in (2, 3):
        assert bench.rhs_flops_per_element(p) == 2 * _count_sumfact_fmas(p + 1, p + 1)


def test_sweep_bytes_per_dof():
    # in-plane x+y: read R, write the y-solved field; z with the Newmark
    # update: read X and the stepping fields (w, b), write (w, b, u'')
    assert bench.SWEEP_BYTES["sweep_xy"] == 8 + 8
    assert bench.SWEEP_BYTES["sweep_z"] == 8 + 2 * 8 + 3 * 8


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_rhs_bytes_and_roofline_entries():
    """Algorithmic bytes of the Kronecker-form right-hand side (the
    predictor field in, R out) and the roofline entries built from a
    kernel-table row."""
    import workloads as W
    assert bench.RHS_BYTES == 8 + 8
    cfg = W.C3
    nfree = 128 ** 3 * 4
    row = {"kernel": "sweep_z", "ms": 0.1, "gbs": round(48 * nfree / 1e-4 / 1e9, 1)}
    e = bench.roofline_entry(row, cfg, 4, True, True)
    assert e["bound"] == "hbm" and e["unit"] == "GB/s" and e["peak"] == 8000.0
    assert abs(e["frac"] - 48 * nfree / 1e-4 / 1e9 / 8000.0) < 1e-4
    row = {"kernel": "rhs", "ms": 0.1, "gbs": 100.0, "tflops": 1.0}
    assert bench.roofline_entry(row, cfg, 4, True, True)["bound"] == "hbm"
    q = bench.roofline_entry(row, cfg, 4, False, True)
    assert q["bound"] == "alu" and q["peak"] == bench.FP32_PEAK_TFLOPS
    assert bench.roofline_entry(row, cfg, 1, False, False)["peak"] == bench.FP64_PEAK_TFLOPS
    # a traffic record only counts for the sources it was measured on
    assert bench.kernel_traffic("sweep_xy", 4) is None and bench.kernel_traffic("rhs", 1) is None
