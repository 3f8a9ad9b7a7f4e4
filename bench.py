#!/usr/bin/env python3
"""Benchmark of the per-step hot path on one MI355X.

A "step" is one pass of the whole hot path over the batch: right-hand side
by sum-factorized Gauss quadrature, x-, y- and z-sweeps of the banded LU
factors, Newmark update (fused into the z-sweep).  Default workload: the
3D P-wave with 128^3 elements, p = 2 (130^3 DOFs), tau = 2e-3.

Prints ONE JSON line (rank 0):
  value            whole-job DOF-steps/s (n^3 DOFs per simulation, boundary
                   DOFs included) over the timed steps, inputs resident in HBM
  roofline         dominant kernel (the right-hand side) against the FP64
                   vector peak, with algorithmic flops per launch
  kernels          every kernel of the step with its mean duration and
                   algorithmic rate (HIP events on the sim's stream)
  cpu_baseline     the CPU oracle timed on this host on a bounded sample
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DOF-steps/s, 3D P-wave p=2: batched mixed vs plain FP64; p99 step latency"
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector: 256 CU x 64 FMA/clk x 2 x 2.4 GHz
HBM_PEAK_GBS = 8000.0


def rhs_flops_per_element(p, q=None):
    """Sum-factorized quadrature of the stiffness action, tile-shared:
    2 P (2q + 3q^2 + 3q^3) + 3 q^3 FMAs per element (forward, pointwise,
    backward), 2 flops per FMA."""
    P = p + 1
    q = P if q is None else q
    return 2 * (2 * P * (2 * q + 3 * q * q + 3 * q ** 3) + 3 * q ** 3)


SWEEP_BYTES = {"sweep_x": 16, "sweep_y": 16, "sweep_z": 56}   # per free DOF (z fused with Newmark update)


def gpu_info():
    import torch
    p = torch.cuda.get_device_properties(0)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", ""), "cus": p.multi_processor_count}


def make_sim(cfg, precision):
    import torch

    import workloads as W
    from paper_1911_08158_amd import Sim
    sim = Sim(cfg, device="cuda:0", precision=precision)
    xs = [sim.quad_points(d) for d in range(3)]
    u0 = sim.project(torch.from_numpy(np.ascontiguousarray(W.initial_values(cfg, *xs))).to("cuda:0"))
    sim.set_state(u0, None, None, 0)
    if cfg.load == "ricker_point":
        sim.set_point_load(W.source_point(cfg.seed), W.load_amplitudes(cfg))
    sim.factor()
    return sim


def measure_single(cfg, precision, steps, warmup):
    """Plain per-simulation form: one simulation, per-kernel launches."""
    import torch
    sim = make_sim(cfg, precision)
    sim.step(warmup)
    torch.cuda.synchronize()
    sim.profile(True)
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, kinds, step_ms = sim.profile_read(steps)
    sim.check_finite()
    sim.close()
    wall = t1 - t0
    nx, ny, nz = cfg.n
    dofs = nx * ny * nz * cfg.comps
    nfree = (nx - 2) * (ny - 2) * (nz - 2)
    nel = int(np.prod(cfg.nelem))
    kern = []
    for m, k in zip(ms, kinds):
        e = {"kernel": k, "ms": round(float(m), 5)}
        if k == "rhs":
            fl = rhs_flops_per_element(cfg.p) * nel
            e.update(algorithmic_flops=fl, tflops=round(fl / (m * 1e-3) / 1e12, 3))
        elif k in SWEEP_BYTES:
            by = SWEEP_BYTES[k] * nfree
            e.update(algorithmic_bytes=by, gbs=round(by / (m * 1e-3) / 1e9, 1))
        kern.append(e)
    return {
        "dof_steps_per_s": dofs * steps / wall,
        "ms_per_step": wall / steps * 1e3,
        "kernels": kern,
        "step_ms_p50": float(np.percentile(step_ms, 50)) if len(step_ms) else None,
        "step_ms_p99": float(np.percentile(step_ms, 99)) if len(step_ms) else None,
    }


def cpu_baseline(cfg, seconds):
    """The CPU oracle, as it stands, on a bounded sample of the same workload:
    setup and the start are untimed; steps are timed until ``seconds``
    elapse (at least 2)."""
    import workloads as W
    from oracle import pwave
    try:
        from threadpoolctl import threadpool_info
        threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    pw = pwave.PWave(cfg.nelem, cfg.p, cfg.q, cfg.tau)
    u = pw.project(W.initial_values(cfg, *[pw.quad_points(d) for d in range(3)]))
    v = np.zeros_like(u)
    a = pw.initial_accel(u)
    n = 0
    t0 = time.perf_counter()
    while True:
        u, v, a = pw.step(u, v, a)
        n += 1
        dt = time.perf_counter() - t0
        if n >= 2 and dt >= seconds:
            break
    nx, ny, nz = cfg.n
    return {"value": nx * ny * nz * n / dt, "unit": "DOF-steps/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{n} steps of {cfg.nelem[0]}x{cfg.nelem[1]}x{cfg.nelem[2]} p={cfg.p} P-wave "
                      f"(NumPy FP64 oracle; setup, projection and start untimed)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (the hot path is measured on one "
              "MI355X; multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import workloads as W
    cfg = W.C3
    fp64 = measure_single(cfg.with_(precision="fp64"), "fp64", args.steps, args.warmup)
    rhs = next(k for k in fp64["kernels"] if k["kernel"] == "rhs")
    roof = {"bound": "alu", "achieved": rhs["tflops"], "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(rhs["tflops"] / FP64_PEAK_TFLOPS, 4), "traffic": None,
            "kernel": "rhs_pwave_kernel<3,3>",
            "per_launch": f"{rhs_flops_per_element(cfg.p)} flops/element x {int(np.prod(cfg.nelem))} elements"}
    out = {
        "metric": METRIC,
        "value": fp64["dof_steps_per_s"],
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fp64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "C3 P-wave 128^3 elements p=2 (130^3 DOFs) tau=2e-3, one simulation, "
                               "FP64 right-hand side (plain per-simulation form)",
                   "form": "plain_fp64", "batch": 1},
        "p50_step_ms": fp64["step_ms_p50"],
        "p99_step_ms": fp64["step_ms_p99"],
        "kernels": fp64["kernels"],
        "roofline": roof,
        "gpu": gpu_info(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
