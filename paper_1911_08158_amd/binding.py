"""ctypes binding of include/ads.h (argument marshalling only).

Every numerical step runs in the HIP library; nothing here computes on the
CPU, and there is no fallback: if ``lib/libads.so`` is missing the first
call raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

ADS_PWAVE, ADS_ELASTIC = 0, 1
ADS_FP64, ADS_MIXED_FP32, ADS_MIXED_BF16 = 0, 1, 2
STATUS = {0: "ADS_OK", -1: "ADS_EINVAL", -2: "ADS_ENOMEM", -3: "ADS_EDEVICE", -4: "ADS_ESTATE",
          -5: "ADS_ENUMERIC"}
PRECISION = {"fp64": ADS_FP64, "mixed_fp32": ADS_MIXED_FP32, "mixed_bf16": ADS_MIXED_BF16}


class AdsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("problem", c_int32), ("nelem", c_int32 * 3), ("p", c_int32), ("nquad", c_int32),
                ("bc", c_int32), ("precision", c_int32), ("tau", c_double), ("rho", c_double),
                ("lam", c_double), ("mu", c_double)]

    @classmethod
    def of(cls, cfg=None, **kw) -> "Params":
        """From any object with attributes problem ('pwave'/'elastic'), nelem,
        p, tau and optionally q, precision, rho, lam, mu (or keywords)."""
        d = {}
        if cfg is not None:
            for k in ("problem", "nelem", "p", "q", "tau", "precision", "rho", "lam", "mu"):
                if hasattr(cfg, k):
                    d[k] = getattr(cfg, k)
        d.update(kw)
        prob = d.get("problem", "pwave")
        prob = {"pwave": ADS_PWAVE, "elastic": ADS_ELASTIC}.get(prob, prob)
        prec = d.get("precision", "fp64")
        prec = PRECISION.get(prec, prec)
        ne = d["nelem"]
        if np.isscalar(ne):
            ne = (ne,) * 3
        q = d.get("q", 0) or 0
        p = int(d["p"])
        return cls(int(prob), (c_int32 * 3)(*[int(e) for e in ne]), p, int(q) if q != p + 1 else 0, 0,
                   int(prec), float(d["tau"]), float(d.get("rho", 1.0)), float(d.get("lam", 1.0)),
                   float(d.get("mu", 1.0)))

    @property
    def n(self):
        return tuple(int(self.nelem[d]) + int(self.p) for d in range(3))

    @property
    def comps(self):
        return 3 if self.problem == ADS_ELASTIC else 1

    @property
    def full_shape(self):
        nx, ny, nz = self.n
        return ((3,) if self.comps == 3 else ()) + (nz, ny, nx)


def lib_path() -> str:
    return os.path.join(_HERE, "lib", "libads.so")


def load_library():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run `python -m paper_1911_08158_amd.build`)")
    L = ctypes.CDLL(path)
    P = POINTER(Params)
    sig = {
        "ads_workspace_bytes": [P, POINTER(c_size_t)],
        "ads_quad_points": [P, c_int32, c_void_p],
        "ads_project_scratch_bytes": [P, POINTER(c_size_t)],
        "ads_create": [P, c_void_p, c_size_t, c_void_p, c_void_p, c_void_p, POINTER(c_void_p)],
        "ads_project": [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t],
        "ads_set_load": [c_void_p, c_void_p, c_void_p, c_int32],
        "ads_set_point_load": [c_void_p, c_void_p, c_void_p, c_int32],
        "ads_factor": [c_void_p],
        "ads_step": [c_void_p, c_int32],
        "ads_get_state": [c_void_p, c_void_p, c_void_p, c_void_p],
        "ads_set_state": [c_void_p, c_void_p, c_void_p, c_void_p, c_int64],
        "ads_get_step": [c_void_p, POINTER(c_int64)],
        "ads_check_finite": [c_void_p],
        "ads_profile": [c_void_p, c_int32],
        "ads_profile_read": [c_void_p, c_void_p, c_void_p, c_int32, POINTER(c_int32), c_void_p, c_int32,
                             POINTER(c_int32)],
        "ads_destroy": [c_void_p],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = c_int32
    L.ads_last_error.argtypes = []
    L.ads_last_error.restype = ctypes.c_char_p
    _LIB = L
    return L


def _check(st):
    if st != 0:
        raise AdsError(st, load_library().ads_last_error().decode())


def workspace_bytes(prm: Params) -> int:
    n = c_size_t()
    _check(load_library().ads_workspace_bytes(byref(prm), byref(n)))
    return n.value


def quad_points(prm: Params, d: int) -> np.ndarray:
    out = np.zeros(int(prm.nelem[d]) * (prm.p + 1))
    _check(load_library().ads_quad_points(byref(prm), d, out.ctypes.data))
    return out


def _ptr(t):
    if t is None:
        return None
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "FP64 contiguous device tensor"
    return t.data_ptr()


class Sim:
    """One simulation on one GPU: workspace, factors and state in HBM."""

    def __init__(self, cfg=None, device=None, stream=None, u0=None, v0=None, **kw):
        import torch
        self.prm = Params.of(cfg, **kw)
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L = load_library()
        nb = workspace_bytes(self.prm)
        self.ws_bytes = nb
        self._ws = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        h = c_void_p()
        _check(L.ads_create(byref(self.prm), self._ws_ptr, nb, self.stream.cuda_stream, _ptr(u0), _ptr(v0),
                            byref(h)))
        self._h = h

    # -- helpers ----------------------------------------------------------
    def _empty_full(self):
        import torch
        return torch.zeros(self.prm.full_shape, dtype=torch.float64, device=self.device)

    def quad_points(self, d):
        return quad_points(self.prm, d)

    # -- API --------------------------------------------------------------
    def project(self, vals):
        """L2 projection of data sampled at the Gauss points; returns the
        full-layout coefficient tensor."""
        import torch
        L = load_library()
        n = c_size_t()
        _check(L.ads_project_scratch_bytes(byref(self.prm), byref(n)))
        scratch = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        out = self._empty_full()
        vals = vals.to(self.device, torch.float64).contiguous()
        _check(L.ads_project(self._h, _ptr(vals), _ptr(out), scratch.data_ptr(), n.value))
        return out

    def set_load(self, b, amps):
        amps = np.ascontiguousarray(amps, dtype=np.float64)
        _check(load_library().ads_set_load(self._h, _ptr(b), amps.ctypes.data, int(amps.size)))

    def set_point_load(self, xs, amps):
        xs = np.ascontiguousarray(xs, dtype=np.float64)
        amps = np.ascontiguousarray(amps, dtype=np.float64)
        _check(load_library().ads_set_point_load(self._h, xs.ctypes.data, amps.ctypes.data, int(amps.size)))

    def factor(self):
        _check(load_library().ads_factor(self._h))

    def step(self, n=1):
        _check(load_library().ads_step(self._h, int(n)))

    def get_state(self):
        u, v = self._empty_full(), self._empty_full()
        a = self._empty_full() if self.prm.comps == 1 else None
        _check(load_library().ads_get_state(self._h, _ptr(u), _ptr(v), _ptr(a)))
        self.stream.synchronize()
        return u, v, a

    def set_state(self, u, v=None, a=None, step=0):
        _check(load_library().ads_set_state(self._h, _ptr(u), _ptr(v), _ptr(a), int(step)))

    def step_index(self):
        s = c_int64()
        _check(load_library().ads_get_step(self._h, byref(s)))
        return s.value

    def check_finite(self):
        _check(load_library().ads_check_finite(self._h))

    def profile(self, enable=True):
        _check(load_library().ads_profile(self._h, 1 if enable else 0))

    KIND_NAMES = {0: "rhs", 1: "sweep_x", 2: "sweep_y", 3: "sweep_z", 4: "couple"}

    def profile_read(self, max_steps=100000):
        """Mean kernel durations (ms) per launch position of one step, their
        kinds, and the per-step durations (ms) since ads_profile(1)."""
        cap = 64
        ms = np.zeros(cap)
        kind = np.zeros(cap, dtype=np.int32)
        steps = np.zeros(max_steps)
        nl, ns = c_int32(), c_int32()
        _check(load_library().ads_profile_read(self._h, ms.ctypes.data, kind.ctypes.data, cap, byref(nl),
                                               steps.ctypes.data, max_steps, byref(ns)))
        n = nl.value
        return ms[:n].copy(), [self.KIND_NAMES.get(int(k), str(k)) for k in kind[:n]], steps[:min(ns.value,
                                                                                                max_steps)].copy()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().ads_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
