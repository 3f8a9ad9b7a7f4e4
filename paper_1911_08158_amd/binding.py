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
ADS_BC_DIRICHLET0, ADS_BC_NATURAL = 0, 1
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
            for k in ("problem", "nelem", "p", "q", "tau", "precision", "rho", "lam", "mu", "bc"):
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
        bc = d.get("bc", "dirichlet")
        bc = {"dirichlet": ADS_BC_DIRICHLET0, "natural": ADS_BC_NATURAL, "neumann": ADS_BC_NATURAL}.get(bc, bc)
        return cls(int(prob), (c_int32 * 3)(*[int(e) for e in ne]), p, int(q) if q != p + 1 else 0, int(bc),
                   int(prec), float(d["tau"]), float(d.get("rho", 1.0)), float(d.get("lam", 1.0)),
                   float(d.get("mu", 1.0)))

    @property
    def n(self):
        """Basis functions per direction (nelem[2] = 0: two-dimensional, n_z = 1)."""
        return tuple((1 if (d == 2 and int(self.nelem[2]) == 0) else int(self.nelem[d]) + int(self.p))
                     for d in range(3))

    @property
    def comps(self):
        return 3 if self.problem == ADS_ELASTIC else 1

    @property
    def full_shape(self):
        nx, ny, nz = self.n
        return ((3,) if self.comps == 3 else ()) + (nz, ny, nx)

    @property
    def full_numel(self):
        return int(np.prod(self.full_shape))

    @property
    def gauss_numel(self):
        """Gauss points of one component ([(E_z q)][(E_y q)][(E_x q)]; the
        flat z-direction of a two-dimensional problem has one element)."""
        q = int(self.nquad) or int(self.p) + 1
        return int(np.prod([max(int(self.nelem[d]), 1) * q for d in range(3)]))


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
    # torch ships its own HIP runtime under the same soname as the system's;
    # loading torch first makes the library bind to that one copy (loaded
    # the other way round, two runtimes meet in the process and the
    # library's finds no device)
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    P = POINTER(Params)
    sig = {
        "ads_workspace_bytes": [P, POINTER(c_size_t)],
        "ads_quad_points": [P, c_int32, c_void_p],
        "ads_project_scratch_bytes": [P, POINTER(c_size_t)],
        "ads_create": [P, c_void_p, c_size_t, c_void_p, c_void_p, c_void_p, POINTER(c_void_p)],
        "ads_project": [c_void_p, c_void_p, c_void_p, c_void_p, c_size_t],
        "ads_project_static": [c_void_p, c_void_p, c_void_p],
        "ads_set_load": [c_void_p, c_void_p, c_void_p, c_int32],
        "ads_set_point_load": [c_void_p, c_void_p, c_void_p, c_int32],
        "ads_factor": [c_void_p],
        "ads_set_scheme": [c_void_p, c_int32],
        "ads_set_coefficient": [c_void_p, c_void_p, c_double],
        "ads_energy": [c_void_p, c_void_p],
        "ads_step": [c_void_p, c_int32],
        "ads_get_state": [c_void_p, c_void_p, c_void_p, c_void_p],
        "ads_checkpoint_save": [c_void_p, c_void_p, c_void_p, c_void_p],
        "ads_checkpoint_load": [c_void_p, c_void_p, c_void_p, c_void_p, c_int64],
        "ads_set_state": [c_void_p, c_void_p, c_void_p, c_void_p, c_int64],
        "ads_get_step": [c_void_p, POINTER(c_int64)],
        "ads_check_finite": [c_void_p],
        "ads_tune": [c_void_p, POINTER(c_int32), c_void_p, c_int32],
        "ads_set_launch_shape": [c_void_p, c_int32, c_int32, c_void_p],
        "ads_set_coupling": [c_void_p, c_int32],
        "ads_coupling_fused": [c_void_p],
        "ads_pool_tune": [c_void_p, POINTER(c_int32), c_void_p, c_int32],
        "ads_profile": [c_void_p, c_int32],
        "ads_profile_read": [c_void_p, c_void_p, c_void_p, c_int32, POINTER(c_int32), c_void_p, c_int32,
                             POINTER(c_int32)],
        "ads_destroy": [c_void_p],
        "ads_pool_create": [c_void_p, c_size_t, c_int32, c_void_p, c_int32, POINTER(c_void_p)],
        "ads_pool_admit": [c_void_p, P, c_void_p, c_void_p, POINTER(c_int32)],
        "ads_pool_sim": [c_void_p, c_int32, POINTER(c_void_p)],
        "ads_pool_activate": [c_void_p, c_int32],
        "ads_pool_step": [c_void_p, c_int32],
        "ads_pool_set_branches": [c_void_p, c_int32],
        "ads_pool_retire": [c_void_p, c_int32, c_void_p, c_void_p, c_void_p],
        "ads_pool_step_times": [c_void_p, c_void_p, c_int32, POINTER(c_int32)],
        "ads_pool_info": [c_void_p, POINTER(c_int32), POINTER(c_size_t), POINTER(c_size_t)],
        "ads_pool_destroy": [c_void_p],
        "ads_pool_profile": [c_void_p, c_int32],
        "ads_pool_profile_read": [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int32, POINTER(c_int32)],
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
    ne = int(prm.nelem[d])
    if d == 2 and ne == 0:   # two-dimensional: the flat direction has one element
        ne = 1
    q = int(prm.nquad) or int(prm.p) + 1   # the library writes ne * q points
    out = np.zeros(ne * q)
    _check(load_library().ads_quad_points(byref(prm), d, out.ctypes.data))
    return out


def _ptr(t, numel=None, what="tensor"):
    """Device address of an FP64 contiguous device tensor holding exactly
    ``numel`` entries (a wrongly sized array would make the kernels read or
    write past its end).  None passes through."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{what}: an FP64 contiguous device tensor is required")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: {t.numel()} entries, {numel} expected")
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
        nf = self.prm.full_numel
        _check(L.ads_create(byref(self.prm), self._ws_ptr, nb, self.stream.cuda_stream, _ptr(u0, nf, "u0"),
                            _ptr(v0, nf, "v0"), byref(h)))
        self._h = h

    # -- helpers ----------------------------------------------------------
    def _empty_full(self):
        # the library writes every entry (boundary ones as 0): no fill kernel
        import torch
        return torch.empty(self.prm.full_shape, dtype=torch.float64, device=self.device)

    def _pre(self):
        """Order the library's stream after torch's current stream (inputs)."""
        import torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _post(self):
        """Order torch's current stream after the library's stream (outputs)."""
        import torch
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.wait_stream(self.stream)

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
        self._pre()
        _check(L.ads_project(self._h, _ptr(vals, self.prm.gauss_numel * self.prm.comps, "vals"),
                             _ptr(out, self.prm.full_numel, "out"), scratch.data_ptr(), n.value))
        self._post()
        return out

    def project_static(self, vals):
        """The projection through ads_project_static (the library's static
        staging memory; nothing allocated by the library)."""
        import torch
        out = self._empty_full()
        vals = vals.to(self.device, torch.float64).contiguous()
        self._pre()
        _check(load_library().ads_project_static(self._h, _ptr(vals, self.prm.gauss_numel * self.prm.comps, "vals"),
                                                 _ptr(out, self.prm.full_numel, "out")))
        self._post()
        return out

    def set_load(self, b, amps):
        amps = np.ascontiguousarray(amps, dtype=np.float64)
        self._pre()
        _check(load_library().ads_set_load(self._h, _ptr(b, self.prm.full_numel, "load"), amps.ctypes.data,
                                           int(amps.size)))

    def set_point_load(self, xs, amps):
        xs = np.ascontiguousarray(xs, dtype=np.float64)
        amps = np.ascontiguousarray(amps, dtype=np.float64)
        _check(load_library().ads_set_point_load(self._h, xs.ctypes.data, amps.ctypes.data, int(amps.size)))

    def set_coefficient(self, c2, c2ref):
        """Wave-speed field c^2 at the Gauss points (device tensor laid out like
        project()'s input, or None) and the c^2 of the split left-hand side.
        The tensor is kept referenced for the simulation's lifetime.  Before
        factor()."""
        import torch
        if c2 is not None:
            c2 = c2.to(self.device, torch.float64).contiguous()
        self._coef = c2
        self._pre()
        _check(load_library().ads_set_coefficient(self._h, _ptr(c2, self.prm.gauss_numel, "c2"), float(c2ref)))

    SCHEMES = {"newmark": 0, "literal": 1}

    def set_scheme(self, scheme):
        """'newmark' (default) or 'literal' (the printed coefficient set; a
        P-wave diagnostic).  Before factor()."""
        _check(load_library().ads_set_scheme(self._h, int(self.SCHEMES.get(scheme, scheme))))

    def factor(self):
        _check(load_library().ads_factor(self._h))

    def energy(self):
        """Discrete energy of the current state (host float; P-wave or
        elasticity, see ads_energy)."""
        e = c_double()
        _check(load_library().ads_energy(self._h, byref(e)))
        return e.value

    def step(self, n=1):
        _check(load_library().ads_step(self._h, int(n)))

    def get_state(self):
        u, v = self._empty_full(), self._empty_full()
        a = self._empty_full() if self.prm.comps == 1 else None
        self._pre()
        nf = self.prm.full_numel
        _check(load_library().ads_get_state(self._h, _ptr(u, nf, "u"), _ptr(v, nf, "v"), _ptr(a, nf, "a")))
        self.stream.synchronize()
        return u, v, a

    def set_state(self, u, v=None, a=None, step=0):
        self._pre()
        nf = self.prm.full_numel
        _check(load_library().ads_set_state(self._h, _ptr(u, nf, "u"), _ptr(v, nf, "v"), _ptr(a, nf, "a"),
                                            int(step)))

    def checkpoint(self):
        """The time-stepping state (full layout) and the step index, from
        which checkpoint_restore continues bitwise: P-wave (w, b, u''),
        w = u + tau u' + tau^2/4 u'' and b = u' + tau/2 u'' (printed
        coefficient set: (w, u', u''), w = u + tau u'); elasticity
        (U^n, U^{n-1}, None)."""
        s0, s1 = self._empty_full(), self._empty_full()
        s2 = self._empty_full() if self.prm.comps == 1 else None
        self._pre()
        nf = self.prm.full_numel
        _check(load_library().ads_checkpoint_save(self._h, _ptr(s0, nf, "s0"), _ptr(s1, nf, "s1"),
                                                  _ptr(s2, nf, "s2")))
        self.stream.synchronize()
        return (s0, s1, s2), self.step_index()

    def checkpoint_restore(self, state, step):
        self._pre()
        nf = self.prm.full_numel
        s0, s1, s2 = state
        _check(load_library().ads_checkpoint_load(self._h, _ptr(s0, nf, "s0"), _ptr(s1, nf, "s1"),
                                                  _ptr(s2, nf, "s2"), int(step)))

    def step_index(self):
        s = c_int64()
        _check(load_library().ads_get_step(self._h, byref(s)))
        return s.value

    def check_finite(self):
        _check(load_library().ads_check_finite(self._h))

    def set_launch_shape(self, rhs_var=-1, rhs_tz=-1, sweep_w=None):
        """Launch shapes set explicitly (-1 keeps, 0 = default; sweep_w: one
        tile width per direction x, y, z)."""
        w = None
        if sweep_w is not None:
            w = (c_int32 * 3)(*[int(x) for x in sweep_w])
        _check(load_library().ads_set_launch_shape(self._h, int(rhs_var), int(rhs_tz), w))

    def set_coupling(self, fused=True):
        """Elasticity couplings in the in-plane sweeps (True, where the
        plane fits) or by separate launches (False, the default)."""
        _check(load_library().ads_set_coupling(self._h, 1 if fused else 0))

    @property
    def coupling_fused(self):
        """True when the step applies the couplings in the in-plane sweeps."""
        return bool(load_library().ads_coupling_fused(self._h))

    def tune(self):
        """Autotune the right-hand-side tiling on this mesh; returns the
        chosen variant and the measured ms per variant (NaN if cached)."""
        ch = c_int32()
        ms = np.full(8, np.nan)
        _check(load_library().ads_tune(self._h, byref(ch), ms.ctypes.data, 8))
        return ch.value, ms

    def profile(self, enable=True):
        _check(load_library().ads_profile(self._h, 1 if enable else 0))

    KIND_NAMES = {0: "rhs", 1: "sweep_x", 2: "sweep_y", 3: "sweep_z", 4: "couple", 6: "sweep_xy"}

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


class PooledSim(Sim):
    """A simulation living in a Pool slot (the pool owns its memory)."""

    def __init__(self, pool, slot, prm):
        self.prm = prm
        self.device = pool.device
        self.stream = pool.stream
        self.slot = slot
        h = c_void_p()
        _check(load_library().ads_pool_sim(pool._h, slot, byref(h)))
        self._h = h

    def close(self):          # released by Pool.retire
        self._h = c_void_p()


class Pool:
    """Batched serving pool: admission by memory, one graph replay per step
    for all active simulations (include/ads.h, ads_pool_*)."""

    def __init__(self, nbytes, max_slots=64, device=None, stream=None, use_graph=True):
        import torch
        self.device = torch.device(device if device is not None else "cuda")
        # graph capture needs a non-default stream; default priority
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self._ws = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=self.device)
        ptr = (self._ws.data_ptr() + 255) // 256 * 256
        h = c_void_p()
        _check(load_library().ads_pool_create(ptr, int(nbytes), int(max_slots), self.stream.cuda_stream,
                                              1 if use_graph else 0, byref(h)))
        self._h = h
        self.sims = {}

    def admit(self, cfg=None, u0=None, v0=None, **kw):
        """Returns a PooledSim, or None when memory or slots are exhausted.
        u0 / v0: initial coefficients (full layout, FP64 device tensors) or
        None (zero)."""
        prm = Params.of(cfg, **kw)
        slot = c_int32()
        nf = prm.full_numel
        st = load_library().ads_pool_admit(self._h, byref(prm), _ptr(u0, nf, "u0"), _ptr(v0, nf, "v0"), byref(slot))
        if st == -2:
            return None
        _check(st)
        s = PooledSim(self, slot.value, prm)
        self.sims[slot.value] = s
        return s

    def activate(self, sim):
        _check(load_library().ads_pool_activate(self._h, sim.slot))

    def step(self, n=1):
        _check(load_library().ads_pool_step(self._h, int(n)))

    def set_branches(self, n):
        """Concurrent branches of the following steps (1 or 2)."""
        _check(load_library().ads_pool_set_branches(self._h, int(n)))

    def tune(self):
        """Autotune the launch shapes of the current batch; returns the
        number of launch classes whose shape changed and the shape of every
        launch position (variant, tile width, 0, or -1 when not launched)."""
        n = c_int32()
        shape = np.full(256, -1, dtype=np.int32)
        _check(load_library().ads_pool_tune(self._h, byref(n), shape.ctypes.data, shape.size))
        return n.value, shape

    def retire(self, sim, state=False):
        """Release the slot; with state=True first copy out and return its
        final (u, v, a) as ads_get_state gives it (a None for elasticity)."""
        out = None
        if state:
            u, v = sim._empty_full(), sim._empty_full()
            a = sim._empty_full() if sim.prm.comps == 1 else None
            nf = sim.prm.full_numel
            _check(load_library().ads_pool_retire(self._h, sim.slot, _ptr(u, nf, "u"), _ptr(v, nf, "v"),
                                                  _ptr(a, nf, "a")))
            self.stream.synchronize()
            out = (u, v, a)
        else:
            _check(load_library().ads_pool_retire(self._h, sim.slot, None, None, None))
        self.sims.pop(sim.slot, None)
        sim.close()
        return out

    def step_times(self, cap=1 << 16):
        ms = np.zeros(cap)
        n = c_int32()
        _check(load_library().ads_pool_step_times(self._h, ms.ctypes.data, cap, byref(n)))
        return ms[:n.value].copy()

    POOL_KINDS = {0: "rhs", 5: "rhs_elastic", 1: "sweep_x", 2: "sweep_y", 3: "sweep_z", 4: "couple", 6: "sweep_xy"}

    def profile(self, enable=True):
        _check(load_library().ads_pool_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """[(kind, p, mixed, mean ms)] per launch position of a pool step."""
        cap = 64
        ms = np.zeros(cap)
        kind, pp, mx = (np.zeros(cap, dtype=np.int32) for _ in range(3))
        n = c_int32()
        _check(load_library().ads_pool_profile_read(self._h, ms.ctypes.data, kind.ctypes.data, pp.ctypes.data,
                                                    mx.ctypes.data, cap, byref(n)))
        return [(self.POOL_KINDS.get(int(kind[i]), str(kind[i])), int(pp[i]), int(mx[i]), float(ms[i]))
                for i in range(n.value)]

    def info(self):
        a, u, f = c_int32(), c_size_t(), c_size_t()
        _check(load_library().ads_pool_info(self._h, byref(a), byref(u), byref(f)))
        return {"active": a.value, "used_bytes": u.value, "free_bytes": f.value}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().ads_pool_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
