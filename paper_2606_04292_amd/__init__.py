"""MI355X (gfx950) NGS-FAS solver for the BDF-discretised Richards equation.

Thin Python binding of the C ABI in ``include/richards.h``: argument
marshalling only.  Every step of the solver runs in the HIP kernels of
``_lib/librichards.so``; PyTorch supplies device memory (workspaces, state
arrays) and streams.  If the library is not built this module raises on use,
it never falls back to another implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import workloads

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "librichards.so")

RS_OK, RS_EINVAL, RS_ENOMEM, RS_EHIP, RS_ESTATE, RS_ENONFINITE, RS_ENOTCONV, RS_EBUSY = range(8)
RS_STATIC_WORKSPACE_BYTES = 32 << 20
RS_FP64, RS_MIXED = 0, 1
RS_COARSE_INJECT, RS_COARSE_FW = 0, 1
FIELD_PSI, FIELD_KSTAR, FIELD_G, FIELD_PSIBAR = 0, 1, 2, 3

EXPORTS = [
    "rs_workspace_bytes", "rs_create_grid", "rs_set_constitutive", "rs_set_state",
    "rs_get_state", "rs_begin_step", "rs_sweep", "rs_vcycle", "rs_residual_norm",
    "rs_residual", "rs_end_step", "rs_bdf_step", "rs_copy_field", "rs_set_field",
    "rs_num_levels", "rs_level_shape", "rs_destroy_grid", "rs_last_error",
    "rs_profile_enable", "rs_profile_read", "rs_correction_cycle", "rs_fmg",
    "rs_bdf_step_static",
    # include/richards_serve.h
    "rs_engine_default_opts", "rs_engine_control_bytes", "rs_engine_request_bytes",
    "rs_engine_create", "rs_engine_submit", "rs_engine_tick", "rs_engine_fetch",
    "rs_engine_capacity", "rs_engine_destroy",
]


class RsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("richards error %d: %s" % (code, msg))
        self.code = code


class GridDesc(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("dim", C.c_int), ("n", C.c_int * 3),
                ("L", C.c_double * 3), ("face_bc", C.c_int * 6), ("face_value", C.c_double * 6),
                ("patch_face", C.c_int), ("patch_lo", C.c_int * 2), ("patch_hi", C.c_int * 2),
                ("patch_value", C.c_double)]


class Soil(C.Structure):
    _fields_ = [("model", C.c_int), ("theta_s", C.c_double), ("theta_r", C.c_double),
                ("Ks", C.c_double), ("vg_alpha", C.c_double), ("vg_n", C.c_double),
                ("hk_alpha", C.c_double), ("hk_beta", C.c_double), ("hk_A", C.c_double),
                ("hk_gamma", C.c_double), ("psi_unit", C.c_double), ("lin_c", C.c_double),
                ("gd_alpha", C.c_double)]


class Constitutive(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("model", C.c_int), ("theta_s", C.c_double),
                ("theta_r", C.c_double), ("Ks", C.c_double), ("vg_alpha", C.c_double),
                ("vg_n", C.c_double), ("hk_alpha", C.c_double), ("hk_beta", C.c_double),
                ("hk_A", C.c_double), ("hk_gamma", C.c_double), ("psi_unit", C.c_double),
                ("lin_c", C.c_double), ("sink", C.c_int), ("Tp", C.c_double),
                ("root_len", C.c_double), ("h1", C.c_double), ("h2", C.c_double),
                ("h3", C.c_double), ("h4", C.c_double), ("xi", C.c_double),
                ("kappa_rule", C.c_int), ("kappa", C.c_double), ("newton_iters", C.c_int),
                ("lag_extrap", C.c_int), ("newton_tol", C.c_double),
                ("Ks_field", C.POINTER(C.c_double)), ("gd_alpha", C.c_double),
                ("n_soils", C.c_int), ("soils", C.POINTER(Soil)), ("soil_id", C.c_void_p),
                ("coarse_kstar", C.c_int)]


class SolveOpts(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("nu1", C.c_int), ("nu2", C.c_int),
                ("nu_coarse", C.c_int), ("max_cycles", C.c_int), ("tol_abs", C.c_double),
                ("stagnation", C.c_int), ("mp_inner_cycles", C.c_int), ("fmg", C.c_int)]


class StepStats(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("cycles", C.c_int), ("status", C.c_int),
                ("res0", C.c_double), ("res", C.c_double), ("n_hist", C.c_int),
                ("res_hist", C.c_double * 64), ("cell_updates", C.c_double)]


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("HIP library not built: %s (run __graft_entry__.build())" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp, D, I = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.rs_last_error.restype = C.c_char_p
        L.rs_workspace_bytes.argtypes = [C.POINTER(GridDesc), C.c_int, C.POINTER(C.c_size_t)]
        L.rs_create_grid.argtypes = [C.POINTER(GridDesc), C.c_int, vp, C.c_size_t, vp,
                                     C.POINTER(vp)]
        L.rs_set_constitutive.argtypes = [vp, C.POINTER(Constitutive)]
        L.rs_set_state.argtypes = [vp, vp, vp, C.c_int, C.c_double]
        L.rs_get_state.argtypes = [vp, vp, vp, I, D]
        L.rs_begin_step.argtypes = [vp, C.c_double, C.c_int]
        L.rs_sweep.argtypes = [vp, C.c_int, C.c_int]
        L.rs_vcycle.argtypes = [vp, C.c_int, C.c_int, D]
        L.rs_residual_norm.argtypes = [vp, D]
        L.rs_residual.argtypes = [vp, vp]
        L.rs_end_step.argtypes = [vp]
        L.rs_bdf_step.argtypes = [vp, C.c_double, C.c_int, C.POINTER(SolveOpts),
                                  C.POINTER(StepStats)]
        L.rs_copy_field.argtypes = [vp, C.c_int, C.c_int, vp]
        L.rs_set_field.argtypes = [vp, C.c_int, C.c_int, vp]
        L.rs_num_levels.argtypes = [vp]
        L.rs_level_shape.argtypes = [vp, C.c_int, I]
        L.rs_destroy_grid.argtypes = [vp]
        L.rs_profile_enable.argtypes = [vp, C.c_int]
        L.rs_profile_read.argtypes = [vp, D, C.POINTER(C.c_longlong), D, C.c_int]
        L.rs_correction_cycle.argtypes = [vp, C.c_int, C.c_int, C.c_int, D]
        L.rs_bdf_step_static.argtypes = [C.POINTER(GridDesc), C.POINTER(Constitutive), vp, vp,
                                         C.c_int, C.c_double, C.c_int, C.POINTER(SolveOpts), vp,
                                         C.POINTER(StepStats), vp]
        L.rs_fmg.argtypes = [vp, C.c_int, C.c_int, D]
        _lib = L
    return _lib


def check(code):
    if code != RS_OK:
        raise RsError(code, lib().rs_last_error().decode())


def grid_desc(g: "workloads.GridSpec") -> GridDesc:
    d = GridDesc()
    d.struct_size = C.sizeof(GridDesc)
    d.dim = g.dim
    for l in range(3):
        d.n[l] = g.n[l] if l < g.dim else 1
        d.L[l] = g.L[l] if l < g.dim else 1.0
    for f in range(6):
        d.face_bc[f] = g.face_bc[f] if f < 2 * g.dim else 0
        d.face_value[f] = g.face_value[f] if f < 2 * g.dim else 0.0
    d.patch_face = g.patch_face
    for t in range(2):
        d.patch_lo[t] = g.patch_lo[t]
        d.patch_hi[t] = g.patch_hi[t]
    d.patch_value = g.patch_value
    return d


def constitutive(law: "workloads.LawSpec", ks_field=None, soils=None, soil_id=None):
    """Marshal a law (and optionally a per-node Ks field, or a soil table with
    one soil index per node) into rs_constitutive; returns it with the arrays
    it points to, which the caller keeps alive for the call."""
    c = Constitutive()
    c.struct_size = C.sizeof(Constitutive)
    for name, _ in Constitutive._fields_:
        if name in ("struct_size", "Ks_field", "n_soils", "soils", "soil_id", "coarse_kstar"):
            continue
        setattr(c, name, getattr(law, name))
    c.coarse_kstar = law.coarse_k
    keep = []
    if ks_field is not None:
        ks = np.ascontiguousarray(ks_field, dtype=np.float64)
        c.Ks_field = ks.ctypes.data_as(C.POINTER(C.c_double))
        keep.append(ks)
    if soils:
        tab = (Soil * len(soils))()
        for s, spec in enumerate(soils):
            for name, _ in Soil._fields_:
                setattr(tab[s], name, getattr(spec, name))
        ids = np.ascontiguousarray(soil_id, dtype=np.uint8)
        c.n_soils = len(soils)
        c.soils = tab
        c.soil_id = ids.ctypes.data
        keep += [tab, ids]
    return c, keep


def workspace_bytes(g, precision=RS_FP64) -> int:
    out = C.c_size_t()
    check(lib().rs_workspace_bytes(C.byref(grid_desc(g)), precision, C.byref(out)))
    return out.value


def solve_opts(nu1=2, nu2=2, nu_coarse=32, max_cycles=50, tol_abs=1e-10, stagnation=0,
               mp_inner_cycles=1, fmg=0) -> SolveOpts:
    o = SolveOpts()
    o.struct_size = C.sizeof(SolveOpts)
    o.nu1, o.nu2, o.nu_coarse, o.max_cycles = nu1, nu2, nu_coarse, max_cycles
    o.tol_abs, o.stagnation, o.mp_inner_cycles = tol_abs, stagnation, mp_inner_cycles
    o.fmg = fmg
    return o


class Grid:
    """One solver instance on the current CUDA/HIP device.

    Device memory (the workspace and state arrays) is allocated as torch
    tensors; the stream is torch's current stream unless one is given.
    """

    def __init__(self, w: "workloads.Workload", precision=RS_FP64, stream=None, device=None):
        import torch
        self.torch = torch
        self.w = w
        self.device = torch.device("cuda" if device is None else device)
        self.precision = precision
        self.desc = grid_desc(w.grid)
        nbytes = workspace_bytes(w.grid, precision)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        self._ws_bytes = nbytes
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = C.c_void_p()
        check(lib().rs_create_grid(C.byref(self.desc), precision, C.c_void_p(self._ws_ptr),
                                   nbytes, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.h = h
        self.nlev = lib().rs_num_levels(h)
        self.shapes = []
        for l in range(self.nlev):
            n = (C.c_int * 3)()
            check(lib().rs_level_shape(h, l, n))
            self.shapes.append(tuple(reversed([n[a] for a in range(w.grid.dim)])))
        c, keep = constitutive(w.law, w.Ks_field, w.soils, w.soil_id)
        check(lib().rs_set_constitutive(h, C.byref(c)))
        del keep
        self.set_state(torch.as_tensor(np.ascontiguousarray(w.psi0), device=self.device))

    def close(self):
        if getattr(self, "h", None):
            lib().rs_destroy_grid(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # helpers ---------------------------------------------------------------
    def _dev(self, t):
        assert t.is_cuda and t.dtype == self.torch.float64 and t.is_contiguous()
        return C.c_void_p(t.data_ptr())

    def empty(self, level=0):
        return self.torch.empty(self.shapes[level], dtype=self.torch.float64, device=self.device)

    # C ABI calls -------------------------------------------------------------
    def set_state(self, psi_n, psi_nm1=None, nstep=0, t=0.0):
        psi_n = psi_n.to(self.device, self.torch.float64).contiguous()
        p2 = None
        if psi_nm1 is not None:
            psi_nm1 = psi_nm1.to(self.device, self.torch.float64).contiguous()
            p2 = self._dev(psi_nm1)
        check(lib().rs_set_state(self.h, self._dev(psi_n), p2, nstep, t))
        self.stream.synchronize()

    def get_state(self):
        a, b = self.empty(), self.empty()
        n = C.c_int()
        t = C.c_double()
        check(lib().rs_get_state(self.h, self._dev(a), self._dev(b), C.byref(n), C.byref(t)))
        return a, b, n.value, t.value

    def begin_step(self, dt=None, order=None):
        check(lib().rs_begin_step(self.h, self.w.dt if dt is None else dt,
                                  self.w.order if order is None else order))

    def sweep(self, n=1, level=0):
        check(lib().rs_sweep(self.h, level, n))

    def vcycle(self, nu1=None, nu2=None, want_norm=False):
        r = C.c_double()
        check(lib().rs_vcycle(self.h, self.w.nu1 if nu1 is None else nu1,
                              self.w.nu2 if nu2 is None else nu2,
                              C.byref(r) if want_norm else None))
        return r.value if want_norm else None

    def residual_norm(self):
        r = C.c_double()
        check(lib().rs_residual_norm(self.h, C.byref(r)))
        return r.value

    def residual(self):
        d = self.empty()
        check(lib().rs_residual(self.h, self._dev(d)))
        return d

    def end_step(self):
        check(lib().rs_end_step(self.h))

    def bdf_step(self, dt=None, order=None, opts=None):
        st = StepStats()
        st.struct_size = C.sizeof(StepStats)
        o = opts if opts is not None else solve_opts(self.w.nu1, self.w.nu2, self.w.nu_coarse)
        code = lib().rs_bdf_step(self.h, self.w.dt if dt is None else dt,
                                 self.w.order if order is None else order, C.byref(o),
                                 C.byref(st))
        return code, st

    def field(self, which, level=0):
        out = self.empty(level)
        check(lib().rs_copy_field(self.h, level, which, self._dev(out)))
        return out

    def set_field(self, which, t, level=0):
        t = t.to(self.device, self.torch.float64).contiguous()
        check(lib().rs_set_field(self.h, level, which, self._dev(t)))
        self.stream.synchronize()

    def psi(self, level=0):
        return self.field(FIELD_PSI, level)

    def profile_enable(self, on=True):
        check(lib().rs_profile_enable(self.h, 1 if on else 0))

    def profile_read(self, reset=True):
        """(finest-level sweep ms, kernel launches, pointwise updates)."""
        ms = C.c_double()
        n = C.c_longlong()
        cells = C.c_double()
        check(lib().rs_profile_read(self.h, C.byref(ms), C.byref(n), C.byref(cells),
                                    1 if reset else 0))
        return ms.value, n.value, cells.value

    def fmg(self, nu1=None, nu2=None, want_norm=False):
        """One full-multigrid cycle FMG(nu1, nu2) on the active step."""
        r = C.c_double()
        check(lib().rs_fmg(self.h, self.w.nu1 if nu1 is None else nu1,
                           self.w.nu2 if nu2 is None else nu2,
                           C.byref(r) if want_norm else None))
        return r.value if want_norm else None

    def correction_cycle(self, inner=1, nu1=None, nu2=None, want_norm=False):
        """One FP64 defect correction with FP32 V-cycles (RS_MIXED grids)."""
        r = C.c_double()
        check(lib().rs_correction_cycle(self.h, inner, self.w.nu1 if nu1 is None else nu1,
                                        self.w.nu2 if nu2 is None else nu2,
                                        C.byref(r) if want_norm else None))
        return r.value if want_norm else None


def bdf_step_static(w, psi_n, psi_nm1=None, nstep=0, opts=None, out=None, stream=None):
    """rs_bdf_step_static: one step of workload w from the device state psi_n
    (psi_nm1) with nstep steps taken, in the library's static workspace (no
    allocation by the library).  Returns (code, stats, out)."""
    import torch
    dev = psi_n.device
    if out is None:
        out = torch.empty_like(psi_n)
    for t in (psi_n, out) + (() if psi_nm1 is None else (psi_nm1,)):
        assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        assert tuple(t.shape) == tuple(w.grid.shape)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    d = grid_desc(w.grid)
    c, keep = constitutive(w.law, w.Ks_field, w.soils, w.soil_id)
    o = opts if opts is not None else solve_opts(w.nu1, w.nu2, w.nu_coarse)
    st = StepStats()
    st.struct_size = C.sizeof(StepStats)
    code = lib().rs_bdf_step_static(
        C.byref(d), C.byref(c), C.c_void_p(psi_n.data_ptr()),
        None if psi_nm1 is None else C.c_void_p(psi_nm1.data_ptr()), nstep, w.dt, w.order,
        C.byref(o), C.c_void_p(out.data_ptr()), C.byref(st), C.c_void_p(stream.cuda_stream))
    del keep
    return code, st, out
