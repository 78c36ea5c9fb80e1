"""ctypes wrapper of the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users; the product library never imports this.
It shares no code with the HIP path: it consumes the same problem
descriptions (``paper_2606_04292_amd.workloads``) and marshals them into its
own C structures.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORDER_LEX = 0
ORDER_RB = 1
FIELD_PSI, FIELD_KSTAR, FIELD_G, FIELD_PSIBAR, FIELD_PSI_N, FIELD_PSI_NM1 = range(6)
COARSE_INJECT, COARSE_FW = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off",
               "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("L", C.c_double * 3),
                ("face_bc", C.c_int * 6), ("face_value", C.c_double * 6),
                ("patch_face", C.c_int), ("patch_lo", C.c_int * 2),
                ("patch_hi", C.c_int * 2), ("patch_value", C.c_double)]


class Params(C.Structure):
    _fields_ = [("model", C.c_int), ("theta_s", C.c_double), ("theta_r", C.c_double),
                ("Ks", C.c_double), ("vg_alpha", C.c_double), ("vg_n", C.c_double),
                ("hk_alpha", C.c_double), ("hk_beta", C.c_double), ("hk_A", C.c_double),
                ("hk_gamma", C.c_double), ("psi_unit", C.c_double), ("lin_c", C.c_double),
                ("sink", C.c_int), ("Tp", C.c_double), ("root_len", C.c_double),
                ("h1", C.c_double), ("h2", C.c_double), ("h3", C.c_double),
                ("h4", C.c_double), ("xi", C.c_double), ("kappa_rule", C.c_int),
                ("kappa", C.c_double), ("newton_iters", C.c_int), ("lag_extrap", C.c_int),
                ("newton_tol", C.c_double), ("gd_alpha", C.c_double), ("coarse_k", C.c_int)]


_lib = None
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp = C.c_void_p
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.POINTER(Grid), C.POINTER(Params), _D, C.c_int, C.c_int]
        L.orc_destroy.argtypes = [vp]
        L.orc_nlevels.argtypes = [vp]
        L.orc_level_shape.argtypes = [vp, C.c_int, _I]
        L.orc_set_state.argtypes = [vp, _D, _D, C.c_int]
        L.orc_begin_step.argtypes = [vp, C.c_double, C.c_int]
        L.orc_end_step.argtypes = [vp]
        L.orc_sweep.argtypes = [vp, C.c_int, C.c_int]
        L.orc_residual.restype = C.c_double
        L.orc_residual.argtypes = [vp, C.c_int, _D]
        L.orc_defect_scale.restype = C.c_double
        L.orc_defect_scale.argtypes = [vp, C.c_int]
        L.orc_apply_N.argtypes = [vp, C.c_int, _D, _D]
        L.orc_restrict.argtypes = [vp, C.c_int]
        L.orc_prolong.argtypes = [vp, C.c_int]
        L.orc_vcycle.argtypes = [vp, C.c_int, C.c_int]
        L.orc_fmg.argtypes = [vp, C.c_int, C.c_int]
        L.orc_solve_step.restype = C.c_int
        L.orc_solve_step.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_double, _D]
        L.orc_get_field.argtypes = [vp, C.c_int, C.c_int, _D]
        L.orc_set_field.argtypes = [vp, C.c_int, C.c_int, _D]
        L.orc_update_points.argtypes = [vp, C.c_int, C.c_int, _I, _D]
        L.orc_node_kinds.argtypes = [vp, C.c_int, C.POINTER(C.c_int8)]
        L.orc_dense_M.restype = C.c_int
        L.orc_dense_M.argtypes = [vp, C.c_int, _D, _D, _I]
        L.orc_get_a.restype = C.c_double
        L.orc_get_a.argtypes = [vp]
        L.orc_set_a.argtypes = [vp, C.c_double]
        L.orc_get_lambdaU.restype = C.c_double
        L.orc_get_lambdaU.argtypes = [vp, C.c_int]
        L.orc_set_soils.restype = C.c_int
        L.orc_set_soils.argtypes = [vp, C.c_int, C.POINTER(Params), C.c_void_p]
        L.orc_local_solve.restype = C.c_double
        L.orc_local_solve.argtypes = [C.POINTER(Params), C.c_double, C.c_double, C.c_double,
                                      C.c_double, C.c_double, C.c_int, _I]
        for nm in ("orc_theta", "orc_dtheta", "orc_Krel", "orc_feddes", "orc_dfeddes"):
            f = getattr(L, nm)
            f.restype = C.c_double
            f.argtypes = [C.POINTER(Params), C.c_double]
        L.orc_eval_law.argtypes = [C.POINTER(Params), C.c_int, _D, _D, _D, _D]
        L.orc_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


def make_grid(g) -> Grid:
    G = Grid()
    G.dim = g.dim
    for l in range(3):
        G.n[l] = g.n[l] if l < g.dim else 1
        G.L[l] = g.L[l] if l < g.dim else 1.0
    for f in range(6):
        G.face_bc[f] = g.face_bc[f] if f < 2 * g.dim else 0
        G.face_value[f] = g.face_value[f] if f < 2 * g.dim else 0.0
    G.patch_face = g.patch_face
    for t in range(2):
        G.patch_lo[t] = g.patch_lo[t]
        G.patch_hi[t] = g.patch_hi[t]
    G.patch_value = g.patch_value
    return G


def make_params(law) -> Params:
    P = Params()
    for name, _ in Params._fields_:
        setattr(P, name, getattr(law, name))
    return P


def threads() -> int:
    return lib().orc_threads()


class Solver:
    """One oracle solver instance for a workload (grid + law + Ks field)."""

    def __init__(self, w, ordering=ORDER_RB, nu_coarse=None):
        self.w = w
        self.G = make_grid(w.grid)
        self.P = make_params(w.law)
        ks = None if w.Ks_field is None else np.ascontiguousarray(w.Ks_field, dtype=np.float64)
        self._ks = ks
        nc = w.nu_coarse if nu_coarse is None else nu_coarse
        self.h = lib().orc_create(C.byref(self.G), C.byref(self.P), _dp(ks), ordering, nc)
        self.nlev = lib().orc_nlevels(self.h)
        self.shapes = []
        for l in range(self.nlev):
            n = (C.c_int * 3)()
            lib().orc_level_shape(self.h, l, n)
            self.shapes.append(tuple(reversed([n[a] for a in range(w.grid.dim)])))
        if w.soils:
            table = (Params * len(w.soils))(*[make_params(s) for s in w.soils])
            ids = np.ascontiguousarray(w.soil_id, dtype=np.uint8)
            if lib().orc_set_soils(self.h, len(w.soils), table, ids.ctypes.data_as(C.c_void_p)) != 0:
                raise ValueError("bad soil table or soil index")
        self.set_state(w.psi0)

    def __del__(self):
        try:
            if self.h:
                lib().orc_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # state -----------------------------------------------------------------
    def set_state(self, psi_n, psi_nm1=None, nstep=0):
        a = np.ascontiguousarray(psi_n, dtype=np.float64)
        b = None if psi_nm1 is None else np.ascontiguousarray(psi_nm1, dtype=np.float64)
        lib().orc_set_state(self.h, _dp(a), _dp(b), nstep)

    def begin_step(self, dt=None, order=None):
        lib().orc_begin_step(self.h, self.w.dt if dt is None else dt,
                             self.w.order if order is None else order)

    def end_step(self):
        lib().orc_end_step(self.h)

    @property
    def a(self):
        return lib().orc_get_a(self.h)

    @a.setter
    def a(self, v):
        lib().orc_set_a(self.h, v)

    # fields ----------------------------------------------------------------
    def get(self, which, level=0):
        shape = self.shapes[0] if which >= FIELD_PSI_N else self.shapes[level]
        out = np.empty(shape, dtype=np.float64)
        lib().orc_get_field(self.h, level, which, _dp(out))
        return out

    def set(self, which, arr, level=0):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        lib().orc_set_field(self.h, level, which, _dp(a))

    def psi(self, level=0):
        return self.get(FIELD_PSI, level)

    def kinds(self, level=0):
        out = np.empty(self.shapes[level], dtype=np.int8)
        lib().orc_node_kinds(self.h, level, out.ctypes.data_as(C.POINTER(C.c_int8)))
        return out

    # operations ------------------------------------------------------------
    def sweep(self, n=1, level=0):
        lib().orc_sweep(self.h, level, n)

    def residual(self, level=0, want_vector=False):
        d = np.empty(self.shapes[level], dtype=np.float64) if want_vector else None
        r = lib().orc_residual(self.h, level, _dp(d))
        return (r, d) if want_vector else r

    def defect_scale(self, level=0):
        """Largest per-node sum of the magnitudes of the defect's terms."""
        return lib().orc_defect_scale(self.h, level)

    def apply_N(self, psi, level=0):
        a = np.ascontiguousarray(psi, dtype=np.float64)
        out = np.empty(self.shapes[level], dtype=np.float64)
        lib().orc_apply_N(self.h, level, _dp(a), _dp(out))
        return out

    def vcycle(self, nu1=None, nu2=None):
        lib().orc_vcycle(self.h, self.w.nu1 if nu1 is None else nu1,
                         self.w.nu2 if nu2 is None else nu2)

    def fmg(self, nu1=None, nu2=None):
        """One full-multigrid cycle FMG(nu1, nu2) on the active step."""
        lib().orc_fmg(self.h, self.w.nu1 if nu1 is None else nu1,
                      self.w.nu2 if nu2 is None else nu2)

    def solve_step(self, max_cycles=50, tol=0.0, nu1=None, nu2=None):
        hist = np.zeros(max_cycles + 1)
        c = lib().orc_solve_step(self.h, self.w.nu1 if nu1 is None else nu1,
                                 self.w.nu2 if nu2 is None else nu2, max_cycles, tol, _dp(hist))
        return c, hist[:c + 1]

    def update_points(self, idx, level=0):
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        out = np.empty(idx.shape[0], dtype=np.float64)
        lib().orc_update_points(self.h, level, idx.shape[0],
                                idx.ctypes.data_as(_I), _dp(out))
        return out

    def dense_M(self, level=0):
        nu = lib().orc_dense_M(self.h, level, None, None, None)
        M = np.zeros((nu, nu))
        kap = np.zeros(nu)
        unk = np.zeros(nu, dtype=np.int32)
        lib().orc_dense_M(self.h, level, _dp(M), _dp(kap), unk.ctypes.data_as(_I))
        return M, kap, unk

    def lambdaU(self, level=0):
        return lib().orc_get_lambdaU(self.h, level)


def law_fns(law):
    """Scalar theta, dtheta, Krel, feddes, dfeddes bound to a law."""
    P = make_params(law)
    L = lib()
    return (lambda x: L.orc_theta(C.byref(P), float(x)),
            lambda x: L.orc_dtheta(C.byref(P), float(x)),
            lambda x: L.orc_Krel(C.byref(P), float(x)),
            lambda x: L.orc_feddes(C.byref(P), float(x)),
            lambda x: L.orc_dfeddes(C.byref(P), float(x)))


def local_solve(law, a, beta, c, f, x0, iters, evals=False):
    """The pointwise solve; with evals=True also the number of F evaluations."""
    P = make_params(law)
    n = C.c_int(0)
    x = lib().orc_local_solve(C.byref(P), a, beta, c, f, x0, iters, C.byref(n))
    return (x, n.value) if evals else x


def run_steps(w, steps=None, ordering=ORDER_RB, max_cycles=60, tol=0.0, stagnation=True):
    """Run the time loop; each step iterates V-cycles until the residual is
    <= tol or stops decreasing.  Returns the solver (state = last step)."""
    S = Solver(w, ordering)
    steps = w.steps if steps is None else steps
    for _ in range(steps):
        S.begin_step()
        solve_to_floor(S, max_cycles, tol, stagnation)
        S.end_step()
    return S


def solve_to_floor(S, max_cycles=60, tol=0.0, stagnation=True):
    """V-cycles until ||r|| <= tol, or (stagnation) the rounding floor is
    reached: two cycles in a row set no new minimum of the norm; or
    max_cycles.  A slow but steady contraction keeps iterating."""
    r = S.residual()
    hist = [r]
    best = r
    slow = 0
    for _ in range(max_cycles):
        if r <= tol:
            break
        S.vcycle()
        r = S.residual()
        hist.append(r)
        if stagnation:
            if r < best:
                best, slow = r, 0
            else:
                slow += 1
                if slow >= 2:
                    break
    return hist
