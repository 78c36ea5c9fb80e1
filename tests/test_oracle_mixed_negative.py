"""Why the mixed-precision path solves a correction equation.

On a 1-D van Genuchten column (one BDF1 step of the 65-node configuration
column) two FP32 inner solves sit inside the same FP64 defect-correction
loop r = g - N(psi) (FP64, the oracle's operator):

* naive: FP32 solve of the full variable, N32(p) = N32(fl32(psi)) + fl32(r),
  then psi = p.  The iterate is an FP32 number, so the error stagnates near
  the FP32 spacing of psi (about 1e-7 relative);
* correction form: FP32 solve of N32(psi_b + d) - N32(psi_b) = fl32(r) for d,
  with theta(psi_b + d) - theta(psi_b) formed without cancellation
  (dP = P expm1(n log1p(-t)), dSe = Se expm1(-m log1p(dP / X)), t = d / |psi_b|),
  then psi += d in FP64: it converges to the FP64 step solution.

The operator used by the FP32 solves is written here from the discretisation
(vGM theta, faces m_ij = (K*_i + K*_j) / (2 h^2), xi psi_i, no sink) and checked
first in FP64 against the oracle's N.
"""
import numpy as np
import pytest

import oracle
from paper_2606_04292_amd import workloads as W


def _column():
    w = W.config1(65)
    S = oracle.Solver(w, oracle.ORDER_RB)
    S.begin_step()
    return w, S


def _parts(w, S, dtype):
    law = w.law
    n = w.grid.n[0]
    h = w.grid.L[0] / (n - 1)
    K = S.get(oracle.FIELD_KSTAR).astype(dtype)
    m_face = ((K[:-1] + K[1:]) / dtype(2.0 * h * h)).astype(dtype)   # face i, i + 1
    ts, tr = dtype(law.theta_s), dtype(law.theta_r)
    al, nn = dtype(law.vg_alpha), dtype(law.vg_n)
    mm = dtype(1.0) - dtype(1.0) / nn
    return K, m_face, ts, tr, al, nn, mm


def _theta(x, ts, tr, al, nn, mm):
    se = np.power(np.float64(1.0).astype(x.dtype) + np.power(al * np.abs(x), nn), -mm)
    return np.where(x < 0, tr + (ts - tr) * se, ts)


def _N(x, w, S, dtype):
    """a theta(x) + xi x + sum_j m_ij (x_i - x_j) on the unknowns (rows 1..n-2)."""
    K, m, ts, tr, al, nn, mm = _parts(w, S, dtype)
    a = dtype(S.a)
    x = x.astype(dtype)
    out = a * _theta(x, ts, tr, al, nn, mm) + dtype(w.law.xi) * x
    out[1:-1] += m[1:] * (x[1:-1] - x[2:]) + m[:-1] * (x[1:-1] - x[:-2])
    return out


def _jac(x, w, S, dtype, dth):
    K, m, *_ = _parts(w, S, dtype)
    n = x.shape[0]
    J = np.zeros((n - 2, n - 2), dtype=dtype)
    for r in range(n - 2):
        i = r + 1
        J[r, r] = dtype(S.a) * dth[i] + dtype(w.law.xi) + m[i] + m[i - 1]
        if r > 0:
            J[r, r - 1] = -m[i - 1]
        if r < n - 3:
            J[r, r + 1] = -m[i]
    return J


def _dtheta_dx(x, w, S, dtype):
    _, _, ts, tr, al, nn, mm = _parts(w, S, dtype)
    u = np.power(al * np.abs(x), nn)
    return np.where(x < 0, (ts - tr) * mm * nn * al * np.power(al * np.abs(x), nn - 1)
                    * np.power(1 + u, -mm - 1), 0).astype(dtype)


def _fp64_solution(S):
    oracle.solve_to_floor(S, 400, 0.0)
    return S.psi().copy()


def test_operator_written_here_is_the_oracles():
    w, S = _column()
    rng = np.random.default_rng(3)
    x = S.psi() + rng.uniform(-0.05, 0.05, S.psi().shape)
    x[0], x[-1] = S.psi()[0], S.psi()[-1]
    mine = _N(x, w, S, np.float64)[1:-1]
    ref = S.apply_N(x)[1:-1]
    assert np.abs(mine - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("form", ["naive", "correction"])
def test_fp32_inner_solve_forms(form):
    w, S = _column()
    g = S.get(oracle.FIELD_G)
    start = S.psi().copy()
    ref = _fp64_solution(S)
    f32 = np.float32
    _, _, ts, tr, al, nn, mm = _parts(w, S, f32)
    psi = start.copy()
    errs = []
    for _ in range(12):
        r = g - _N(psi, w, S, np.float64)          # FP64 defect (Dirichlet rows unused)
        r[0] = r[-1] = 0.0
        pb = psi.astype(f32)
        if form == "naive":
            rhs = _N(pb, w, S, f32) + r.astype(f32)
            p = pb.copy()
            for _ in range(8):                       # FP32 Newton on the full variable
                F = (_N(p, w, S, f32) - rhs)[1:-1]
                J = _jac(p, w, S, f32, _dtheta_dx(p, w, S, f32))
                p[1:-1] -= np.linalg.solve(J, F).astype(f32)
            psi = p.astype(np.float64)
        else:
            d = np.zeros_like(pb)
            ab = np.abs(pb)
            P = np.power(al * ab, nn)
            X = f32(1.0) + P
            Se = np.power(X, -mm)
            for _ in range(8):                       # FP32 Newton on the correction
                t = d / ab
                dP = P * np.expm1(nn * np.log1p(-t))
                dSe = Se * np.expm1(-mm * np.log1p(dP / X))
                dth = (ts - tr) * dSe
                Nd = f32(S.a) * dth + f32(w.law.xi) * d
                K, m, *_ = _parts(w, S, f32)
                Nd[1:-1] += m[1:] * (d[1:-1] - d[2:]) + m[:-1] * (d[1:-1] - d[:-2])
                F = (Nd - r.astype(f32))[1:-1]
                J = _jac(pb + d, w, S, f32, _dtheta_dx(pb + d, w, S, f32))
                d[1:-1] -= np.linalg.solve(J, F).astype(f32)
            psi = psi + d.astype(np.float64)
        errs.append(float(np.abs(psi - ref).max() / np.abs(ref).max()))
    floor32 = np.finfo(np.float32).eps / 2
    if form == "naive":
        # stuck at the FP32 representation of psi: no better than a tenth of an
        # FP32 half-ulp, however many outer corrections
        assert min(errs[4:]) >= 0.1 * floor32, errs
    else:
        assert errs[-1] <= 1e-12, errs
