"""Pins of the root-uptake sink against what its definition fixes.

The root-uptake configuration prescribes S(psi) = beta(z) a(psi) with a root
density decaying exponentially with depth below the surface (e-folding 0.2 m)
and normalised so that the column takes up the potential transpiration
T_p = 5 mm/day; a(psi) is the Feddes stress factor, 1 on its plateau.  The
paper's sink enters eq. model and eq. fully-bdf1 as a volumetric rate.  These
tests read beta(z) out of the oracle's operator and check the normalisation
and the decay law themselves, and that a closed box loses exactly T_p per unit
area in one step (the water balance of eq. fully-bdf1 with no boundary flux).
"""
import dataclasses

import numpy as np

from paper_2606_04292_amd import workloads as W
from tests.balance import volumes_and_weights


def _beta_from_operator(orc, w):
    """beta at every node of the fine grid: N(psi) with a = 0, a linear law of
    zero slope, xi = 0 and a uniform psi on the plateau of a(psi) (a = 1), so
    that theta does not enter, M psi = 0 and N(psi)_i = beta(z_i)."""
    law = dataclasses.replace(w.law, model=W.MODEL_LINEAR, lin_c=0.0, xi=0.0)
    psi = np.full(w.grid.shape, -1.0)
    ww = dataclasses.replace(w, law=law, psi0=psi)
    S = orc.Solver(ww, orc.ORDER_RB)
    S.begin_step()
    S.a = 0.0
    return S.apply_N(psi), law


def test_root_density_integrates_to_potential_transpiration(orc):
    """sum_k w_k h_z beta(z_k) over a column (trapezoidal weights w = 1/2 at the
    two ends, the control volumes of the vertex grid) equals T_p."""
    for nz in (17, 129):
        w = W.config4(9, nz)
        beta, law = _beta_from_operator(orc, w)
        col = beta[:, 3, 4]                      # one vertical column (z first)
        hz = w.grid.L[2] / (nz - 1)
        wk = np.ones(nz)
        wk[0] = wk[-1] = 0.5
        total = float(np.sum(wk * hz * col))
        assert abs(total - law.Tp) <= 1e-14 * law.Tp, (nz, total, law.Tp)
        # 5 mm/day in m/s
        assert abs(law.Tp - 5e-3 / 86400.0) <= 1e-16


def test_root_density_decays_exponentially_with_depth(orc):
    """beta(z) / beta(top) = exp(-(L_z - z) / 0.2 m): largest at the surface,
    e-folding depth 0.2 m, the same in every column."""
    w = W.config4(9, 65)
    beta, law = _beta_from_operator(orc, w)
    nz = w.grid.n[2]
    z = np.arange(nz) * (w.grid.L[2] / (nz - 1))
    ratio = beta[:, 0, 0] / beta[-1, 0, 0]
    expect = np.exp(-(w.grid.L[2] - z) / 0.2)
    assert np.abs(ratio - expect).max() <= 1e-14
    assert np.all(np.diff(beta[:, 0, 0]) > 0)         # increases towards the surface
    assert np.abs(beta - beta[:, :1, :1]).max() == 0.0  # laterally uniform


def test_closed_box_loses_transpiration_times_area(orc):
    """A closed box (no-flux faces) on the plateau of a(psi): one converged
    BDF1 step of eq. fully-bdf1 with xi = 0 loses sum_i V_i (theta_i^n -
    theta_i^{n+1}) / tau = T_p times the surface area, up to V_tot ||r||_inf
    and rounding."""
    w = W.config4(9, 17)
    w = dataclasses.replace(w, grid=dataclasses.replace(w.grid, L=[0.5, 0.25, 0.5]),
                            order=1, steps=1)
    S = orc.Solver(w, orc.ORDER_RB)
    S.begin_step()
    hist = orc.solve_to_floor(S, max_cycles=200)
    psi = S.psi()
    r = hist[-1]
    theta = orc.law_fns(w.law)[0]
    th1 = np.vectorize(theta)(psi)
    th0 = np.vectorize(theta)(w.psi0)
    V, _, _ = volumes_and_weights(w.grid)
    loss = float(np.sum(V * (th0 - th1)) / w.dt)
    area = w.grid.L[0] * w.grid.L[1]
    assert psi.min() > -4.0 and psi.max() < -0.25      # stayed on the plateau
    expect = w.law.Tp * area
    assert abs(loss - expect) <= V.sum() * r + 1e-12 * expect, (loss, expect, r)
