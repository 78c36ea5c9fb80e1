"""Pins of the oracle's constitutive laws (Table tab:models) against what the
paper prints and what the formulas fix in closed form."""
import dataclasses
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq

from paper_2606_04292_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "constitutive_matching.json")))


def hk_law_cm():
    """The paper's 1-D Haverkamp soil with psi already in cm (psi_unit 1)."""
    return W.LawSpec(model=W.MODEL_HAVERKAMP, theta_s=GOLD["theta_s"], theta_r=GOLD["theta_r"],
                     Ks=GOLD["Ks_cm_per_s"], hk_alpha=GOLD["hk_alpha"], hk_A=GOLD["hk_A"],
                     hk_beta=GOLD["hk_beta"], hk_gamma=GOLD["hk_gamma"], psi_unit=1.0)


def vg_law_cm(alpha, n):
    return W.LawSpec(model=W.MODEL_VGM, theta_s=GOLD["theta_s"], theta_r=GOLD["theta_r"],
                     Ks=GOLD["Ks_cm_per_s"], vg_alpha=alpha, vg_n=n)


def _tol(key):
    return 0.5 * 10.0 ** (-GOLD["printed_decimals"][key])


def test_haverkamp_half_suctions_match_printed_values(orc):
    """Section 4.1: theta hits (theta_s+theta_r)/2 at |psi| = alpha^(1/beta) ~ 36.94 cm and
    K hits Ks/2 at |psi| = A^(1/gamma) ~ 19.08 cm.  Found by root finding on the oracle's law."""
    th, _, Kr, _, _ = orc.law_fns(hk_law_cm())
    mid = 0.5 * (GOLD["theta_s"] + GOLD["theta_r"])
    h_th = brentq(lambda h: th(-h) - mid, 1.0, 1000.0, xtol=1e-13)
    h_K = brentq(lambda h: Kr(-h) - 0.5, 1.0, 1000.0, xtol=1e-13)
    assert abs(h_th - GOLD["printed"]["h_half_theta_cm"]) <= _tol("h_half_theta_cm")
    assert abs(h_K - GOLD["printed"]["h_half_K_cm"]) <= _tol("h_half_K_cm")
    # Gardner's alpha from the WRC half suction (printed 0.01877 /cm)
    assert abs(math.log(2.0) / h_th - GOLD["printed"]["alpha_G_per_cm"]) <= _tol("alpha_G_per_cm")


def test_vgm_matching_reproduces_printed_n_alpha_m(orc):
    """Section 4.1 / Table tab:constitutive_param: with l = 1/2, matching the vGM
    half suctions to Haverkamp's gives n* ~ 3.349, alpha* ~ 0.03165 /cm, m ~ 0.701.
    The root finding uses the oracle's theta and K (l enters through the oracle)."""
    h_th = GOLD["hk_alpha"] ** (1.0 / GOLD["hk_beta"])
    h_K = GOLD["hk_A"] ** (1.0 / GOLD["hk_gamma"])
    mid = 0.5 * (GOLD["theta_s"] + GOLD["theta_r"])

    def alpha_of(n):
        # alpha such that the oracle's vGM theta equals mid at suction h_th
        def fa(a):
            th, _, _, _, _ = orc.law_fns(vg_law_cm(a, n))
            return th(-h_th) - mid
        return brentq(fa, 1e-4, 1.0, xtol=1e-15)

    def kmatch(n):
        a = alpha_of(n)
        _, _, Kr, _, _ = orc.law_fns(vg_law_cm(a, n))
        return Kr(-h_K) - 0.5

    n_star = brentq(kmatch, 1.5, 8.0, xtol=1e-12)
    a_star = alpha_of(n_star)
    assert abs(n_star - GOLD["printed"]["n_star"]) <= _tol("n_star")
    assert abs(a_star - GOLD["printed"]["alpha_VG_star_per_cm"]) <= _tol("alpha_VG_star_per_cm")
    assert abs((1 - 1 / n_star) - GOLD["printed"]["m_star"]) <= _tol("m_star")


def test_vgm_printed_parameters_and_l_sensitivity(orc):
    """With the printed (alpha*, n*) the oracle's vGM law puts theta at the
    Haverkamp midpoint at h_theta and K at Ks/2 at h_K (to the printed digits),
    and the check is sensitive to l: an l = 1 law (the oracle's K divided by
    Se^(1/2)) misses Ks/2 by far more."""
    h_th = GOLD["hk_alpha"] ** (1.0 / GOLD["hk_beta"])
    h_K = GOLD["hk_A"] ** (1.0 / GOLD["hk_gamma"])
    mid = 0.5 * (GOLD["theta_s"] + GOLD["theta_r"])
    dT = GOLD["theta_s"] - GOLD["theta_r"]
    th, _, Kr, _, _ = orc.law_fns(vg_law_cm(GOLD["printed"]["alpha_VG_star_per_cm"],
                                            GOLD["printed"]["n_star"]))
    assert abs(th(-h_th) - mid) / dT < 2e-3
    assert abs(Kr(-h_K) - 0.5) < 5e-3
    Se = (th(-h_K) - GOLD["theta_r"]) / dT
    assert abs(Kr(-h_K) * Se ** 0.5 - 0.5) > 0.02


@pytest.mark.parametrize("which", ["hk", "vg"])
def test_closed_forms_and_limits(orc, which):
    if which == "hk":
        law = dataclasses.replace(W.config3().law)
        th, dth, Kr, _, _ = orc.law_fns(law)
        u = law.psi_unit
        h_th = law.hk_alpha ** (1 / law.hk_beta) / u
        h_K = law.hk_A ** (1 / law.hk_gamma) / u
        assert th(-h_th) == pytest.approx(0.5 * (law.theta_s + law.theta_r), rel=1e-14)
        assert Kr(-h_K) == pytest.approx(0.5, rel=1e-14)
    else:
        law = W.config1().law
        th, dth, Kr, _, _ = orc.law_fns(law)
        # Se = 2^-m at alpha |psi| = 1
        m = 1 - 1 / law.vg_n
        assert th(-1 / law.vg_alpha) == pytest.approx(
            law.theta_r + (law.theta_s - law.theta_r) * 2.0 ** (-m), rel=1e-14)
    # saturated branch (reading: psi >= 0 is saturated)
    assert th(0.0) == law.theta_s and th(0.3) == law.theta_s
    assert dth(0.0) == 0.0 and Kr(0.0) == 1.0 and Kr(2.0) == 1.0
    # continuity at saturation and the dry limit
    assert th(-1e-12) == pytest.approx(law.theta_s, abs=1e-9)
    assert th(-1e6) == pytest.approx(law.theta_r, abs=1e-6)
    assert Kr(-1e-12) == pytest.approx(1.0, abs=1e-6)


@pytest.mark.parametrize("cfg", [W.config1, W.config2, W.config3, W.config4])
def test_dtheta_matches_richardson_difference_and_is_positive(orc, cfg):
    """theta' against a Richardson-extrapolated central difference of the
    oracle's theta (independent of the analytic derivative), and assumption A1
    (theta' > 0) on psi < 0."""
    law = cfg(n=5) if cfg is not W.config4 else cfg(5, 5)
    law = law.law
    th, dth, _, _, _ = orc.law_fns(law)
    for psi in -np.geomspace(2e-2, 5.0, 40):
        h = 1e-3 * abs(psi)
        d1 = (th(psi + h) - th(psi - h)) / (2 * h)
        d2 = (th(psi + h / 2) - th(psi - h / 2)) / h
        rich = (4 * d2 - d1) / 3
        an = dth(psi)
        assert an > 0.0
        assert an == pytest.approx(rich, rel=1e-6, abs=1e-300)


def test_feddes_piecewise_shape(orc):
    law = W.config4(5, 5).law
    _, _, _, a, da = orc.law_fns(law)
    assert a(-100.0) == 0.0 and a(-80.0) == 0.0
    assert a(-42.0) == pytest.approx(0.5)            # halfway up the rising branch
    assert a(-4.0) == 1.0 and a(-1.0) == 1.0
    assert a(-0.175) == pytest.approx(0.5)           # halfway down the falling branch
    assert a(-0.1) == 0.0 and a(0.5) == 0.0
    assert da(-42.0) == pytest.approx(1 / 76.0) and da(-0.2) == pytest.approx(-1 / 0.15)
    assert da(-1.0) == 0.0
    # A2: non-negative slope on [psi_start, psi_opt] = [h4, h2)
    for x in np.linspace(-80.0, -0.2500001, 50):
        assert da(x) >= 0.0


def test_gardner_law_closed_forms_and_printed_matching(orc):
    """Table tab:models, Gardner: theta_r + dT e^(alpha psi) and Ks e^(alpha psi)
    below saturation.  With the printed alpha_G = 0.01877 /cm, theta passes the
    Haverkamp midpoint at the printed 36.94 cm (to the printed digits) and WRC
    and HCF share that half suction; theta' against a Richardson difference."""
    soil = W.celia_soils()[0]
    assert soil.gd_alpha == GOLD["printed"]["alpha_G_per_cm"]
    th, dth, Kr, _, _ = orc.law_fns(soil)
    dT = soil.theta_s - soil.theta_r
    h_half = math.log(2.0) / soil.gd_alpha
    assert abs(h_half - GOLD["printed"]["h_half_theta_cm"]) <= 0.02
    assert th(-h_half) == pytest.approx(soil.theta_r + 0.5 * dT, rel=1e-15)
    assert Kr(-h_half) == pytest.approx(0.5, rel=1e-15)
    for psi in (-0.5, -12.0, -61.5, -400.0):
        e = math.exp(soil.gd_alpha * psi)
        assert th(psi) == pytest.approx(soil.theta_r + dT * e, rel=1e-15)
        assert Kr(psi) == pytest.approx(e, rel=1e-15)
        h = 1e-3 * abs(psi)
        d1 = (th(psi + h) - th(psi - h)) / (2 * h)
        d2 = (th(psi + h / 2) - th(psi - h / 2)) / h
        assert dth(psi) == pytest.approx((4 * d2 - d1) / 3, rel=1e-6)
        assert dth(psi) > 0.0
    assert th(0.0) == soil.theta_s and dth(0.0) == 0.0 and Kr(0.0) == 1.0 and Kr(5.0) == 1.0
    # psi_unit scales psi before the law, as for Haverkamp
    m = dataclasses.replace(soil, psi_unit=100.0, gd_alpha=soil.gd_alpha)
    thm, _, Krm, _, _ = orc.law_fns(m)
    assert thm(-0.3) == pytest.approx(th(-30.0), rel=1e-15)
    assert Krm(-0.3) == pytest.approx(Kr(-30.0), rel=1e-15)
