"""Truncation bounds of the binomial series for (1 + u)^e - 1 that the sweeps use
for the power terms of the Haverkamp and van Genuchten laws (later Newton
iterates in FP64, the correction increments in FP32): for exponents in
[-1, 7], |binom(e, k)| <= |e| for every k >= 7, so the terms left out after
u^7 (FP64, |u| < 2^-8) stay below 2^-63 |e| and those after u^6 (FP32,
|u| < 1/16) below 1.07 * 2^-24 |e u|.  Also checks that the exponents of the
shipped workloads lie in that range (the series is in use for them)."""
import numpy as np

from paper_2606_04292_amd import workloads as W


def binom(e, k):
    v = 1.0
    for j in range(k):
        v *= (e - j) / (j + 1)
    return v


def exps():
    es = np.linspace(-1.0, 7.0, 3201)
    return es[np.abs(es) > 1e-12]


def test_coefficients_beyond_the_sixth_are_bounded_by_the_exponent():
    for e in exps():
        assert max(abs(binom(e, k)) for k in range(7, 60)) <= abs(e) * (1 + 1e-12), e


def test_fp64_series_tail_below_two_to_minus_63():
    u = 2.0 ** -8
    for e in exps():
        tail = sum(abs(binom(e, k)) * u ** k for k in range(8, 80))
        assert tail < 2.0 ** -63 * abs(e), e


def test_fp32_series_tail_below_one_rounding_of_the_leading_term():
    u = 1.0 / 16
    for e in exps():
        tail = sum(abs(binom(e, k)) * u ** k for k in range(7, 80))
        assert tail < 1.07 * 2.0 ** -24 * abs(e * u), e


def test_series_matches_the_power_where_it_is_used():
    rng = np.random.default_rng(5)
    for e in (-0.6, -0.23, 1.3, 2.5, 3.96):
        c = [binom(e, k) for k in range(1, 8)]
        for u in rng.uniform(-2.0 ** -8, 2.0 ** -8, 50):
            p = 0.0
            for ck in reversed(c):
                p = p * u + ck
            exact = np.expm1(e * np.log1p(u))
            assert abs(p * u - exact) <= 4e-16 * abs(exact) + 1e-300, (e, u)


def test_shipped_workload_exponents_lie_in_the_bounded_range():
    laws = [W.config1().law, W.config2().law, W.config3().law, W.config4().law,
            W.celia_column(65).law]
    laws += [r.law for r in W.serving_requests(64)]
    for L in laws:
        if L.hk_beta:
            assert -1.0 <= L.hk_beta <= 7.0
        if L.vg_n:
            assert -1.0 <= L.vg_n <= 7.0 and 0.0 < 1.0 - 1.0 / L.vg_n <= 1.0
