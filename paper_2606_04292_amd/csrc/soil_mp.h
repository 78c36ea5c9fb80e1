// FP32 correction equation of the mixed-precision solve.
//
// With psi the current FP64 iterate and r = g - N(psi) its FP64 defect, the
// correction delta solves N(psi + delta) - N(psi) = r, i.e.
//   a [theta(psi+delta) - theta(psi)] + [S(psi+delta) - S(psi)] + xi delta + M delta = r
// (eq. Nh-def written for the increment).  The FP32 cycles see the base state
// psi_b = fl32(psi) and evaluate the increments without cancellation, so every
// term is proportional to delta and delta = 0 is an exact fixed point when
// r = 0:
//   Haverkamp, both states unsaturated, t = delta/|psi_b|:
//     dQ = Q_b expm1(beta log1p(-t)),  dtheta = -alpha dT dQ / ((alpha+Q_b)(alpha+Q_b+dQ));
//   vGM: dP = P_b expm1(n log1p(-t)),  dSe = Se_b expm1(-m log1p(dP/X_b)),  dtheta = dT dSe;
//   crossing saturation: theta_s - theta(psi) = dT Q/(alpha+Q) (Haverkamp),
//     = -dT expm1(-m log1p(P)) (vGM);
//   Feddes sink: exact piecewise-linear increments.
// Transcendentals use the hardware FP32 log2/exp2; log1p and expm1 use short
// series near zero.  The increments (1 + u)^e - 1 of the power laws take the
// binomial series to u^6 while |u| < 1/16 (coefficients per law, set on the
// host), else expm1(e log1p(u)).
#pragma once

#include "rs_internal.h"

namespace rs {

__device__ __forceinline__ float f_ln(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945f; }
__device__ __forceinline__ float f_exp(float y) { return __builtin_amdgcn_exp2f(y * 1.44269504088896f); }
__device__ __forceinline__ float f_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// ln(1+x), x > -1: 2 atanh(x/(2+x)) series for |x| < 1/2, else ln(1+x).
__device__ __forceinline__ float f_log1p(float x)
{
    if (fabsf(x) < 0.5f) {
        const float s = x * f_rcp(2.0f + x);
        const float s2 = s * s;
        float p = 1.0f / 11.0f;
        p = fmaf(p, s2, 1.0f / 9.0f);
        p = fmaf(p, s2, 1.0f / 7.0f);
        p = fmaf(p, s2, 1.0f / 5.0f);
        p = fmaf(p, s2, 1.0f / 3.0f);
        return fmaf(2.0f * s * s2, p, 2.0f * s);
    }
    return f_ln(1.0f + x);
}

// e^y - 1: Taylor series to y^9/9! for |y| < 1/2, else e^y - 1.
__device__ __forceinline__ float f_expm1(float y)
{
    if (fabsf(y) < 0.5f) {
        float p = 1.0f / 362880.0f;
        p = fmaf(p, y, 1.0f / 40320.0f);
        p = fmaf(p, y, 1.0f / 5040.0f);
        p = fmaf(p, y, 1.0f / 720.0f);
        p = fmaf(p, y, 1.0f / 120.0f);
        p = fmaf(p, y, 1.0f / 24.0f);
        p = fmaf(p, y, 1.0f / 6.0f);
        p = fmaf(p, y, 0.5f);
        p = fmaf(p, y, 1.0f);
        return p * y;
    }
    return f_exp(y) - 1.0f;
}

// Single-precision copy of the law parameters used by the FP32 cycles.
struct Law32 {
    int model;
    float ts, tr, dT;
    float vg_alpha, vg_n, vg_m;
    float hk_alpha, hk_beta, unit;
    float lin_c;
    int sink;
    float h1, h2, h3, h4;
    float xi, kappa;
    int kappa_rule;
    int newton;
    float newton_tol;   // a Newton step of at most newton_tol |d| ends the correction solve
    // binomial coefficients binom(e, k), k = 1..6, of (1 + u)^e - 1 for the
    // exponents of the increments: e = hk_beta (Haverkamp) or vg_n (vGM) in
    // bin1, e = -vg_m (vGM) in bin2
    float bin1[6], bin2[6];
    float series_u;   // 1/16, or 0 when an exponent lies outside [-1, 7]
};

// (1 + u)^e - 1.  For |u| < series_u (1/16) the binomial series u (c1 + u (c2 + ... + u c6))
// with c_k = binom(e, k): for -1 <= e <= 7, |binom(e, k)| <= |e| for k >= 7, so the
// terms left out sum to at most |e u| |u|^6 / (1 - |u|) < 1.07 * 2^-24 |e u|, about
// an FP32 rounding of the leading term; otherwise expm1(e log1p(u)).
// Proportional to u, so u = 0 gives 0.
__device__ __forceinline__ float pow1p_m1(float u, float e, const float *c, float series_u)
{
    if (fabsf(u) < series_u) {
        float p = c[5];
        p = fmaf(p, u, c[4]);
        p = fmaf(p, u, c[3]);
        p = fmaf(p, u, c[2]);
        p = fmaf(p, u, c[1]);
        p = fmaf(p, u, c[0]);
        return p * u;
    }
    return f_expm1(e * f_log1p(u));
}

// Base-state quantities of one node (evaluated once per update).
struct Base {
    float psi;       // psi_b
    bool sat;        // psi_b >= 0
    float q, den;    // Haverkamp: Q_b, alpha + Q_b; vGM: P_b, X_b = 1 + P_b
    float se;        // vGM: Se_b
    float ipsi, iden;   // 1 / (-psi_b), 1 / den (unsaturated base states)
};

template <int MODEL>
__device__ __forceinline__ Base base_of(const Law32 &L, float pb)
{
    Base b;
    b.psi = pb;
    b.sat = !(pb < 0.0f);
    b.q = 0.0f;
    b.den = 1.0f;
    b.se = 1.0f;
    b.ipsi = 0.0f;
    b.iden = 1.0f;
    if (MODEL == kLinear || b.sat) return b;
    if (MODEL == kHaverkamp) {
        b.q = f_exp(L.hk_beta * f_ln(-L.unit * pb));
        b.den = L.hk_alpha + b.q;
    } else {
        b.q = f_exp(L.vg_n * f_ln(-L.vg_alpha * pb));
        b.den = 1.0f + b.q;
        b.se = f_exp(-L.vg_m * f_log1p(b.q));
    }
    b.ipsi = f_rcp(-pb);
    b.iden = f_rcp(b.den);
    return b;
}

// theta_s - theta(psi_b) and theta(psi_b) - theta_r, without cancellation.
template <int MODEL>
__device__ __forceinline__ void base_room(const Law32 &L, const Base &b, float &up, float &down)
{
    if (MODEL == kLinear) {
        up = INFINITY;
        down = INFINITY;
    } else if (b.sat) {
        up = 0.0f;
        down = L.dT;
    } else if (MODEL == kHaverkamp) {
        up = L.dT * b.q * b.iden;
        down = L.hk_alpha * L.dT * b.iden;
    } else {
        up = -L.dT * f_expm1(-L.vg_m * f_log1p(b.q));
        down = L.dT * b.se;
    }
}

// theta(psi_b + delta) - theta(psi_b) and theta'(psi_b + delta).
template <int MODEL>
__device__ __forceinline__ void dtheta32(const Law32 &L, const Base &b, float delta, float &dth,
                                         float &slope)
{
    if (MODEL == kLinear) {
        dth = L.lin_c * delta;
        slope = L.lin_c;
        return;
    }
    const float x = b.psi + delta;
    const bool xsat = !(x < 0.0f);
    if (b.sat && xsat) {
        dth = 0.0f;
        slope = 0.0f;
        return;
    }
    if (MODEL == kHaverkamp) {
        if (!b.sat && !xsat) {
            const float t = delta * b.ipsi;
            const float dq = b.q * pow1p_m1(-t, L.hk_beta, L.bin1, L.series_u);
            const float den = b.den + dq;
            const float hu = -L.unit * x;
            // one reciprocal serves 1/den = hu w and 1/hu = den w
            const float w = f_rcp(hu * den);
            const float r = hu * w;
            dth = -L.hk_alpha * L.dT * dq * r * b.iden;
            slope = L.unit * L.hk_beta * (L.hk_alpha * L.dT * r) * ((b.q + dq) * r) * (den * w);
            return;
        }
        if (!b.sat) {          // wets up to saturation
            dth = L.dT * b.q * b.iden;
            slope = 0.0f;
            return;
        }
        const float hu = -L.unit * x;    // dries from saturation
        const float q = f_exp(L.hk_beta * f_ln(hu));
        const float r = f_rcp(L.hk_alpha + q);
        dth = -L.dT * q * r;
        slope = L.unit * L.hk_beta * (L.hk_alpha * L.dT * r) * (q * r) * f_rcp(hu);
        return;
    }
    // van Genuchten - Mualem
    if (!b.sat && !xsat) {
        const float t = delta * b.ipsi;
        const float dp = b.q * pow1p_m1(-t, L.vg_n, L.bin1, L.series_u);
        const float dse = b.se * pow1p_m1(dp * b.iden, -L.vg_m, L.bin2, L.series_u);
        dth = L.dT * dse;
        const float P = b.q + dp, X = b.den + dp, Se = b.se + dse;
        slope = L.dT * L.vg_m * L.vg_n * P * Se * f_rcp(X * (-x));
        return;
    }
    if (!b.sat) {
        dth = -L.dT * f_expm1(-L.vg_m * f_log1p(b.q));
        slope = 0.0f;
        return;
    }
    const float P = f_exp(L.vg_n * f_ln(-L.vg_alpha * x));
    const float Se = f_exp(-L.vg_m * f_log1p(P));
    dth = L.dT * f_expm1(-L.vg_m * f_log1p(P));
    slope = L.dT * L.vg_m * L.vg_n * P * Se * f_rcp((1.0f + P) * (-x));
}

// Feddes a(psi_b + delta) - a(psi_b) as exact piecewise-linear increments, and
// the slope at psi_b + delta.
__device__ __forceinline__ float seg_inc(float pb, float delta, float lo, float hi)
{
    const float x = pb + delta;
    const bool in_b = pb >= lo && pb < hi;
    const bool in_x = x >= lo && x < hi;
    if (in_b && in_x) return delta;
    return fminf(fmaxf(x, lo), hi) - fminf(fmaxf(pb, lo), hi);
}

__device__ __forceinline__ void dfeddes32(const Law32 &L, float pb, float delta, float &da,
                                          float &slope)
{
    const float s1 = f_rcp(L.h3 - L.h4), s2 = -f_rcp(L.h1 - L.h2);
    da = s1 * seg_inc(pb, delta, L.h4, L.h3) + s2 * seg_inc(pb, delta, L.h2, L.h1);
    const float x = pb + delta;
    slope = (x >= L.h4 && x < L.h3) ? s1 : ((x >= L.h2 && x < L.h1) ? s2 : 0.0f);
}

__device__ __forceinline__ float feddes_value32(const Law32 &L, float x)
{
    if (x < L.h4) return 0.0f;
    if (x < L.h3) return (x - L.h4) * f_rcp(L.h3 - L.h4);
    if (x < L.h2) return 1.0f;
    if (x < L.h1) return (L.h1 - x) * f_rcp(L.h1 - L.h2);
    return 0.0f;
}

// Scalar correction update: a dtheta(d) + beta da(d) + c d = f by the same
// safeguarded Newton iteration as the FP64 smoother (bracket from the room
// theta has to move and the sink range, widened by 1e-6 of its ends), ending
// after a Newton step of at most newton_tol |d|.
template <int MODEL, bool SINK>
__device__ __forceinline__ float local_solve32(const Law32 &L, float a, float beta, float c,
                                               float f, const Base &b, float d0)
{
    float lo, hi;
    if (MODEL == kLinear) {
        lo = -INFINITY;
        hi = INFINITY;
    } else {
        float up, down;
        base_room<MODEL>(L, b, up, down);
        float ab = 0.0f;
        if (SINK) ab = feddes_value32(L, b.psi);
        const float ic = f_rcp(c);
        lo = (f - a * up - (SINK ? beta * (1.0f - ab) : 0.0f)) * ic;
        hi = (f + a * down + (SINK ? beta * ab : 0.0f)) * ic;
        const float pad = 1e-6f * (fabsf(lo) + fabsf(hi));
        lo -= pad;
        hi += pad;
    }
    float d = d0;
    bool done = false;
    for (int k = 0; k < L.newton; ++k) {
        float dth, slope;
        dtheta32<MODEL>(L, b, d, dth, slope);
        float F = a * dth + c * d - f;
        float dF = a * slope + c;
        if (SINK) {
            float da, ds;
            dfeddes32(L, b.psi, d, da, ds);
            F += beta * da;
            dF += beta * ds;
        }
        if (F > 0.0f) hi = fminf(hi, d);
        else if (F < 0.0f) lo = fmaxf(lo, d);
        else { lo = d; hi = d; }
        float dn = d - F * f_rcp(dF);
        const bool bisect = !(dF > 0.0f) || (dn != d && !(dn > lo && dn < hi));
        if (bisect) dn = 0.5f * (lo + hi);
        const bool small = !bisect && fabsf(dn - d) <= L.newton_tol * fabsf(dn);
        if (!done) d = dn;
        done = done || small;
        if (__all(done)) break;
    }
    return d;
}

}  // namespace rs
