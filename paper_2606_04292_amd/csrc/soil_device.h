// Device-side constitutive laws, sink and the pointwise Newton solve.
//
// theta(psi), theta'(psi), K(psi)/Ks follow Table tab:models (Haverkamp;
// van Genuchten - Mualem with m = 1 - 1/n and l = 1/2); psi >= 0 is saturated.
// The vGM forms are rearranged to avoid cancellation:
//   P = (alpha|psi|)^n = exp(n log(alpha|psi|)),  Se = exp(-m log1p(P)),
//   1 - Se^(1/m) = P / (1 + P), so the Mualem bracket is
//   1 - (P/(1+P))^m = -expm1(m (n log(alpha|psi|) - log1p(P))).
// Haverkamp uses Q = |u psi|^beta = exp(beta log|u psi|) and
//   theta' = u beta (theta - theta_r) (Q / (alpha + Q)) / |u psi|.
// The sweep and residual evaluate ln, ln(1+p) and exp with the short
// series below (a few ulp); the once-per-step K(psi) uses the library ones.
// Each law is a template specialisation so the sweep kernels carry no model
// switch; the generic entry points dispatch on Law::model.
#pragma once

#include "rs_internal.h"

namespace rs {

// 1/x from the hardware estimate refined by two Newton-Raphson steps
// (error of a few ulp; used where a correctly rounded quotient is not needed).
__device__ __forceinline__ double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// 1/x from the hardware estimate (about 2^-24) refined by one Newton-Raphson
// step: within ~11 ulp, enough where the quotient only feeds a self-correcting
// iteration or a term already carrying that much rounding.
__device__ __forceinline__ double rcp_1nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Natural logarithm of a positive normal double.  x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), ln x = e ln2 + 2 atanh(s), s = (m-1)/(m+1), |s| <= 0.1716,
// with the atanh series 2 s (1 + s^2/3 + ... + s^18/19) (truncation < 3e-17)
// and ln2 split Cody-Waite style so that e ln2_hi is exact.
constexpr double kLn2Hi = 6.93147180369123816490e-01;
constexpr double kLn2Lo = 1.90821492927058770002e-10;
constexpr double kInvLn2 = 1.44269504088896338700e+00;

// p * r + c with the coefficient c in a scalar register pair (one VOP3 FMA;
// no vector moves to materialise the constant).
__device__ __forceinline__ double fma_sc(double p, double r, double c)
{
    double out;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(out) : "v"(p), "v"(r), "s"(c));
    return out;
}

__device__ __forceinline__ double atanh2_series(double s)
{
    const double s2 = s * s;
    double p = 1.0 / 19.0;
    p = fma_sc(p, s2, 1.0 / 17.0);
    p = fma_sc(p, s2, 1.0 / 15.0);
    p = fma_sc(p, s2, 1.0 / 13.0);
    p = fma_sc(p, s2, 1.0 / 11.0);
    p = fma_sc(p, s2, 1.0 / 9.0);
    p = fma_sc(p, s2, 1.0 / 7.0);
    p = fma_sc(p, s2, 1.0 / 5.0);
    p = fma_sc(p, s2, 1.0 / 3.0);
    return fma(2.0 * s * s2, p, 2.0 * s);   // 2 atanh(s)
}

__device__ __forceinline__ double rs_log(double x)
{
    int e = __builtin_amdgcn_frexp_exp(x);
    double m = __builtin_amdgcn_frexp_mant(x);      // [0.5, 1)
    if (m < 0.70710678118654752440) {
        m += m;
        e -= 1;
    }
    const double s = (m - 1.0) * rcp_1nr(m + 1.0);
    const double de = (double)e;
    return fma(de, kLn2Hi, fma(de, kLn2Lo, atanh2_series(s)));
}

// ln(1 + p) for p >= 0: the atanh series with s = p/(2+p) while p < sqrt(2)-1
// (no cancellation for small p), else ln of the rounded sum.
__device__ __forceinline__ double rs_log1p(double p)
{
    if (p < 0.41421356237309504880) return atanh2_series(p * rcp_1nr(2.0 + p));
    return rs_log(1.0 + p);
}

// e^y: y = n ln2 + r (Cody-Waite, |r| <= ln2/2), e^r by its Taylor series to
// r^13/13! (truncation < 5e-18), scaled by 2^n (overflows to inf, underflows
// to 0 past the double range).
__device__ __forceinline__ double rs_exp(double y)
{
    double n = rint(y * kInvLn2);
    n = fmin(fmax(n, -2100.0), 2100.0);
    double r = fma(-n, kLn2Hi, y);
    r = fma(-n, kLn2Lo, r);
    double p = 1.0 / 6227020800.0;                   // 1/13!
    p = fma_sc(p, r, 1.0 / 479001600.0);
    p = fma_sc(p, r, 1.0 / 39916800.0);
    p = fma_sc(p, r, 1.0 / 3628800.0);
    p = fma_sc(p, r, 1.0 / 362880.0);
    p = fma_sc(p, r, 1.0 / 40320.0);
    p = fma_sc(p, r, 1.0 / 5040.0);
    p = fma_sc(p, r, 1.0 / 720.0);
    p = fma_sc(p, r, 1.0 / 120.0);
    p = fma_sc(p, r, 1.0 / 24.0);
    p = fma_sc(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return __builtin_amdgcn_ldexp(p, (int)n);
}

struct ThetaEval {
    double th;
    double dth;
};

template <int MODEL>
__device__ __forceinline__ ThetaEval theta_t(const Law &L, double x)
{
    ThetaEval r;
    if (MODEL == kLinear) {
        r.th = L.tr + L.lin_c * x;
        r.dth = L.lin_c;
        return r;
    }
    if (!(x < 0.0)) {
        r.th = L.ts;
        r.dth = 0.0;
        return r;
    }
    if (MODEL == kGardner) {
        const double au = L.gd_alpha * L.unit;
        const double E = rs_exp(au * x);
        r.th = L.tr + L.dT * E;
        r.dth = au * L.dT * E;
        return r;
    }
    if (MODEL == kHaverkamp) {
        // one reciprocal serves 1/(alpha + Q) = hu w and 1/hu = (alpha + Q) w
        double hu = -L.unit * x;
        double Q = rs_exp(L.hk_beta * rs_log(hu));
        double den = L.hk_alpha + Q;
        double w = rcp_1nr(hu * den);
        double tmr = L.hk_alpha * L.dT * (hu * w);      // theta - theta_r
        r.th = L.tr + tmr;
        r.dth = L.unit * L.hk_beta * tmr * Q * w;
        return r;
    }
    // van Genuchten - Mualem
    double ax = -L.vg_alpha * x;
    double P = rs_exp(L.vg_n * rs_log(ax));
    double Se = rs_exp(-L.vg_m * rs_log1p(P));
    r.th = L.tr + L.dT * Se;
    r.dth = L.dT * L.vg_m * L.vg_n * P * Se * rcp_1nr((1.0 + P) * (-x));
    return r;
}

// (1 + u)^e - 1 by the binomial series to u^7 (c[k - 1] = binom(e, k)), for
// |u| < 2^-8: for -1 <= e <= 7, |binom(e, k)| <= |e| for k >= 8, so the terms left
// out sum to at most |e| |u|^8 / (1 - |u|) < 2^-63 |e|.
__device__ __forceinline__ double pow1p_m1_series(double u, const double *c)
{
    double p = c[6];
    p = fma(p, u, c[5]);
    p = fma(p, u, c[4]);
    p = fma(p, u, c[3]);
    p = fma(p, u, c[2]);
    p = fma(p, u, c[1]);
    p = fma(p, u, c[0]);
    return p * u;
}

// Power terms of the last law evaluation of a pointwise Newton solve.
struct PowState {
    bool ok;       // the last iterate was unsaturated (Haverkamp, vGM)
    double x;      // that iterate
    double ix;     // 1 / x
    double q;      // Haverkamp: Q = (unit |x|)^beta; vGM: P = (alpha |x|)^n
    double se;     // vGM: Se = (1 + P)^-m
    double ix1p;   // vGM: 1 / (1 + P)
};

// theta and theta' at x within a Newton solve.  The power terms of the
// Haverkamp and vGM laws scale from the last iterate's: Q(x) = Q(x') (1 + u)^beta
// and P(x) = P(x') (1 + u)^n with u = x / x' - 1, then Se(x) = Se(x') (1 + v)^-m
// with v = (P(x) - P(x')) / (1 + P(x')); each factor is taken by the binomial
// series while its u or v is below L.series_u (2^-8; 0 for exponents outside
// [-1, 7]) in magnitude, else the powers are evaluated afresh.
template <int MODEL>
__device__ __forceinline__ ThetaEval theta_next(const Law &L, double x, PowState &s)
{
    if (MODEL != kHaverkamp && MODEL != kVgm) return theta_t<MODEL>(L, x);
    ThetaEval r;
    if (!(x < 0.0)) {
        r.th = L.ts;
        r.dth = 0.0;
        s.ok = false;
        return r;
    }
    const double u = (x - s.x) * s.ix;
    const bool ser = s.ok && fabs(u) < L.series_u;
    if (MODEL == kHaverkamp) {
        const double hu = -L.unit * x;
        double Q;
        if (ser) Q = fma(s.q, pow1p_m1_series(u, L.bin1), s.q);
        else Q = rs_exp(L.hk_beta * rs_log(hu));
        const double den = L.hk_alpha + Q;
        const double w = rcp_1nr(hu * den);
        const double tmr = L.hk_alpha * L.dT * (hu * w);
        r.th = L.tr + tmr;
        r.dth = L.unit * L.hk_beta * tmr * Q * w;
        s.q = Q;
        s.ix = -L.unit * (den * w);   // 1/x = -unit / hu
    } else {
        double P, Se;
        bool fresh = !ser;
        if (ser) {
            const double dP = s.q * pow1p_m1_series(u, L.bin1);
            const double v = dP * s.ix1p;
            P = s.q + dP;
            if (fabs(v) < L.series_u) Se = fma(s.se, pow1p_m1_series(v, L.bin2), s.se);
            else fresh = true;
        }
        if (fresh) {
            P = rs_exp(L.vg_n * rs_log(-L.vg_alpha * x));
            Se = rs_exp(-L.vg_m * rs_log1p(P));
        }
        const double w = rcp_1nr((1.0 + P) * (-x));
        r.th = L.tr + L.dT * Se;
        r.dth = L.dT * L.vg_m * L.vg_n * P * Se * w;
        s.q = P;
        s.se = Se;
        s.ix = -(1.0 + P) * w;
        s.ix1p = -x * w;
    }
    s.x = x;
    s.ok = true;
    return r;
}

template <int MODEL>
__device__ __forceinline__ double theta_only_t(const Law &L, double x)
{
    if (MODEL == kLinear) return L.tr + L.lin_c * x;
    if (!(x < 0.0)) return L.ts;
    if (MODEL == kGardner) return L.tr + L.dT * rs_exp(L.gd_alpha * L.unit * x);
    if (MODEL == kHaverkamp) {
        double hu = -L.unit * x;
        double Q = rs_exp(L.hk_beta * rs_log(hu));
        double den = L.hk_alpha + Q;
        double w = rcp_nr(hu * den);
        return L.tr + L.hk_alpha * L.dT * (hu * w);
    }
    double P = rs_exp(L.vg_n * rs_log(-L.vg_alpha * x));
    return L.tr + L.dT * rs_exp(-L.vg_m * rs_log1p(P));
}

__device__ __forceinline__ double theta_only(const Law &L, double x)
{
    switch (L.model) {
    case kGardner: return theta_only_t<kGardner>(L, x);
    case kHaverkamp: return theta_only_t<kHaverkamp>(L, x);
    case kVgm: return theta_only_t<kVgm>(L, x);
    default: return theta_only_t<kLinear>(L, x);
    }
}

// K(psi) / Ks.
__device__ __forceinline__ double krel(const Law &L, double x)
{
    if (L.model == kLinear || !(x < 0.0)) return 1.0;
    if (L.model == kGardner) return exp(L.gd_alpha * L.unit * x);
    if (L.model == kHaverkamp) {
        double hu = -L.unit * x;
        return L.hk_A / (L.hk_A + exp(L.hk_gamma * log(hu)));
    }
    double lg = log(-L.vg_alpha * x);
    double P = exp(L.vg_n * lg);
    double l1 = log1p(P);
    double Se = exp(-L.vg_m * l1);
    double br = -expm1(L.vg_m * (L.vg_n * lg - l1));
    return sqrt(Se) * br * br;
}

// Feddes stress factor a(psi) and its segment slope (half-open segments).
__device__ __forceinline__ void feddes(const Law &L, double x, double &a, double &da)
{
    if (x < L.h4) { a = 0.0; da = 0.0; }
    else if (x < L.h3) { da = 1.0 / (L.h3 - L.h4); a = (x - L.h4) * da; }
    else if (x < L.h2) { a = 1.0; da = 0.0; }
    else if (x < L.h1) { da = -1.0 / (L.h1 - L.h2); a = (L.h1 - x) / (L.h1 - L.h2); }
    else { a = 0.0; da = 0.0; }
}

// Pointwise equation of the NGS update (eq. point-update with the BDF
// coefficient a and sink beta * a_F):  a theta(x) + beta a_F(x) + c x = f.
// NEWTON (or L.newton when NEWTON == 0) safeguarded Newton steps from x0: the
// root stays inside [lo, hi] (initially [(f - a theta_s - beta)/c,
// (f - a theta_r)/c] widened by 1e-12 of the ends' magnitudes, so that the
// root of a saturated cell -- the lower end, F being linear there -- lies
// strictly inside; narrowed by the sign of F at each iterate); a step that does
// not land strictly inside, or a non-positive F', becomes a bisection, unless
// the step leaves the iterate unchanged.  A Newton step (not a bisection) that
// moves x by at most L.newton_tol |x_new| ends the solve for that cell: the
// steps left out would move it by about that step squared times F''/2F'.
template <int MODEL, bool SINK, int NEWTON>
__device__ __forceinline__ double local_solve_t(const Law &L, double a, double beta, double c,
                                                double f, double x0)
{
    double lo, hi;
    if (MODEL == kLinear) {
        lo = -INFINITY;
        hi = INFINITY;
    } else {
        double ic = rcp_nr(c);
        lo = (f - a * L.ts - beta) * ic;
        hi = (f - a * L.tr) * ic;
        double pad = 1e-12 * (fabs(lo) + fabs(hi));
        lo -= pad;
        hi += pad;
    }
    double x = x0;
    bool done = false;
    PowState ps;
    ps.ok = false;
    ps.x = 0.0;
    ps.ix = 0.0;
    ps.q = 0.0;
    ps.se = 1.0;
    ps.ix1p = 0.0;
    const int iters = NEWTON > 0 ? NEWTON : L.newton;
    for (int k = 0; k < iters; ++k) {
        ThetaEval t = theta_next<MODEL>(L, x, ps);
        double F = a * t.th + c * x - f;
        double dF = a * t.dth + c;
        if (SINK) {
            double fa, dfa;
            feddes(L, x, fa, dfa);
            F += beta * fa;
            dF += beta * dfa;
        }
        if (F > 0.0) {
            hi = fmin(hi, x);
        } else if (F < 0.0) {
            lo = fmax(lo, x);
        } else {
            lo = x;
            hi = x;
        }
        double xn = x - F * rcp_1nr(dF);
        const bool bisect = !(dF > 0.0) || (xn != x && !(xn > lo && xn < hi));
        if (bisect) xn = 0.5 * (lo + hi);
        const bool small = !bisect && fabs(xn - x) <= L.newton_tol * fabs(xn);
        // lanes whose solve has ended keep their value while the rest of the
        // wave iterates; the wave leaves once every lane has ended
        if (!done) x = xn;
        done = done || small;
        if (__all(done)) break;
    }
    return x;
}

__device__ __forceinline__ double local_solve(const Law &L, double a, double beta, double c,
                                              double f, double x0)
{
    const bool s = L.sink == kSinkFeddes;
    switch (L.model) {
    case kGardner:
        return s ? local_solve_t<kGardner, true, 0>(L, a, beta, c, f, x0)
                 : local_solve_t<kGardner, false, 0>(L, a, beta, c, f, x0);
    case kHaverkamp:
        return s ? local_solve_t<kHaverkamp, true, 0>(L, a, beta, c, f, x0)
                 : local_solve_t<kHaverkamp, false, 0>(L, a, beta, c, f, x0);
    case kVgm:
        return s ? local_solve_t<kVgm, true, 0>(L, a, beta, c, f, x0)
                 : local_solve_t<kVgm, false, 0>(L, a, beta, c, f, x0);
    default:
        return s ? local_solve_t<kLinear, true, 0>(L, a, beta, c, f, x0)
                 : local_solve_t<kLinear, false, 0>(L, a, beta, c, f, x0);
    }
}

// The pointwise solve with the law of one soil picked at run time (layered
// media): the same iteration as local_solve_t for that soil's model.
template <bool SINK, int NEWTON>
__device__ __forceinline__ double local_solve_soil(const Law &Ls, double a, double beta, double c,
                                                   double f, double x0)
{
    switch (Ls.model) {
    case kGardner: return local_solve_t<kGardner, SINK, NEWTON>(Ls, a, beta, c, f, x0);
    case kHaverkamp: return local_solve_t<kHaverkamp, SINK, NEWTON>(Ls, a, beta, c, f, x0);
    case kVgm: return local_solve_t<kVgm, SINK, NEWTON>(Ls, a, beta, c, f, x0);
    default: return local_solve_t<kLinear, SINK, NEWTON>(Ls, a, beta, c, f, x0);
    }
}

// Node kinds from indices (no node-type array): Dirichlet if on a Dirichlet
// face or on the patch; value = patch value, else the highest-numbered
// Dirichlet face holding the node (*from_state: that face takes its values
// from the state psi^n).
__device__ __forceinline__ bool dirichlet_at(const Geo &g, int i, int j, int k, double *val,
                                             bool *from_state = nullptr)
{
    const int c[3] = {i, j, k};
    bool dir = false;
    double v = 0.0;
    int face = -1;
    // every array below is indexed by constants only (the loops unroll), so
    // the level's descriptor stays in scalar registers
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (l >= g.dim) break;
        if (c[l] == 0 && g.bc[2 * l] == kBcDirichlet) { dir = true; v = g.bcval[2 * l]; face = 2 * l; }
        if (c[l] == g.n[l] - 1 && g.bc[2 * l + 1] == kBcDirichlet) {
            dir = true;
            v = g.bcval[2 * l + 1];
            face = 2 * l + 1;
        }
    }
    if (g.pface >= 0) {
        const int ax = g.pax;
        if ((ax == 0 ? i : (ax == 1 ? j : k)) == g.pat) {
            // the tangential axes in increasing order: (1, 2), (0, 2) or (0, 1)
            const int t0 = ax == 0 ? j : i;
            const int t1 = ax == 2 ? j : k;
            bool in = t0 >= g.plo[0] && t0 <= g.phi[0];
            if (g.dim == 3) in = in && t1 >= g.plo[1] && t1 <= g.phi[1];
            if (in) { dir = true; v = g.pval; face = -1; }
        }
    }
    if (val) *val = v;
    if (from_state) *from_state = face >= 0 && ((g.state_mask >> face) & 1);
    return dir;
}

// dirichlet_at's test (without the value) on a level of DIM axes, every
// descriptor field read unconditionally, so that the reads issue together
// instead of one scalar-load round trip per branch.
template <int DIM>
__device__ __forceinline__ bool dirichlet_t(const Geo &g, int i, int j, int k)
{
    const int c[3] = {i, j, k};
    bool dir = false;
#pragma unroll
    for (int l = 0; l < DIM; ++l)
        dir = dir | ((c[l] == 0) & (g.bc[2 * l] == kBcDirichlet)) |
              ((c[l] == g.n[l] - 1) & (g.bc[2 * l + 1] == kBcDirichlet));
    const int ax = g.pax;
    const int cp = ax == 0 ? i : (ax == 1 ? j : k);
    const int t0 = ax == 0 ? j : i;
    const int t1 = ax == 2 ? j : k;
    bool in = (g.pface >= 0) & (cp == g.pat) & (t0 >= g.plo[0]) & (t0 <= g.phi[0]);
    if (DIM == 3) in = in & (t1 >= g.plo[1]) & (t1 <= g.phi[1]);
    return dir | in;
}

// Division of a 32-bit index by a run-time constant d (Granlund-Montgomery):
// with l = ceil(log2 d) and p = 31 + l, m = ceil(2^p / d) satisfies
// m d - 2^p = e < d <= 2^l, so t m / 2^p = t/d + t e / (d 2^p) < t/d + 1/d for
// t < 2^31 and floor(t m / 2^p) = floor(t / d).  d = 1 is carried as m = 0.
struct FastDiv {
    unsigned m;   // ceil(2^p / d), or 0 for d = 1
    unsigned s;   // p - 32
};

inline FastDiv make_fastdiv(unsigned d)
{
    FastDiv f;
    if (d <= 1) {
        f.m = 0;
        f.s = 0;
        return f;
    }
    unsigned l = 0;
    while ((1ull << l) < d) ++l;
    const unsigned long long p = 31ull + l;
    f.m = (unsigned)(((1ull << p) + d - 1) / d);
    f.s = (unsigned)(p - 32);
    return f;
}

// floor(t / d) for t < 2^31 (grids are limited to 2^31 nodes).
__device__ __forceinline__ unsigned udiv(unsigned t, const FastDiv &f)
{
    return f.m ? (__umulhi(t, f.m) >> f.s) : t;
}

}  // namespace rs
