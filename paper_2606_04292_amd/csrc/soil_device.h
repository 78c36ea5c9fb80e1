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
#pragma once

#include "rs_internal.h"

namespace rs {

struct ThetaEval {
    double th;
    double dth;
};

__device__ __forceinline__ ThetaEval theta_eval(const Law &L, double x)
{
    ThetaEval r;
    if (L.model == kLinear) {
        r.th = L.tr + L.lin_c * x;
        r.dth = L.lin_c;
        return r;
    }
    if (!(x < 0.0)) {
        r.th = L.ts;
        r.dth = 0.0;
        return r;
    }
    if (L.model == kHaverkamp) {
        double hu = -L.unit * x;
        double Q = exp(L.hk_beta * log(hu));
        double rden = 1.0 / (L.hk_alpha + Q);
        double tmr = L.hk_alpha * L.dT * rden;          // theta - theta_r
        r.th = L.tr + tmr;
        r.dth = L.unit * L.hk_beta * tmr * (Q * rden) / hu;
        return r;
    }
    // van Genuchten - Mualem
    double ax = -L.vg_alpha * x;
    double P = exp(L.vg_n * log(ax));
    double Se = exp(-L.vg_m * log1p(P));
    r.th = L.tr + L.dT * Se;
    r.dth = L.dT * L.vg_m * L.vg_n * P * Se / ((1.0 + P) * (-x));
    return r;
}

__device__ __forceinline__ double theta_only(const Law &L, double x)
{
    return theta_eval(L, x).th;
}

// K(psi) / Ks.
__device__ __forceinline__ double krel(const Law &L, double x)
{
    if (L.model == kLinear || !(x < 0.0)) return 1.0;
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
// Exactly L.newton safeguarded Newton steps from x0: the root stays inside
// [lo, hi] (initially [(f - a theta_s - beta)/c, (f - a theta_r)/c] widened by
// 1e-12 of the ends' magnitudes, so that the root of a saturated cell -- the
// lower end, F being linear there -- lies strictly inside; narrowed by the
// sign of F at each iterate); a step that does not land strictly
// inside, or a non-positive F', becomes a bisection, unless the step leaves
// the iterate unchanged.
__device__ __forceinline__ double local_solve(const Law &L, double a, double beta, double c,
                                              double f, double x0)
{
    double lo, hi;
    if (L.model == kLinear) {
        lo = -INFINITY;
        hi = INFINITY;
    } else {
        lo = (f - a * L.ts - beta) / c;
        hi = (f - a * L.tr) / c;
        double pad = 1e-12 * (fabs(lo) + fabs(hi));
        lo -= pad;
        hi += pad;
    }
    double x = x0;
    for (int k = 0; k < L.newton; ++k) {
        ThetaEval t = theta_eval(L, x);
        double F = a * t.th + c * x - f;
        double dF = a * t.dth + c;
        if (L.sink == kSinkFeddes) {
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
        double xn = x - F / dF;
        bool bisect = !(dF > 0.0) || (xn != x && !(xn > lo && xn < hi));
        x = bisect ? 0.5 * (lo + hi) : xn;
    }
    return x;
}

// Node kinds from indices (no node-type array): Dirichlet if on a Dirichlet
// face or on the patch; value = patch value, else the highest-numbered
// Dirichlet face holding the node.
__device__ __forceinline__ bool dirichlet_at(const Geo &g, int i, int j, int k, double *val)
{
    int c[3] = {i, j, k};
    bool dir = false;
    double v = 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (l >= g.dim) break;
        if (c[l] == 0 && g.bc[2 * l] == kBcDirichlet) { dir = true; v = g.bcval[2 * l]; }
        if (c[l] == g.n[l] - 1 && g.bc[2 * l + 1] == kBcDirichlet) { dir = true; v = g.bcval[2 * l + 1]; }
    }
    if (g.pface >= 0) {
        int ax = g.pface >> 1;
        int at = (g.pface & 1) ? g.n[ax] - 1 : 0;
        if (c[ax] == at) {
            bool in = true;
            int t = 0;
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                if (l >= g.dim) break;
                if (l == ax) continue;
                if (c[l] < g.plo[t] || c[l] > g.phi[t]) in = false;
                ++t;
            }
            if (in) { dir = true; v = g.pval; }
        }
    }
    if (val) *val = v;
    return dir;
}

}  // namespace rs
