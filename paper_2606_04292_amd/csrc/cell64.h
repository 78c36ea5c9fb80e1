// Per-node FP64 quantities of the step system, shared by the single-grid
// kernels and the batched serving kernels: lagged conductivity K*, right-hand
// side g and the operator N (eq. Nh-def with the BDF2 history of the time
// discretisation).
#pragma once

#include "rs_internal.h"
#include "soil_device.h"
#include "grid_device.h"

namespace rs {

// K*_i = Ks_i K_r(psi*_i), psi* the lagged state (psi^n, or 2 psi^n - psi^{n-1}
// with the extrapolated BDF2 lag; the boundary value at Dirichlet nodes).
// *psi0 receives the first iterate of the step (psi^n, or the boundary value).
__device__ __forceinline__ double kstar_at(const Geo &g, const Law &L, const Step &st,
                                           const double *psi_n, const double *psi_nm1, double ks,
                                           int i, int j, int k, long long idx, double *psi0)
{
    double bv;
    double ps;
    bool from_state;
    if (dirichlet_at(g, i, j, k, &bv, &from_state)) {
        if (from_state) bv = psi_n[idx];
        ps = bv;
        *psi0 = bv;
    } else {
        double pn = psi_n[idx];
        ps = (st.order == 2 && st.lag_extrap) ? 2.0 * pn - psi_nm1[idx] : pn;
        *psi0 = pn;
    }
    if (L.soils) {
        // layered media: the node's own soil, with that soil's Ks
        const Law &Ls = L.soils[g.soil[idx]];
        return Ls.Ks * krel(Ls, ps);
    }
    return ks * krel(L, ps);
}

// g_i = H_i + xi psi*_i - (M z)_i - free-drainage outflow (0 at Dirichlet nodes);
// H = theta(psi^n)/dt (BDF1) or (4 theta(psi^n) - theta(psi^{n-1}))/(2 dt) (BDF2).
__device__ __forceinline__ double g_at(const Geo &g, const Law &L, const Step &st,
                                       const double *psi_n, const double *psi_nm1, const double *K,
                                       int i, int j, int k, long long idx)
{
    if (dirichlet_at(g, i, j, k, nullptr)) return 0.0;
    int c[3] = {i, j, k};
    double pn = psi_n[idx];
    double H, ps;
    const double pm = st.order == 1 ? pn : psi_nm1[idx];
    // history term with the node's soil (layered media) or the one law
    auto history = [&](const Law &Lt) {
        return st.order == 1 ? theta_only(Lt, pn) / st.dt
                             : (4.0 * theta_only(Lt, pn) - theta_only(Lt, pm)) / (2.0 * st.dt);
    };
    H = L.soils ? history(L.soils[g.soil[idx]]) : history(L);
    ps = (st.order == 2 && st.lag_extrap) ? 2.0 * pn - pm : pn;
    // gravity (M z)_i: only faces along the vertical axis, z_i - z_j = -side h
    double Ki = K[idx];
    double mz = 0.0;
    const int v = g.vert;
    for_each_nb(g, c, idx, [&](long long jn, double cf, int l, int side) {
        if (l == v) mz += cf * (Ki + K[jn]) * (-side * g.h[v]);
    });
    double gi = H + L.xi * ps - mz;
    if (c[v] == 0 && g.bc[2 * v] == kBcFreedrain) {
        double iw = 2.0;   // bottom node: half control volume
        gi -= Ki * iw / g.h[v];
    }
    return gi;
}

// N(psi)_i = a theta(psi_i) + beta a_F(psi_i) + xi psi_i + (M psi)_i
// (the whole stencil is loaded before the law is evaluated, so that the loads
// overlap the theta chain instead of following it; XPAD as for stencil()).
// With scale set, *scale also receives the sum of the magnitudes of the terms
// (a |theta|, the sink, xi |psi_i|, m_ij (|psi_i| + |psi_j|) per face): the
// size of the rounding floor of the defect at this node.
template <int MODEL, bool SINK, int DIM, bool XPAD = false>
__device__ __forceinline__ double apply_N_t(const Geo &g, const Law &L, double a,
                                            const double *beta, const double *K,
                                            const double *psi, int i, int j, int k, long long idx,
                                            double *scale = nullptr)
{
    const Stencil<DIM> st = stencil<DIM, XPAD>(g, i, j, k, idx);
    const double x = psi[idx];
    const double Ki = K[idx];
    double Kn[2 * DIM], pn[2 * DIM];
#pragma unroll
    for (int q = 0; q < 2 * DIM; ++q) {
        Kn[q] = K[st.jn[q]];
        pn[q] = psi[st.jn[q]];
    }
    double bz = 0.0;
    if (SINK) bz = beta[(DIM == 1) ? i : (DIM == 2 ? j : k)];
    double s;
    if constexpr (MODEL == kMulti) s = a * theta_only(L.soils[g.soil[idx]], x);
    else s = a * theta_only_t<MODEL>(L, x);
    if (SINK) {
        double fa, dfa;
        feddes(L, x, fa, dfa);
        s += bz * fa;
    }
    double mpsi = 0.0;
#pragma unroll
    for (int q = 0; q < 2 * DIM; ++q) mpsi += st.cf[q] * (Ki + Kn[q]) * (x - pn[q]);
    if (scale) {
        double t = fabs(s) + fabs(L.xi * x);
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q) t += fabs(st.cf[q] * (Ki + Kn[q])) * (fabs(x) + fabs(pn[q]));
        *scale = t;
    }
    return s + (L.xi * x + mpsi);
}

}  // namespace rs
