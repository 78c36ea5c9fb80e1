// Per-node FP32 operations of the correction equation
// N(psi_b + delta) - N(psi_b) = r (see soil_mp.h), shared by the single-grid
// mixed-precision kernels and the batched serving kernels.
#pragma once

#include "rs_internal.h"
#include "soil_device.h"
#include "grid_device.h"
#include "soil_mp.h"

namespace rs {

template <int DIM>
__device__ __forceinline__ int vert_index(int i, int j, int k)
{
    return (DIM == 1) ? i : (DIM == 2 ? j : k);
}

// The scalars of one unknown's correction problem: c = xi + kappa + m_ii, the
// right-hand side f (rhs plus the neighbour couplings plus kappa delta_i) and
// the root density.  cf: the stencil coefficients in FP32.  REMARK = false:
// the caller has excluded the Remark's kappa rule.
struct PointEq32 {
    float c, f, bz;
};

template <bool SINK, int DIM, bool REMARK = true>
__device__ __forceinline__ PointEq32 ngs_reduce32(const Geo &g, const Law32 &L, const double *beta,
                                                  float lambdaU, const float *cf, float Ki,
                                                  const float *Kn, const float *dn, float f,
                                                  float d0, int i, int j, int k, int colour)
{
    float mii = 0.0f;
#pragma unroll
    for (int q = 0; q < 2 * DIM; ++q) {
        const float m = cf[q] * (Ki + Kn[q]);
        mii += m;
        f += m * dn[q];
    }
    float kap;
    if (L.kappa_rule == kKappaConst) {
        kap = L.kappa;
    } else if (!REMARK || L.kappa_rule == kKappaRel) {
        kap = L.kappa * mii;
    } else if (colour == 0) {
        float usum = 0.0f;
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q) {
            int d[3] = {i, j, k};
            d[q >> 1] += (q & 1) ? 1 : -1;
            if (cf[q] != 0.0f && !dirichlet_at(g, d[0], d[1], d[2], nullptr))
                usum += cf[q] * (Ki + Kn[q]);
        }
        kap = lambdaU - usum;
    } else {
        kap = lambdaU;
    }
    PointEq32 e;
    e.f = f + kap * d0;
    e.c = L.xi + kap + mii;
    e.bz = SINK ? (float)beta[vert_index<DIM>(i, j, k)] : 0.0f;
    return e;
}

template <int MODEL, bool SINK>
__device__ __forceinline__ float ngs_solve32(const Law32 &L, float a, const PointEq32 &e, float d0,
                                             float pbi)
{
    const Base b = base_of<MODEL>(L, pbi);
    return local_solve32<MODEL, SINK>(L, a, e.bz, e.c, e.f, b, d0);
}

// New delta of unknown (i, j, k) from gathered values: the stencil, K*_i, the
// right-hand side f = rhs_i, the old delta d0, the base state pb, and the K*
// and current delta of the 2 DIM neighbours.
template <int MODEL, bool SINK, int DIM>
__device__ __forceinline__ float ngs_point32(const Geo &g, const Law32 &L, float a,
                                             const double *beta, float lambdaU,
                                             const Stencil<DIM> &st, float Ki, const float *Kn,
                                             const float *dn, float f, float d0, float pbi, int i,
                                             int j, int k, int colour)
{
    float cf[2 * DIM];
#pragma unroll
    for (int q = 0; q < 2 * DIM; ++q) cf[q] = (float)st.cf[q];
    const PointEq32 e =
        ngs_reduce32<SINK, DIM>(g, L, beta, lambdaU, cf, Ki, Kn, dn, f, d0, i, j, k, colour);
    return ngs_solve32<MODEL, SINK>(L, a, e, d0, pbi);
}

// New delta at unknown (i, j, k): f = rhs + sum_j m_ij delta_j + kappa delta_i,
// c = xi + kappa + m_ii, then the scalar correction solve; true unless the
// stored delta moved by at most 4 FP32 ulp (FP32 rounding keeps a converged
// nonlinear update from settling bitwise).  XPAD: the arrays
// have finite padding around them (see stencil()).  SPLIT: the level has
// parity-split rows and padded arrays; the axis-0 neighbours are loaded as
// one pair from xl (idx and xl < 0: computed here).
template <int MODEL, bool SINK, int DIM, bool XPAD = false, bool SPLIT = false>
__device__ __forceinline__ bool ngs_cell32(const Geo &g, const Law32 &L, float a,
                                           const double *beta, float lambdaU, const float *K,
                                           const float *rhs, const float *pb, float *dl, int i,
                                           int j, int k, int colour, long long idx = -1,
                                           long long xl = -1)
{
    if (idx < 0) idx = lin(g, i, j, k);
    Stencil<DIM> st;
    float Kn[2 * DIM], dn[2 * DIM];
    if constexpr (SPLIT) {
        if (xl < 0) xl = xnb(g, i, idx, -1);
        st = stencil_split<DIM>(g, i, j, k, idx, xl);
        const float2_u kx = load_pair(K + xl), dx = load_pair(dl + xl);
        Kn[0] = kx.x;
        Kn[1] = kx.y;
        dn[0] = dx.x;
        dn[1] = dx.y;
#pragma unroll
        for (int q = 2; q < 2 * DIM; ++q) {
            Kn[q] = K[st.jn[q]];
            dn[q] = dl[st.jn[q]];
        }
    } else {
        st = stencil<DIM, XPAD>(g, i, j, k, idx);
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q) {
            Kn[q] = K[st.jn[q]];
            dn[q] = dl[st.jn[q]];
        }
    }
    const float d0 = dl[idx];
    const float d1 = ngs_point32<MODEL, SINK, DIM>(g, L, a, beta, lambdaU, st, K[idx], Kn, dn,
                                                   rhs[idx], d0, pb[idx], i, j, k, colour);
    dl[idx] = d1;
    return !(fabsf(d1 - d0) <= 4.0f * 1.1920929e-7f * fabsf(d1));
}

// N_delta(delta)_i = a dtheta + beta da + xi delta_i + sum_j m_ij (delta_i - delta_j)
template <int MODEL, bool SINK, int DIM, bool XPAD = false>
__device__ __forceinline__ float apply_Nd(const Geo &g, const Law32 &L, float a,
                                          const double *beta, const float *K, const float *pb,
                                          const float *dl, int i, int j, int k, long long idx)
{
    const Stencil<DIM> st = stencil<DIM, XPAD>(g, i, j, k, idx);
    const float x = dl[idx];
    const float Ki = K[idx];
    const float p = pb[idx];
    float Kn[2 * DIM], dn[2 * DIM];
#pragma unroll
    for (int q = 0; q < 2 * DIM; ++q) {
        Kn[q] = K[st.jn[q]];
        dn[q] = dl[st.jn[q]];
    }
    const float bz = SINK ? (float)beta[vert_index<DIM>(i, j, k)] : 0.0f;
    const Base b = base_of<MODEL>(L, p);
    float dth, slope;
    dtheta32<MODEL>(L, b, x, dth, slope);
    float s = a * dth;
    if (SINK) {
        float da, ds;
        dfeddes32(L, b.psi, x, da, ds);
        s += bz * da;
    }
    float md = 0.0f;
#pragma unroll
    for (int q = 0; q < 2 * DIM; ++q) md += (float)st.cf[q] * (Ki + Kn[q]) * (x - dn[q]);
    return s + (L.xi * x + md);
}

}  // namespace rs
