// Grid transfers of the FAS cycle (section 3.2 steps 3 and 6), for FP64 and
// FP32 level data.
#pragma once

#include "rs_internal.h"
#include "soil_device.h"
#include "grid_device.h"

namespace rs {

// psibar_H = FW(psi_h), d_H = FW(d_h) stored in g_H (Dirichlet coarse nodes:
// injection of psi, zero defect).  FW: tensor (1/4, 1/2, 1/4) around fine node
// 2I, missing neighbours mirrored at the domain boundary.
template <typename T>
__device__ __forceinline__ void restrict_at(const Geo &gc, const Geo &gf, const T *psi_f,
                                            const T *d_f, T *psibar_c, T *g_c, int I0, int I1,
                                            int I2)
{
    long long I = I0 + (long long)I1 * gc.stride[1] + (long long)I2 * gc.stride[2];
    int F[3] = {2 * I0, 2 * I1, 2 * I2};
    if (dirichlet_at(gc, I0, I1, I2, nullptr)) {
        psibar_c[I] = psi_f[F[0] + (long long)F[1] * gf.stride[1] + (long long)F[2] * gf.stride[2]];
        g_c[I] = T(0);
        return;
    }
    int lo[3], hi[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        lo[l] = (l < gf.dim) ? -1 : 0;
        hi[l] = (l < gf.dim) ? 1 : 0;
    }
    T sp = T(0), sd = T(0);
    for (int o2 = lo[2]; o2 <= hi[2]; ++o2) {
        int f2 = F[2] + o2;
        f2 = f2 < 0 ? -f2 : (f2 > gf.n[2] - 1 ? 2 * (gf.n[2] - 1) - f2 : f2);
        T w2 = (gf.dim > 2) ? (o2 == 0 ? T(0.5) : T(0.25)) : T(1);
        for (int o1 = lo[1]; o1 <= hi[1]; ++o1) {
            int f1 = F[1] + o1;
            f1 = f1 < 0 ? -f1 : (f1 > gf.n[1] - 1 ? 2 * (gf.n[1] - 1) - f1 : f1);
            T w1 = (gf.dim > 1) ? (o1 == 0 ? T(0.5) : T(0.25)) : T(1);
            for (int o0 = -1; o0 <= 1; ++o0) {
                int f0 = F[0] + o0;
                f0 = f0 < 0 ? -f0 : (f0 > gf.n[0] - 1 ? 2 * (gf.n[0] - 1) - f0 : f0);
                T w = (o0 == 0 ? T(0.5) : T(0.25)) * w1 * w2;
                long long fi = f0 + (long long)f1 * gf.stride[1] + (long long)f2 * gf.stride[2];
                sp += w * psi_f[fi];
                sd += w * d_f[fi];
            }
        }
    }
    psibar_c[I] = sp;
    g_c[I] = sd;
}

template <typename T>
__global__ __launch_bounds__(256) void k_restrict(Geo gc, Geo gf, const T *psi_f, const T *d_f,
                                                  T *psibar_c, T *g_c)
{
    int I0 = blockIdx.x * kBX + threadIdx.x;
    int I1 = blockIdx.y * kBY + threadIdx.y;
    int I2 = blockIdx.z;
    if (I0 >= gc.n[0] || I1 >= gc.n[1]) return;
    restrict_at<T>(gc, gf, psi_f, d_f, psibar_c, g_c, I0, I1, I2);
}

// psi_h += I_h^H (psi_H - psibar_H) at fine unknowns (tensor linear
// interpolation: even index -> coarse node, odd -> mean of the two).
template <typename T>
__device__ __forceinline__ void prolong_at(const Geo &gf, const Geo &gc, const T *psi_c,
                                           const T *psibar_c, T *psi_f, int i, int j, int k)
{
    if (dirichlet_at(gf, i, j, k, nullptr)) return;
    int c[3] = {i, j, k};
    int a0[3], a1[3], cnt[3];
    T wt[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        if (c[l] & 1) {
            a0[l] = (c[l] - 1) >> 1;
            a1[l] = (c[l] + 1) >> 1;
            cnt[l] = 2;
            wt[l] = T(0.5);
        } else {
            a0[l] = a1[l] = c[l] >> 1;
            cnt[l] = 1;
            wt[l] = T(1);
        }
    }
    T e = T(0);
    for (int q2 = 0; q2 < cnt[2]; ++q2)
        for (int q1 = 0; q1 < cnt[1]; ++q1)
            for (int q0 = 0; q0 < cnt[0]; ++q0) {
                long long J = (q0 ? a1[0] : a0[0]) + (long long)(q1 ? a1[1] : a0[1]) * gc.stride[1] +
                              (long long)(q2 ? a1[2] : a0[2]) * gc.stride[2];
                e += wt[0] * wt[1] * wt[2] * (psi_c[J] - psibar_c[J]);
            }
    long long idx = i + (long long)j * gf.stride[1] + (long long)k * gf.stride[2];
    psi_f[idx] += e;
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong(Geo gf, Geo gc, const T *psi_c, const T *psibar_c,
                                                 T *psi_f)
{
    int i = blockIdx.x * kBX + threadIdx.x;
    int j = blockIdx.y * kBY + threadIdx.y;
    int k = blockIdx.z;
    if (i >= gf.n[0] || j >= gf.n[1]) return;
    prolong_at<T>(gf, gc, psi_c, psibar_c, psi_f, i, j, k);
}

// Injection to a coarse level: v_H[I] = v_h[2I].
template <typename T>
__global__ __launch_bounds__(256) void k_inject_t(Geo gc, Geo gf, const T *vf, T *vc)
{
    int i = blockIdx.x * kBX + threadIdx.x;
    int j = blockIdx.y * kBY + threadIdx.y;
    int k = blockIdx.z;
    if (i >= gc.n[0] || j >= gc.n[1]) return;
    long long I = i + (long long)j * gc.stride[1] + (long long)k * gc.stride[2];
    long long F = 2LL * i + 2LL * j * gf.stride[1] + 2LL * k * gf.stride[2];
    vc[I] = vf[F];
}

}  // namespace rs
