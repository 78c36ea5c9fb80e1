// Grid transfers of the FAS cycle (section 3.2 steps 3 and 6), for FP64 and
// FP32 level data.
#pragma once

#include <stdlib.h>
#include <string.h>

#include "rs_internal.h"
#include "soil_device.h"
#include "grid_device.h"

namespace rs {

// Fine offsets of the three full-weighting taps of fine node F along every
// axis (mirrored at both ends; axis 0 by row position).
__device__ __forceinline__ void fw_offsets(const Geo &gf, const int F[3], long long off[3][3])
{
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const int n = gf.n[l];
        const int m = F[l] == 0 ? 1 : F[l] - 1;
        const int p = F[l] == n - 1 ? n - 2 : F[l] + 1;
        if (l == 0) {
            off[0][0] = xpos(gf, m);
            off[0][1] = xpos(gf, F[0]);
            off[0][2] = xpos(gf, p);
        } else {
            const long long st = gf.stride[l];
            off[l][0] = (long long)m * st;
            off[l][1] = (long long)F[l] * st;
            off[l][2] = (long long)p * st;
        }
    }
}

// psibar_H = FW(psi_h), d_H = FW(d_h) stored in g_H (Dirichlet coarse nodes:
// injection of psi, zero defect).  FW: tensor (1/4, 1/2, 1/4) around fine node
// 2I, missing neighbours mirrored at the domain boundary.  The taps are summed
// axis 2 outermost, axis 0 innermost, with weight (w0 w1) w2.  XPAD (arrays
// with finite padding around them, as in a grid workspace): the three axis-0
// taps are loaded as the row's nodes 2I0-1 .. 2I0+1 without a bound check and
// mirrored in registers; the sums are the same.
template <int DIM, typename T, bool XPAD = false>
__device__ __forceinline__ void restrict_at(const Geo &gc, const Geo &gf, const T *psi_f,
                                            const T *d_f, T *psibar_c, T *g_c, int I0, int I1,
                                            int I2)
{
    const long long I = lin(gc, I0, I1, I2);
    const int F[3] = {2 * I0, 2 * I1, 2 * I2};
    if (dirichlet_t<DIM>(gc, I0, I1, I2)) {
        psibar_c[I] = psi_f[lin(gf, F[0], F[1], F[2])];
        g_c[I] = T(0);
        return;
    }
    long long off[3][3];
    fw_offsets(gf, F, off);
    const long long x3[3] = {xpos(gf, F[0] - 1), xpos(gf, F[0]), xpos(gf, F[0] + 1)};
    const T wt[3] = {T(0.25), T(0.5), T(0.25)};
    T sp = T(0), sd = T(0);
#pragma unroll
    for (int o2 = 0; o2 < (DIM > 2 ? 3 : 1); ++o2) {
        const T w2 = DIM > 2 ? wt[o2] : T(1);
        const long long b2 = DIM > 2 ? off[2][o2] : 0;
#pragma unroll
        for (int o1 = 0; o1 < (DIM > 1 ? 3 : 1); ++o1) {
            const T w1 = DIM > 1 ? wt[o1] : T(1);
            const long long b1 = b2 + (DIM > 1 ? off[1][o1] : 0);
            if constexpr (XPAD) {
                const T pl = psi_f[b1 + x3[0]], pc = psi_f[b1 + x3[1]], pr = psi_f[b1 + x3[2]];
                const T dl = d_f[b1 + x3[0]], dc = d_f[b1 + x3[1]], dr = d_f[b1 + x3[2]];
                const bool first = F[0] == 0, last = F[0] == gf.n[0] - 1;
                const T P3[3] = {first ? pr : pl, pc, last ? pl : pr};
                const T D3[3] = {first ? dr : dl, dc, last ? dl : dr};
#pragma unroll
                for (int o0 = 0; o0 < 3; ++o0) {
                    const T w = wt[o0] * w1 * w2;
                    sp += w * P3[o0];
                    sd += w * D3[o0];
                }
            } else {
#pragma unroll
                for (int o0 = 0; o0 < 3; ++o0) {
                    const T w = wt[o0] * w1 * w2;
                    const long long fi = b1 + off[0][o0];
                    sp += w * psi_f[fi];
                    sd += w * d_f[fi];
                }
            }
        }
    }
    psibar_c[I] = sp;
    g_c[I] = sd;
}

// Full weighting of v at coarse node (I0, I1, I2): the tensor (1/4, 1/2, 1/4)
// around fine node 2I with missing neighbours mirrored at the ends, summed in
// the order of restrict_at.
template <int DIM, typename T>
__device__ __forceinline__ T fw_value(const Geo &gf, const T *v, int I0, int I1, int I2)
{
    const int F[3] = {2 * I0, 2 * I1, 2 * I2};
    long long off[3][3];
    fw_offsets(gf, F, off);
    const T wt[3] = {T(0.25), T(0.5), T(0.25)};
    T s = T(0);
#pragma unroll
    for (int o2 = 0; o2 < (DIM > 2 ? 3 : 1); ++o2) {
        const T w2 = DIM > 2 ? wt[o2] : T(1);
        const long long b2 = DIM > 2 ? off[2][o2] : 0;
#pragma unroll
        for (int o1 = 0; o1 < (DIM > 1 ? 3 : 1); ++o1) {
            const T w1 = DIM > 1 ? wt[o1] : T(1);
            const long long b1 = b2 + (DIM > 1 ? off[1][o1] : 0);
#pragma unroll
            for (int o0 = 0; o0 < 3; ++o0) s += wt[o0] * w1 * w2 * v[b1 + off[0][o0]];
        }
    }
    return s;
}

// psi_h += I_h^H (psi_H - psibar_H) at fine unknowns (tensor linear
// interpolation: even index -> coarse node, odd -> mean of the two).  Two taps
// per axis, the second with weight 0 at an even index, so the sum has no
// branch and equals the sum over the contributing coarse nodes.
template <int DIM, typename T>
__device__ __forceinline__ void prolong_at(const Geo &gf, const Geo &gc, const T *psi_c,
                                           const T *psibar_c, T *psi_f, int i, int j, int k)
{
    if (dirichlet_t<DIM>(gf, i, j, k)) return;
    const int c[3] = {i, j, k};
    long long off[3][2];
    T wt[3][2];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const bool odd = c[l] & 1;
        off[l][0] = l == 0 ? xpos(gc, c[0] >> 1) : (long long)(c[l] >> 1) * gc.stride[l];
        off[l][1] = l == 0 ? xpos(gc, (c[0] + 1) >> 1) : (long long)((c[l] + 1) >> 1) * gc.stride[l];
        wt[l][0] = odd ? T(0.5) : T(1);
        wt[l][1] = odd ? T(0.5) : T(0);
    }
    T e = T(0);
#pragma unroll
    for (int q2 = 0; q2 < (DIM > 2 ? 2 : 1); ++q2) {
        const T w2 = DIM > 2 ? wt[2][q2] : T(1);
        const long long b2 = DIM > 2 ? off[2][q2] : 0;
#pragma unroll
        for (int q1 = 0; q1 < (DIM > 1 ? 2 : 1); ++q1) {
            const T w1 = DIM > 1 ? wt[1][q1] : T(1);
            const long long b1 = b2 + (DIM > 1 ? off[1][q1] : 0);
#pragma unroll
            for (int q0 = 0; q0 < 2; ++q0) {
                const long long J = b1 + off[0][q0];
                e += wt[0][q0] * w1 * w2 * (psi_c[J] - psibar_c[J]);
            }
        }
    }
    psi_f[lin(gf, i, j, k)] += e;
}

// One coarse node per thread (restriction) / one fine node per thread
// (prolongation), work-groups numbered per XCD.
template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_restrict(Geo gc, Geo gf, const T *psi_f, const T *d_f,
                                                  T *psibar_c, T *g_c, NodeMap nm)
{
    const unsigned long long t =
        (unsigned long long)xcd_block(gridDim.x / 8u) * blockDim.x + threadIdx.x;
    if (t >= (unsigned long long)gc.N) return;
    int i, j, k;
    node_ijk(nm, t, i, j, k);
    restrict_at<DIM, T, true>(gc, gf, psi_f, d_f, psibar_c, g_c, i, j, k);   // workspace arrays are padded
}

// Prolongation by coarse cell: the thread of coarse node I loads psi_H - psibar_H
// on the 2^DIM corners I + {0,1}^DIM once and updates the fine nodes 2I + {0,1}^DIM
// (those inside the grid), each with the sum of prolong_at in the same order.
// FULL: interpolate psi_H itself and assign it (the FMG interpolation;
// psibar_c unused).  The arrays are padded workspace arrays: the two axis-0
// corners and the two axis-0 fine nodes are loaded without a bound check (a
// value past the end of a row has weight 0 or is not stored).
template <int DIM, typename T, bool FULL = false>
__global__ __launch_bounds__(256) void k_prolong(Geo gf, Geo gc, const T *psi_c, const T *psibar_c,
                                                 T *psi_f, NodeMap nmc)
{
    const unsigned long long t =
        (unsigned long long)xcd_block(gridDim.x / 8u) * blockDim.x + threadIdx.x;
    if (t >= (unsigned long long)gc.N) return;
    int Ic[3];
    node_ijk(nmc, t, Ic[0], Ic[1], Ic[2]);
    const long long cx[2] = {xpos(gc, Ic[0]), xpos(gc, Ic[0] + 1)};
    const long long fx[2] = {xpos(gf, 2 * Ic[0]), xpos(gf, 2 * Ic[0] + 1)};
    // corner offsets along axes 1 and 2 (the upper corner clamped at the last
    // coarse node: its weight is 0 there or the fine node lies outside the
    // grid); along axis 0 the pair I0, I0 + 1 is loaded as it is
    long long co[3][2];
#pragma unroll
    for (int l = 1; l < 3; ++l) {
        const int lo = Ic[l];
        const int hi = lo + 1 < gc.n[l] ? lo + 1 : lo;
        co[l][0] = (long long)lo * gc.stride[l];
        co[l][1] = (long long)hi * gc.stride[l];
    }
    constexpr int N2 = DIM > 2 ? 2 : 1, N1 = DIM > 1 ? 2 : 1;
    T E[N2][N1][2];
#pragma unroll
    for (int q2 = 0; q2 < N2; ++q2)
#pragma unroll
        for (int q1 = 0; q1 < N1; ++q1)
        {
            const long long J = (DIM > 2 ? co[2][q2] : 0) + (DIM > 1 ? co[1][q1] : 0);
            const T c0 = psi_c[J + cx[0]], c1 = psi_c[J + cx[1]];
            E[q2][q1][0] = FULL ? c0 : c0 - psibar_c[J + cx[0]];
            E[q2][q1][1] = FULL ? c1 : c1 - psibar_c[J + cx[1]];
        }
#pragma unroll
    for (int a2 = 0; a2 < N2; ++a2) {
        const int f2 = 2 * Ic[2] + a2;
        if (f2 >= gf.n[2]) continue;
#pragma unroll
        for (int a1 = 0; a1 < N1; ++a1) {
            const int f1 = 2 * Ic[1] + a1;
            if (f1 >= gf.n[1]) continue;
            const long long fr = (long long)f1 * gf.stride[1] + (long long)f2 * gf.stride[2];
            T old[2] = {T(0), T(0)};
            if (!FULL) {
                old[0] = psi_f[fr + fx[0]];
                old[1] = psi_f[fr + fx[1]];
            }
#pragma unroll
            for (int a0 = 0; a0 < 2; ++a0) {
                const int f0 = 2 * Ic[0] + a0;
                if (f0 >= gf.n[0]) continue;
                if (dirichlet_t<DIM>(gf, f0, f1, f2)) continue;
                // weights of the two taps along an axis: even fine index (1, 0),
                // odd (1/2, 1/2)
                const T w0[2] = {a0 ? T(0.5) : T(1), a0 ? T(0.5) : T(0)};
                const T w1[2] = {a1 ? T(0.5) : T(1), a1 ? T(0.5) : T(0)};
                const T w2[2] = {a2 ? T(0.5) : T(1), a2 ? T(0.5) : T(0)};
                T e = T(0);
#pragma unroll
                for (int q2 = 0; q2 < N2; ++q2)
#pragma unroll
                    for (int q1 = 0; q1 < N1; ++q1)
#pragma unroll
                        for (int q0 = 0; q0 < 2; ++q0)
                            e += w0[q0] * (DIM > 1 ? w1[q1] : T(1)) * (DIM > 2 ? w2[q2] : T(1)) *
                                 E[q2][q1][q0];
                psi_f[fr + fx[a0]] = FULL ? e : old[a0] + e;
            }
        }
    }
}

// Levels with parity-split rows (Geo::xs = 1 on both levels): one thread per
// coarse pair (2m, 2m + 1) of a row.  Their fine centres 4m and 4m + 2 are
// the even positions 2m, 2m + 1 of a fine row, their odd taps 4m - 1 .. 4m + 3
// the odd positions 2m - 1 .. 2m + 1: per fine row a pair, a pair and a single
// load per array.  Each coarse node's sum is that of restrict_at.  Slots:
// xh of the coarse level per row.
template <int DIM, typename T>
__global__ __launch_bounds__(256) void k_restrict_pair(Geo gc, Geo gf, const T *psi_f,
                                                       const T *d_f, T *psibar_c, T *g_c,
                                                       ColourMap cm)
{
    const unsigned long long t =
        (unsigned long long)xcd_block(gridDim.x / 8u) * blockDim.x + threadIdx.x;
    if (t >= cm.total) return;
    const unsigned row = udiv((unsigned)t, cm.dH);
    const int m = (int)((unsigned)(t - (unsigned long long)row * cm.H));
    int J1 = 0, J2 = 0;
    if (DIM == 3) {
        J2 = (int)udiv(row, cm.dN1);
        J1 = (int)row - J2 * (int)cm.n1;
    } else if (DIM == 2) {
        J1 = (int)row;
    }
    const bool has_b = 2 * m + 1 < gc.n[0];
    const int F1 = 2 * J1, F2 = 2 * J2;
    // fine row offsets of the taps along axes 1 and 2 (mirrored at the ends)
    long long ro[3][3];
#pragma unroll
    for (int l = 1; l < 3; ++l) {
        const int F = l == 1 ? F1 : F2;
        const int n = gf.n[l];
        const int lo = F == 0 ? 1 : F - 1, hi = F == n - 1 ? n - 2 : F + 1;
        const long long st = gf.stride[l];
        ro[l][0] = (long long)lo * st;
        ro[l][1] = (long long)F * st;
        ro[l][2] = (long long)hi * st;
    }
    const long long ce = 2 * m, od = gf.xh + 2 * m - 1;   // even pair, odd window
    const T wt[3] = {T(0.25), T(0.5), T(0.25)};
    T sp[2] = {T(0), T(0)}, sd[2] = {T(0), T(0)};
    T pin[2] = {T(0), T(0)};   // fine values at the centres of the middle row
    // all rows of taps in flight together (one plane at a time was slower:
    // 102 against 71 us for the FP64 restriction at 129^3)
#pragma unroll
    for (int o2 = 0; o2 < (DIM > 2 ? 3 : 1); ++o2) {
        const T w2 = DIM > 2 ? wt[o2] : T(1);
        const long long b2 = DIM > 2 ? ro[2][o2] : 0;
#pragma unroll
        for (int o1 = 0; o1 < (DIM > 1 ? 3 : 1); ++o1) {
            const T w1 = DIM > 1 ? wt[o1] : T(1);
            const long long b1 = b2 + (DIM > 1 ? ro[1][o1] : 0);
            const auto pc = load_pair(psi_f + b1 + ce), dc = load_pair(d_f + b1 + ce);
            const auto po = load_pair(psi_f + b1 + od), dq = load_pair(d_f + b1 + od);
            const T po2 = psi_f[b1 + od + 2], dq2 = d_f[b1 + od + 2];
            if ((DIM < 3 || o2 == 1) && (DIM < 2 || o1 == 1)) {
                pin[0] = pc.x;
                pin[1] = pc.y;
            }
            // node a: taps 4m - 1, 4m, 4m + 1; node b: 4m + 1, 4m + 2, 4m + 3
            const T pl[2] = {po.x, po.y}, pr[2] = {po.y, po2};
            const T dl[2] = {dq.x, dq.y}, dr[2] = {dq.y, dq2};
            const T pm[2] = {pc.x, pc.y}, dm[2] = {dc.x, dc.y};
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int F0 = 4 * m + 2 * a;
                const bool first = F0 == 0, last = F0 == gf.n[0] - 1;
                const T P3[3] = {first ? pr[a] : pl[a], pm[a], last ? pl[a] : pr[a]};
                const T D3[3] = {first ? dr[a] : dl[a], dm[a], last ? dl[a] : dr[a]};
#pragma unroll
                for (int o0 = 0; o0 < 3; ++o0) {
                    const T w = wt[o0] * w1 * w2;
                    sp[a] += w * P3[o0];
                    sd[a] += w * D3[o0];
                }
            }
        }
    }
    const long long rc = (long long)J1 * gc.stride[1] + (long long)J2 * gc.stride[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        if (a == 1 && !has_b) break;
        const int I0 = 2 * m + a;
        const long long I = rc + (a ? gc.xh + m : m);
        if (dirichlet_t<DIM>(gc, I0, J1, J2)) {
            psibar_c[I] = pin[a];
            g_c[I] = T(0);
        } else {
            psibar_c[I] = sp[a];
            g_c[I] = sd[a];
        }
    }
}

// Prolongation on levels with parity-split rows: one thread per coarse pair
// slot m of a row.  Its coarse corners 2m, 2m + 1, 2m + 2 along axis 0 are the
// even positions m, m + 1 (a pair) and the odd position m; the fine nodes
// 4m .. 4m + 3 it updates are the even positions 2m, 2m + 1 and the odd
// positions 2m, 2m + 1 (a pair each).  Fine node 4m + 2a + b takes the taps
// (2m + a, 2m + a + 1) with weights (1, 0) for b = 0 and (1/2, 1/2) for b = 1,
// as in k_prolong, summed in the same order.  A pair is stored as a pair only
// when both of its nodes lie in the row (a Dirichlet node of it gets its own
// value back: no other thread writes it).
template <int DIM, typename T, bool FULL = false>
__global__ __launch_bounds__(256) void k_prolong_pair(Geo gf, Geo gc, const T *psi_c,
                                                      const T *psibar_c, T *psi_f, ColourMap cm)
{
    const unsigned long long t =
        (unsigned long long)xcd_block(gridDim.x / 8u) * blockDim.x + threadIdx.x;
    if (t >= cm.total) return;
    const unsigned row = udiv((unsigned)t, cm.dH);
    const int m = (int)((unsigned)(t - (unsigned long long)row * cm.H));
    int Ic[3] = {0, 0, 0};
    if (DIM == 3) {
        Ic[2] = (int)udiv(row, cm.dN1);
        Ic[1] = (int)row - Ic[2] * (int)cm.n1;
    } else if (DIM == 2) {
        Ic[1] = (int)row;
    }
    long long co[3][2];
#pragma unroll
    for (int l = 1; l < 3; ++l) {
        const int lo = Ic[l];
        const int hi = lo + 1 < gc.n[l] ? lo + 1 : lo;
        co[l][0] = (long long)lo * gc.stride[l];
        co[l][1] = (long long)hi * gc.stride[l];
    }
    constexpr int N2 = DIM > 2 ? 2 : 1, N1 = DIM > 1 ? 2 : 1;
    // E at coarse 2m, 2m + 1, 2m + 2 (the last past the row's end when 2m + 2
    // >= n0: weight 0 or no fine node)
    T E[N2][N1][3];
#pragma unroll
    for (int q2 = 0; q2 < N2; ++q2)
#pragma unroll
        for (int q1 = 0; q1 < N1; ++q1) {
            const long long J = (DIM > 2 ? co[2][q2] : 0) + (DIM > 1 ? co[1][q1] : 0);
            const auto ce = load_pair(psi_c + J + m);
            const T c1 = psi_c[J + gc.xh + m];
            if (FULL) {
                E[q2][q1][0] = ce.x;
                E[q2][q1][1] = c1;
                E[q2][q1][2] = ce.y;
            } else {
                const auto be = load_pair(psibar_c + J + m);
                const T b1 = psibar_c[J + gc.xh + m];
                E[q2][q1][0] = ce.x - be.x;
                E[q2][q1][1] = c1 - b1;
                E[q2][q1][2] = ce.y - be.y;
            }
        }
    const int n0 = gf.n[0];
#pragma unroll
    for (int a2 = 0; a2 < N2; ++a2) {
        const int f2 = 2 * Ic[2] + a2;
        if (f2 >= gf.n[2]) continue;
#pragma unroll
        for (int a1 = 0; a1 < N1; ++a1) {
            const int f1 = 2 * Ic[1] + a1;
            if (f1 >= gf.n[1]) continue;
            const long long fr = (long long)f1 * gf.stride[1] + (long long)f2 * gf.stride[2];
            // fine 4m + 2a + b at position (b ? xh : 0) + 2m + a; the old
            // values are kept at Dirichlet nodes (also under FULL)
            T v[2][2];   // [b][a]
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const auto o = load_pair(psi_f + fr + (b ? gf.xh : 0) + 2 * m);
                v[b][0] = o.x;
                v[b][1] = o.y;
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                bool in[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int f0 = 4 * m + 2 * a + b;
                    in[a] = f0 < n0;
                    if (!in[a] || dirichlet_t<DIM>(gf, f0, f1, f2)) continue;
                    const T w0[2] = {b ? T(0.5) : T(1), b ? T(0.5) : T(0)};
                    const T w1[2] = {a1 ? T(0.5) : T(1), a1 ? T(0.5) : T(0)};
                    const T w2[2] = {a2 ? T(0.5) : T(1), a2 ? T(0.5) : T(0)};
                    T e = T(0);
#pragma unroll
                    for (int q2 = 0; q2 < N2; ++q2)
#pragma unroll
                        for (int q1 = 0; q1 < N1; ++q1)
#pragma unroll
                            for (int q0 = 0; q0 < 2; ++q0)
                                e += w0[q0] * (DIM > 1 ? w1[q1] : T(1)) *
                                     (DIM > 2 ? w2[q2] : T(1)) * E[q2][q1][a + q0];
                    v[b][a] = FULL ? e : v[b][a] + e;
                }
                const long long p = fr + (b ? gf.xh : 0) + 2 * m;
                if (in[1]) {
                    store_pair(psi_f + p, v[b][0], v[b][1]);
                } else if (in[0]) {
                    psi_f[p] = v[b][0];
                }
            }
        }
    }
}

// The pair transfers pay on coarse levels of at least 2^18 nodes (on smaller
// ones, latency-bound, they were slower).  Measured at 129^3, us per launch,
// one node per lane -> pairs: FP64 restriction 86.4 -> 71.4, prolongation
// 72.5 -> 53.8; FP32 62.9 -> 34.0 and 29.6 -> 26.6.  RS_TRANSFER=pair takes
// them on every level with split rows, RS_TRANSFER=single on none.
inline bool pair_transfer(const Geo &gc, const Geo &gf)
{
    if (gc.xs != 1 || gf.xs != 1) return false;
    const char *e = getenv("RS_TRANSFER");
    if (e && strcmp(e, "pair") == 0) return true;
    if (e && strcmp(e, "single") == 0) return false;
    return gc.N >= (1ll << 18);
}

template <typename T>
inline void launch_restrict_t(const Geo &gc, const Geo &gf, const T *psi_f, const T *d_f,
                              T *psibar_c, T *g_c, hipStream_t s)
{
    if (pair_transfer(gc, gf)) {
        const ColourMap cm = pair_map(gc);
        const dim3 pg(xcd_grid((cm.total + 255) / 256));
        if (gc.dim == 1)
            hipLaunchKernelGGL((k_restrict_pair<1, T>), pg, dim3(256), 0, s, gc, gf, psi_f, d_f,
                               psibar_c, g_c, cm);
        else if (gc.dim == 2)
            hipLaunchKernelGGL((k_restrict_pair<2, T>), pg, dim3(256), 0, s, gc, gf, psi_f, d_f,
                               psibar_c, g_c, cm);
        else
            hipLaunchKernelGGL((k_restrict_pair<3, T>), pg, dim3(256), 0, s, gc, gf, psi_f, d_f,
                               psibar_c, g_c, cm);
        return;
    }
    const dim3 grid(xcd_grid(((unsigned long long)gc.N + 255) / 256));
    const NodeMap nm = node_map(gc);
    if (gc.dim == 1)
        hipLaunchKernelGGL((k_restrict<1, T>), grid, dim3(256), 0, s, gc, gf, psi_f, d_f, psibar_c, g_c, nm);
    else if (gc.dim == 2)
        hipLaunchKernelGGL((k_restrict<2, T>), grid, dim3(256), 0, s, gc, gf, psi_f, d_f, psibar_c, g_c, nm);
    else
        hipLaunchKernelGGL((k_restrict<3, T>), grid, dim3(256), 0, s, gc, gf, psi_f, d_f, psibar_c, g_c, nm);
}

template <typename T, bool FULL = false>
inline void launch_prolong_t(const Geo &gf, const Geo &gc, const T *psi_c, const T *psibar_c,
                             T *psi_f, hipStream_t s)
{
    if (pair_transfer(gc, gf)) {
        const ColourMap cm = pair_map(gc);
        const dim3 pg(xcd_grid((cm.total + 255) / 256));
        if (gf.dim == 1)
            hipLaunchKernelGGL((k_prolong_pair<1, T, FULL>), pg, dim3(256), 0, s, gf, gc, psi_c,
                               psibar_c, psi_f, cm);
        else if (gf.dim == 2)
            hipLaunchKernelGGL((k_prolong_pair<2, T, FULL>), pg, dim3(256), 0, s, gf, gc, psi_c,
                               psibar_c, psi_f, cm);
        else
            hipLaunchKernelGGL((k_prolong_pair<3, T, FULL>), pg, dim3(256), 0, s, gf, gc, psi_c,
                               psibar_c, psi_f, cm);
        return;
    }
    const dim3 grid(xcd_grid(((unsigned long long)gc.N + 255) / 256));
    const NodeMap nm = node_map(gc);
    if (gf.dim == 1)
        hipLaunchKernelGGL((k_prolong<1, T, FULL>), grid, dim3(256), 0, s, gf, gc, psi_c, psibar_c,
                           psi_f, nm);
    else if (gf.dim == 2)
        hipLaunchKernelGGL((k_prolong<2, T, FULL>), grid, dim3(256), 0, s, gf, gc, psi_c, psibar_c,
                           psi_f, nm);
    else
        hipLaunchKernelGGL((k_prolong<3, T, FULL>), grid, dim3(256), 0, s, gf, gc, psi_c, psibar_c,
                           psi_f, nm);
}

// Injection to a coarse level: v_H[I] = v_h[2I].
template <typename T>
__global__ __launch_bounds__(256) void k_inject_t(Geo gc, Geo gf, const T *vf, T *vc)
{
    int i = blockIdx.x * kBX + threadIdx.x;
    int j = blockIdx.y * kBY + threadIdx.y;
    int k = blockIdx.z;
    if (i >= gc.n[0] || j >= gc.n[1]) return;
    vc[lin(gc, i, j, k)] = vf[lin(gf, 2 * i, 2 * j, 2 * k)];
}

}  // namespace rs
