// FP32 kernels of the mixed-precision solve: FAS V-cycles in FP32 on the
// correction equation N(psi_b + delta) - N(psi_b) = r (see soil_mp.h), inside
// an FP64 defect-correction loop whose residual, history and stopping test stay
// in FP64 (kernels_fp64.hip).  Per level the FP32 cycles keep delta, K*, the
// right-hand side, the inner defect, the restricted delta and the base state
// psi_b, 4 B each; a sweep moves delta, K*, rhs and psi_b (20 B per update).
#include <cstdio>

#include "rs_internal.h"
#include "soil_device.h"
#include "grid_device.h"
#include "transfer.h"
#include "soil_mp.h"
#include "cell32.h"

namespace rs {

namespace {

// One colour of a red-black FP32 correction sweep, one node per lane; BUF as
// for the FP64 sweep (raw buffer loads with 32-bit offsets).
template <int MODEL, bool SINK, int DIM, bool BUF>
__global__ __launch_bounds__(256) void k_sweep32(Geo g, Law32 L, float a, const double *beta,
                                                 float lambdaU, const float *K, const float *rhs,
                                                 const float *pb, float *dl, int colour,
                                                 ColourMap cm)
{
    const unsigned long long t =
        (unsigned long long)xcd_block_dir(gridDim.x / 8u, colour & 1) * blockDim.x + threadIdx.x;
    if (t >= cm.total) return;
    const unsigned row = udiv((unsigned)t, cm.dH);
    const unsigned ih = (unsigned)(t - (unsigned long long)row * cm.H);
    unsigned j = 0, k = 0;
    if (DIM == 3) {
        k = udiv(row, cm.dN1);
        j = row - k * cm.n1;
    } else if (DIM == 2) {
        j = row;
    }
    const int par = (int)((j + k + colour) & 1);
    const int i = 2 * (int)ih + par;
    if (i >= g.n[0]) return;
    if (dirichlet_t<DIM>(g, i, (int)j, (int)k)) return;
    // parity-split row (see k_sweep): node at ih (+ xh if odd), left neighbour
    // at ih (odd) or xh + ih - 1 (even), the right one just after it
    const long long rb = (long long)j * g.stride[1] + (long long)k * g.stride[2];
    const long long idx = rb + ih + (par ? g.xh : 0);
    const long long xl = rb + ih + (par ? 0 : g.xh - 1);
    if constexpr (BUF) {
        const long long bytes = (g.N + 64) * (long long)sizeof(float);   // + padding
        const __amdgpu_buffer_rsrc_t rK = buf_rsrc(K, bytes), rR = buf_rsrc(rhs, bytes),
                                     rB = buf_rsrc(pb, bytes), rD = buf_rsrc(dl, bytes);
        const int vo = (int)idx * 4, vx = (int)xl * 4;
        const Stencil<DIM> sn = stencil_split<DIM>(g, i, (int)j, (int)k, idx, xl);
        float Kn[2 * DIM], dn[2 * DIM];
        const v2f32 kx = buf_ld2(rK, vx, 0.0f), dx = buf_ld2(rD, vx, 0.0f);
        Kn[0] = kx.x;
        Kn[1] = kx.y;
        dn[0] = dx.x;
        dn[1] = dx.y;
#pragma unroll
        for (int l = 1; l < DIM; ++l) {
            const int so = g.stride[l] * 4;
            Kn[2 * l] = buf_ld<float>(rK, vo - so);
            dn[2 * l] = buf_ld<float>(rD, vo - so);
            Kn[2 * l + 1] = buf_ld<float>(rK, vo + so);
            dn[2 * l + 1] = buf_ld<float>(rD, vo + so);
        }
        const float Ki = buf_ld<float>(rK, vo), d0 = buf_ld<float>(rD, vo);
        const float f = buf_ld<float>(rR, vo), pbi = buf_ld<float>(rB, vo);
        buf_st(rD, vo, ngs_point32<MODEL, SINK, DIM>(g, L, a, beta, lambdaU, sn, Ki, Kn, dn, f, d0,
                                                     pbi, i, (int)j, (int)k, colour));
    } else {
        ngs_cell32<MODEL, SINK, DIM, true, true>(g, L, a, beta, lambdaU, K, rhs, pb, dl, i, (int)j,
                                                 (int)k, colour, idx, xl);
    }
}

// One colour of the FP32 correction sweep, two nodes of that colour per lane
// (half-row positions 2q and 2q + 1, nodes i and i + 2), as k_sweep_pair does
// for FP64: own values one 8-byte load per array, each off-row direction one
// pair, the axis-0 neighbours a pair and a single; the off-row stencil
// coefficients are formed once for both nodes.  Both point problems are
// reduced before the first solve.  Kappa CONST or REL.  Slots: (xh + 1) / 2
// per row.
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(256) void k_sweep32_pair(Geo g, Law32 L, float a, const double *beta,
                                                      const float *K, const float *rhs,
                                                      const float *pb, float *dl, int colour,
                                                      ColourMap cm)
{
    const unsigned long long t =
        (unsigned long long)xcd_block_dir(gridDim.x / 8u, colour & 1) * blockDim.x + threadIdx.x;
    if (t >= cm.total) return;
    const unsigned row = udiv((unsigned)t, cm.dH);
    const int q = (int)((unsigned)(t - (unsigned long long)row * cm.H));
    unsigned j = 0, k = 0;
    if (DIM == 3) {
        k = udiv(row, cm.dN1);
        j = row - k * cm.n1;
    } else if (DIM == 2) {
        j = row;
    }
    const int par = (int)((j + k + colour) & 1);
    const int len = par ? g.n[0] - g.xh : g.xh;
    if (2 * q >= len) return;
    const bool has_b = 2 * q + 1 < len;
    const int ia = 4 * q + par;
    const bool dir_a = dirichlet_t<DIM>(g, ia, (int)j, (int)k);
    const bool dir_b = !has_b || dirichlet_t<DIM>(g, ia + 2, (int)j, (int)k);
    if (dir_a && dir_b) return;
    const long long rb = (long long)j * g.stride[1] + (long long)k * g.stride[2];
    const long long idx = rb + (par ? g.xh : 0) + 2 * q;
    const long long xl = rb + (par ? 0 : g.xh - 1) + 2 * q;
    const long long bytes = (g.N + 64) * (long long)sizeof(float);   // + padding
    const __amdgpu_buffer_rsrc_t rK = buf_rsrc(K, bytes), rR = buf_rsrc(rhs, bytes),
                                 rB = buf_rsrc(pb, bytes), rD = buf_rsrc(dl, bytes);
    const int vo = (int)idx * 4, vx = (int)xl * 4;
    const v2f32 D = buf_ld2(rD, vo, 0.0f), KK = buf_ld2(rK, vo, 0.0f), R2 = buf_ld2(rR, vo, 0.0f),
                B2 = buf_ld2(rB, vo, 0.0f);
    const v2f32 DX = buf_ld2(rD, vx, 0.0f), KX = buf_ld2(rK, vx, 0.0f);
    const float DX2 = buf_ld<float>(rD, vx + 8), KX2 = buf_ld<float>(rK, vx + 8);
    constexpr int NO = 2 * (DIM - 1);
    v2f32 Do[NO > 0 ? NO : 1], Ko[NO > 0 ? NO : 1];
    float cfo[NO > 0 ? NO : 1];
#pragma unroll
    for (int l = 1; l < DIM; ++l) {
        const int so = g.stride[l] * 4;
        Do[2 * l - 2] = buf_ld2(rD, vo - so, 0.0f);
        Ko[2 * l - 2] = buf_ld2(rK, vo - so, 0.0f);
        Do[2 * l - 1] = buf_ld2(rD, vo + so, 0.0f);
        Ko[2 * l - 1] = buf_ld2(rK, vo + so, 0.0f);
        const int cl = l == 1 ? (int)j : (int)k;
        const float cf = (float)(((cl == 0 || cl == g.n[l] - 1) ? 1.0 : 0.5) * g.ih2[l]);
        cfo[2 * l - 2] = cl > 0 ? cf : 0.0f;
        cfo[2 * l - 1] = cl < g.n[l] - 1 ? cf : 0.0f;
    }
    const float dw[3] = {DX.x, DX.y, DX2}, kw[3] = {KX.x, KX.y, KX2};
    PointEq32 e[2];
#pragma unroll
    for (int a2 = 0; a2 < 2; ++a2) {
        const int i = ia + 2 * a2;
        float cf[2 * DIM], Kn[2 * DIM], dn[2 * DIM];
        const float cx = (float)(((i == 0 || i == g.n[0] - 1) ? 1.0 : 0.5) * g.ih2[0]);
        cf[0] = i > 0 ? cx : 0.0f;
        cf[1] = i < g.n[0] - 1 ? cx : 0.0f;
        Kn[0] = kw[a2];
        Kn[1] = kw[a2 + 1];
        dn[0] = dw[a2];
        dn[1] = dw[a2 + 1];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            cf[2 + o] = cfo[o];
            Kn[2 + o] = a2 ? Ko[o].y : Ko[o].x;
            dn[2 + o] = a2 ? Do[o].y : Do[o].x;
        }
        e[a2] = ngs_reduce32<SINK, DIM, false>(g, L, beta, 0.0f, cf, a2 ? KK.y : KK.x, Kn, dn,
                                              a2 ? R2.y : R2.x, a2 ? D.y : D.x, i, (int)j, (int)k,
                                              colour);
    }
    const float xa = dir_a ? D.x : ngs_solve32<MODEL, SINK>(L, a, e[0], D.x, B2.x);
    if (!has_b) {
        buf_st(rD, vo, xa);
        return;
    }
    const float xb = dir_b ? D.y : ngs_solve32<MODEL, SINK>(L, a, e[1], D.y, B2.y);
    const v2f32 out = {xa, xb};
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i32, out), rD, vo, 0, 0);
}

template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(256) void k_sweep32_small(Geo g, Law32 L, float a, const double *beta,
                                                       float lambdaU, const float *K,
                                                       const float *rhs, const float *pb,
                                                       float *dl, int nsweeps)
{
    const int N = (int)g.N;
    for (int s = 0; s < nsweeps; ++s) {
        int changed = 0;
        for (int colour = 0; colour < 2; ++colour) {
            for (int t = threadIdx.x; t < N; t += blockDim.x) {
                int i = t % g.n[0];
                int r = t / g.n[0];
                int j = r % g.n[1];
                int k = r / g.n[1];
                if (((i + j + k) & 1) != colour) continue;
                if (dirichlet_t<DIM>(g, i, j, k)) continue;
                changed |= ngs_cell32<MODEL, SINK, DIM, true, true>(g, L, a, beta, lambdaU, K, rhs, pb,
                                                                    dl, i, j, k, colour);
            }
            // a sweep that moved no value by more than FP32 rounding (4 ulp) has
            // converged in FP32: the correction solve only sets the outer
            // FP64 iteration's contraction, the rest would shuffle rounding
            if (colour == 0) __syncthreads();
            else if (!__syncthreads_or(changed)) return;
        }
    }
}

// Inner defect r32 = rhs - N_delta(delta) (0 at Dirichlet nodes).
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(256) void k_residual32(Geo g, Law32 L, float a, const double *beta,
                                                    const float *K, const float *rhs,
                                                    const float *pb, const float *dl, float *r,
                                                    NodeMap nm)
{
    const unsigned long long t =
        (unsigned long long)xcd_block(gridDim.x / 8u) * blockDim.x + threadIdx.x;
    if (t >= (unsigned long long)g.N) return;
    int i, j, k;
    node_ijk(nm, t, i, j, k);
    const long long idx = (long long)t;
    float v = 0.0f;
    if (!dirichlet_t<DIM>(g, i, j, k))
        v = rhs[idx] - apply_Nd<MODEL, SINK, DIM, true>(g, L, a, beta, K, pb, dl, i, j, k, idx);
    r[idx] = v;
}

// FAS coarse right-hand side of the correction equation:
// rhs_H = N_delta,H(dbar_H) + r_H (rhs_H holds r_H on entry), delta_H = dbar_H.
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(256) void k_coarse_rhs32(Geo g, Law32 L, float a, const double *beta,
                                                      const float *K, const float *pb,
                                                      const float *dbar, float *rhs, float *dl,
                                                      NodeMap nm)
{
    const unsigned long long t =
        (unsigned long long)xcd_block(gridDim.x / 8u) * blockDim.x + threadIdx.x;
    if (t >= (unsigned long long)g.N) return;
    int i, j, k;
    node_ijk(nm, t, i, j, k);
    const long long idx = (long long)t;
    if (!dirichlet_t<DIM>(g, i, j, k))
        rhs[idx] = apply_Nd<MODEL, SINK, DIM, true>(g, L, a, beta, K, pb, dbar, i, j, k, idx) + rhs[idx];
    dl[idx] = dbar[idx];
}

__global__ __launch_bounds__(256) void k_to_f32(long long N, const double *src, float *dst)
{
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N) dst[t] = (float)src[t];
}

// psi += delta in FP64 (delta is 0 at Dirichlet nodes).
__global__ __launch_bounds__(256) void k_apply_delta(long long N, const float *dl, double *psi64)
{
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N) psi64[t] += (double)dl[t];
}

// FP32 red-black sweeps of one level inside the one-work-group cycle; on the
// coarsest level (exit) with the exit of k_sweep32_small (a sweep that moved no
// value by more than 4 FP32 ulp).
template <int MODEL, bool SINK, int DIM>
__device__ void tail_sweeps32(const TailLevel &T, const Law32 &L, float a, int n, bool exit)
{
    const ColourMap cm = tail_cm(T);
    for (int sw = 0; sw < n; ++sw) {
        int changed = 0;
        for (int colour = 0; colour < 2; ++colour) {
            for (unsigned long long t = threadIdx.x; t < cm.total; t += blockDim.x) {
                int i, j, k;
                if (!colour_ijk(T.g, cm, t, colour, i, j, k)) continue;
                if (dirichlet_t<DIM>(T.g, i, j, k)) continue;
                changed |= ngs_cell32<MODEL, SINK, DIM, true, true>(T.g, L, a, T.beta, T.lambdaU32,
                                                                    T.K32, T.rhs32, T.pb32, T.dl,
                                                                    i, j, k, colour);
            }
            if (colour == 0 || !exit) __syncthreads();
            else if (!__syncthreads_or(changed)) return;
        }
    }
}

// The FP32 correction cycle from level top (all of whose levels hold at most
// kTailNodes nodes) down to level last and back, in one work-group, with the
// per-node arithmetic of the launched kernels: sweeps, inner defect
// (k_residual32), full weighting of delta and of the defect, coarse
// right-hand side (k_coarse_rhs32), the coarsest sweeps, prolongation.
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(512) void k_vcycle_tail32(const TailArgs *A, int top, int last,
                                                       Law32 L, float a, int nu1, int nu2, int nuc)
{
    __shared__ TailLevel SL[kMaxLevels];
    for (int l = top + (int)threadIdx.x; l <= last; l += (int)blockDim.x) SL[l] = A->lv[l];
    __syncthreads();
    for (int l = top; l < last; ++l) {
        const TailLevel &F = SL[l], &C = SL[l + 1];
        tail_sweeps32<MODEL, SINK, DIM>(F, L, a, nu1, false);
        const NodeMap nf = tail_nm(F), nc = tail_nm(C);
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)F.g.N; t += blockDim.x) {
            int i, j, k;
            node_ijk(nf, t, i, j, k);
            float v = 0.0f;
            if (!dirichlet_t<DIM>(F.g, i, j, k))
                v = F.rhs32[t] - apply_Nd<MODEL, SINK, DIM, true>(F.g, L, a, F.beta, F.K32, F.pb32,
                                                                   F.dl, i, j, k, (long long)t);
            F.r32[t] = v;
        }
        __syncthreads();
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)C.g.N; t += blockDim.x) {
            int i, j, k;
            node_ijk(nc, t, i, j, k);
            restrict_at<DIM, float, true>(C.g, F.g, F.dl, F.r32, C.dbar32, C.rhs32, i, j, k);
        }
        __syncthreads();
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)C.g.N; t += blockDim.x) {
            int i, j, k;
            node_ijk(nc, t, i, j, k);
            if (!dirichlet_t<DIM>(C.g, i, j, k))
                C.rhs32[t] = apply_Nd<MODEL, SINK, DIM, true>(C.g, L, a, C.beta, C.K32, C.pb32,
                                                              C.dbar32, i, j, k, (long long)t) +
                             C.rhs32[t];
            C.dl[t] = C.dbar32[t];
        }
        __syncthreads();
    }
    tail_sweeps32<MODEL, SINK, DIM>(SL[last], L, a, nuc, true);
    __syncthreads();
    for (int l = last - 1; l >= top; --l) {
        const TailLevel &F = SL[l], &C = SL[l + 1];
        const NodeMap nf = tail_nm(F);
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)F.g.N; t += blockDim.x) {
            int i, j, k;
            node_ijk(nf, t, i, j, k);
            prolong_at<DIM, float>(F.g, C.g, C.dl, C.dbar32, F.dl, i, j, k);
        }
        __syncthreads();
        tail_sweeps32<MODEL, SINK, DIM>(F, L, a, nu2, false);
        __syncthreads();
    }
}

unsigned blocks_for(long long N) { return (unsigned)((N + 255) / 256); }

// Two nodes per lane in the FP32 sweeps of levels of at least 2^22 nodes (at
// 129^3 one node per lane is faster: 11.0 against 11.8 us); RS_SWEEP32=single
// / pair: one on every level / two on every buffer-path level.
bool pair32_level(const Geo &g)
{
    const char *e = getenv("RS_SWEEP32");
    if (e && strcmp(e, "single") == 0) return false;
    if (e && strcmp(e, "pair") == 0) return true;
    return g.N >= (1ll << 22);
}

struct Sweep32Launch {
    const Geo &g; const Law32 &law; float a; const double *beta; float lambdaU; const float *K;
    const float *rhs; const float *pb; float *dl; int nsweeps; hipStream_t s;
    template <int M, bool S, int D>
    void go()
    {
        if (g.N <= 1024) {
            hipLaunchKernelGGL((k_sweep32_small<M, S, D>), dim3(1), dim3(256), 0, s, g, law, a, beta,
                               lambdaU, K, rhs, pb, dl, nsweeps);
            return;
        }
        ColourMap cm = colour_map(g);
        dim3 grid(xcd_grid((cm.total + 255) / 256));
        const bool buf = buffer_ok(g, sizeof(float));
        if (buf && law.kappa_rule != kKappaRemark && pair32_level(g)) {
            ColourMap pm = cm;
            pm.H = (cm.H + 1) / 2;
            pm.dH = make_fastdiv(pm.H);
            pm.total = (unsigned long long)pm.H * g.n[1] * g.n[2];
            const dim3 pgrid(xcd_grid((pm.total + 255) / 256));
            for (int sw = 0; sw < nsweeps; ++sw)
                for (int colour = 0; colour < 2; ++colour)
                    hipLaunchKernelGGL((k_sweep32_pair<M, S, D>), pgrid, dim3(256), 0, s, g, law, a,
                                       beta, K, rhs, pb, dl, colour, pm);
            return;
        }
        for (int sw = 0; sw < nsweeps; ++sw)
            for (int colour = 0; colour < 2; ++colour) {
                if (buf)
                    hipLaunchKernelGGL((k_sweep32<M, S, D, true>), grid, dim3(256), 0, s, g, law, a,
                                       beta, lambdaU, K, rhs, pb, dl, colour, cm);
                else
                    hipLaunchKernelGGL((k_sweep32<M, S, D, false>), grid, dim3(256), 0, s, g, law, a,
                                       beta, lambdaU, K, rhs, pb, dl, colour, cm);
            }
    }
};

struct Residual32Launch {
    const Geo &g; const Law32 &law; float a; const double *beta; const float *K; const float *rhs;
    const float *pb; const float *dl; float *r; hipStream_t s;
    template <int M, bool S, int D>
    void go()
    {
        hipLaunchKernelGGL((k_residual32<M, S, D>), dim3(xcd_grid(((unsigned long long)g.N + 255) / 256)),
                           dim3(256), 0, s, g, law, a, beta, K, rhs, pb, dl, r, node_map(g));
    }
};

struct CoarseRhs32Launch {
    const Geo &g; const Law32 &law; float a; const double *beta; const float *K; const float *pb;
    const float *dbar; float *rhs; float *dl; hipStream_t s;
    template <int M, bool S, int D>
    void go()
    {
        hipLaunchKernelGGL((k_coarse_rhs32<M, S, D>),
                           dim3(xcd_grid(((unsigned long long)g.N + 255) / 256)), dim3(256), 0, s,
                           g, law, a, beta, K, pb, dbar, rhs, dl, node_map(g));
    }
};

// dispatch() keys on Law::model / Law::sink; build a Law carrying those two.
Law dispatch_key(const Law32 &l)
{
    Law k{};
    k.model = l.model;
    k.sink = l.sink;
    return k;
}

}  // namespace

Law32 make_law32(const Law &L)
{
    Law32 f;
    f.model = L.model;
    f.ts = (float)L.ts;
    f.tr = (float)L.tr;
    f.dT = (float)L.dT;
    f.vg_alpha = (float)L.vg_alpha;
    f.vg_n = (float)L.vg_n;
    f.vg_m = (float)L.vg_m;
    f.hk_alpha = (float)L.hk_alpha;
    f.hk_beta = (float)L.hk_beta;
    f.unit = (float)L.unit;
    f.lin_c = (float)L.lin_c;
    f.sink = L.sink;
    f.h1 = (float)L.h1;
    f.h2 = (float)L.h2;
    f.h3 = (float)L.h3;
    f.h4 = (float)L.h4;
    f.xi = (float)L.xi;
    f.kappa = (float)L.kappa;
    f.kappa_rule = L.kappa_rule;
    f.newton = L.newton;
    // The correction solve feeds FP64 defect correction, which only needs it to
    // a few digits: whenever the FP64 solve may stop early, the FP32 one stops
    // after a step of 1e-5 |d| (the steps it leaves out are ~1e-10 |d|).
    f.newton_tol = L.newton_tol > 0.0 ? 1e-5f : 0.0f;
    // binom(e, k) = binom(e, k - 1) (e - k + 1) / k, in double, rounded once
    auto binom = [](double e, float *c) {
        double b = 1.0;
        for (int k = 1; k <= 6; ++k) {
            b *= (e - (k - 1)) / k;
            c[k - 1] = (float)b;
        }
    };
    const double e1 = L.model == kHaverkamp ? L.hk_beta : L.vg_n;
    binom(e1, f.bin1);
    binom(-L.vg_m, f.bin2);
    f.series_u = (e1 >= -1.0 && e1 <= 7.0 && -L.vg_m >= -1.0) ? 0.0625f : 0.0f;
    return f;
}

void launch_sweep32(const Geo &g, const Law32 &law, float a, const double *beta, float lambdaU,
                    const float *K, const float *rhs, const float *pb, float *dl, int nsweeps,
                    hipStream_t s)
{
    if (nsweeps <= 0) return;
    dispatch(dispatch_key(law), g.dim,
             Sweep32Launch{g, law, a, beta, lambdaU, K, rhs, pb, dl, nsweeps, s});
}

struct Tail32Launch {
    const TailArgs *A; int top, last; const Law32 &law; float a; int nu1, nu2, nuc; hipStream_t s;
    template <int M, bool S, int D>
    void go()
    {
        hipLaunchKernelGGL((k_vcycle_tail32<M, S, D>), dim3(1), dim3(512), 0, s, A, top, last, law,
                           a, nu1, nu2, nuc);
    }
};

void launch_vcycle_tail32(const TailArgs *args_dev, int top, int last, const Law32 &law, float a,
                          int nu1, int nu2, int nuc, int dim, hipStream_t s)
{
    dispatch(dispatch_key(law), dim, Tail32Launch{args_dev, top, last, law, a, nu1, nu2, nuc, s});
}

void launch_residual32(const Geo &g, const Law32 &law, float a, const double *beta, const float *K,
                       const float *rhs, const float *pb, const float *dl, float *r, hipStream_t s)
{
    dispatch(dispatch_key(law), g.dim, Residual32Launch{g, law, a, beta, K, rhs, pb, dl, r, s});
}

void launch_coarse_rhs32(const Geo &g, const Law32 &law, float a, const double *beta,
                         const float *K, const float *pb, const float *dbar, float *rhs, float *dl,
                         hipStream_t s)
{
    dispatch(dispatch_key(law), g.dim, CoarseRhs32Launch{g, law, a, beta, K, pb, dbar, rhs, dl, s});
}

void launch_restrict32(const Geo &gc, const Geo &gf, const float *dl_f, const float *r_f,
                       float *dbar_c, float *rhs_c, hipStream_t s)
{
    launch_restrict_t<float>(gc, gf, dl_f, r_f, dbar_c, rhs_c, s);
}

void launch_prolong32(const Geo &gf, const Geo &gc, const float *dl_c, const float *dbar_c,
                      float *dl_f, hipStream_t s)
{
    launch_prolong_t<float>(gf, gc, dl_c, dbar_c, dl_f, s);
}

namespace {

// One level of the base-state injection: its node counts, the row layout and
// strides that lin() uses, and its array.
struct InjLevel {
    int n0, n1, xs, xh;
    long long s1, s2, N;
    float *v;
};

struct InjectPlan {
    int nlev;
    long long first[kMaxLevels + 1];   // first work-group of each coarse level
    InjLevel lv[kMaxLevels];
};

__device__ __forceinline__ long long inj_pos(const InjLevel &L, int i, int j, int k)
{
    return (long long)((i >> L.xs) + (i & 1) * L.xh) + (long long)j * L.s1 + (long long)k * L.s2;
}

// psi_b on every coarse level at once: node (i, j, k) of level l takes the
// finest level's value at (2^l i, 2^l j, 2^l k), the composition of the
// level-to-level injections v_H[I] = v_h[2I].  The work-groups of a level are
// contiguous, so the level is uniform within a group.
__global__ __launch_bounds__(256) void k_inject_base32(InjectPlan P)
{
    const long long b = blockIdx.x;
    int l = 1;
    while (l + 1 < P.nlev && b >= P.first[l + 1]) ++l;
    const InjLevel &c = P.lv[l];
    const long long t = (b - P.first[l]) * 256 + threadIdx.x;
    if (t >= c.N) return;
    const int i = (int)(t % c.n0);
    const long long r = t / c.n0;
    const int j = (int)(r % c.n1), k = (int)(r / c.n1);
    c.v[inj_pos(c, i, j, k)] = P.lv[0].v[inj_pos(P.lv[0], i << l, j << l, k << l)];
}

}  // namespace

void launch_inject_base32(const Geo *geo, float *const *pb, int nlev, hipStream_t s)
{
    if (nlev < 2) return;
    InjectPlan P;
    memset(&P, 0, sizeof P);
    P.nlev = nlev;
    long long blocks = 0;
    for (int l = 0; l < nlev; ++l) {
        const Geo &g = geo[l];
        P.lv[l] = InjLevel{g.n[0], g.n[1], g.xs, g.xh, (long long)g.stride[1],
                           (long long)g.stride[2], g.N, pb[l]};
        if (l >= 1) {
            P.first[l] = blocks;
            blocks += (g.N + 255) / 256;
        }
    }
    P.first[nlev] = blocks;
    hipLaunchKernelGGL(k_inject_base32, dim3((unsigned)blocks), dim3(256), 0, s, P);
}

void launch_to_f32(long long N, const double *src, float *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(N)), dim3(256), 0, s, N, src, dst);
}

void launch_apply_delta(long long N, const float *dl, double *psi64, hipStream_t s)
{
    hipLaunchKernelGGL(k_apply_delta, dim3(blocks_for(N)), dim3(256), 0, s, N, dl, psi64);
}

}  // namespace rs
