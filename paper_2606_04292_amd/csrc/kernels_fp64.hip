// FP64 kernels of the NGS-FAS V-cycle: step setup (history, lagged K*, right-
// hand side), red-black NGS sweeps, defect + max-norm, full-weighting
// restriction with the FAS coarse right-hand side, linear prolongation.
//
// Stencil: for node i and a neighbour j across a face normal to axis l,
// m_ij = (K*_i + K*_j) / 2 / (w_l h_l^2), w_l = 1/2 on a boundary of axis l
// (half control volume at no-flux / free-drainage faces), else 1
// (eq. discrete-strong with arithmetic face averages; the matrix M of
// section 2).  Node kinds come from indices, so a sweep moves only psi, K*
// and g (8 B each per node) plus the psi write.
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "rs_internal.h"
#include "soil_device.h"
#include "grid_device.h"
#include "transfer.h"
#include "cell64.h"

namespace rs {

namespace {

// p[0..n) = v (clears the norm words with a kernel rather than a memset)
__global__ void k_fill_u64(unsigned long long *p, int n, unsigned long long v)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

// Reorder an array of one level between the lexicographic order of the C ABI
// and the level's row layout (Geo::xs): to_level: dst[layout index of node t]
// = src[t], t the lexicographic index; else dst[t] = src[layout index].
template <typename T>
__global__ __launch_bounds__(256) void k_relayout(Geo g, const T *src, T *dst, int to_level,
                                                  FastDiv d0)
{
    const unsigned long long t = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (unsigned long long)g.N) return;
    const unsigned row = udiv((unsigned)t, d0);
    const int i = (int)(t - (unsigned long long)row * (unsigned)g.n[0]);
    const long long m = (long long)row * g.n[0] + xpos(g, i);
    if (to_level) dst[m] = src[t];
    else dst[t] = src[m];
}

// ---------------------------------------------------------------------------
// Step setup (eq. fully-bdf1; BDF2 reading; eq. Nh-def for g)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_setup_kstar(Geo g, Law L, Step st, const double *psi_n,
                                                     const double *psi_nm1, const double *Ks,
                                                     double *K, double *psi)
{
    int i = blockIdx.x * kBX + threadIdx.x;
    int j = blockIdx.y * kBY + threadIdx.y;
    int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    long long idx = lin(g, i, j, k);
    double p0;
    K[idx] = kstar_at(g, L, st, psi_n, psi_nm1, Ks ? Ks[idx] : L.Ks, i, j, k, idx, &p0);
    psi[idx] = p0;
}

__global__ __launch_bounds__(256) void k_setup_g(Geo g, Law L, Step st, const double *psi_n,
                                                 const double *psi_nm1, const double *K,
                                                 double *gv)
{
    int i = blockIdx.x * kBX + threadIdx.x;
    int j = blockIdx.y * kBY + threadIdx.y;
    int k = blockIdx.z;
    if (i >= g.n[0] || j >= g.n[1]) return;
    long long idx = lin(g, i, j, k);
    gv[idx] = g_at(g, L, st, psi_n, psi_nm1, K, i, j, k, idx);
}

__global__ __launch_bounds__(256) void k_inject(Geo gc, Geo gf, const double *Kf, double *Kc)
{
    int i = blockIdx.x * kBX + threadIdx.x;
    int j = blockIdx.y * kBY + threadIdx.y;
    int k = blockIdx.z;
    if (i >= gc.n[0] || j >= gc.n[1]) return;
    Kc[lin(gc, i, j, k)] = Kf[lin(gf, 2 * i, 2 * j, 2 * k)];
}

// Coarse K* as the full-weighting average of the finer level's K* (the
// alternative to k_inject; section 3.2 defines the coarse operator by analogy).
template <int DIM>
__global__ __launch_bounds__(256) void k_fw_coarse(Geo gc, Geo gf, const double *Kf, double *Kc,
                                                   NodeMap nm)
{
    const unsigned long long t =
        (unsigned long long)xcd_block(gridDim.x / 8u) * blockDim.x + threadIdx.x;
    if (t >= (unsigned long long)gc.N) return;
    int i, j, k;
    node_ijk(nm, t, i, j, k);
    Kc[t] = fw_value<DIM, double>(gf, Kf, i, j, k);
}

// max over red unknowns of the row sum of U over unknown neighbours (the red-
// black ordering puts every neighbour of a red node after it)
__global__ __launch_bounds__(256) void k_lambda_u(Geo g, const double *K, unsigned long long *out)
{
    int i = blockIdx.x * kBX + threadIdx.x;
    int j = blockIdx.y * kBY + threadIdx.y;
    int k = blockIdx.z;
    double v = 0.0;
    if (i < g.n[0] && j < g.n[1] && ((i + j + k) & 1) == 0 && !dirichlet_at(g, i, j, k, nullptr)) {
        long long idx = lin(g, i, j, k);
        int c[3] = {i, j, k};
        double Ki = K[idx];
        for_each_nb(g, c, idx, [&](long long jn, double cf, int l, int side) {
            int d[3] = {i, j, k};
            d[l] += side;
            if (!dirichlet_at(g, d[0], d[1], d[2], nullptr)) v += cf * (Ki + K[jn]);
        });
    }
    v = block_max(v);
    if (threadIdx.x == 0 && threadIdx.y == 0) atomicMax(out, (unsigned long long)__double_as_longlong(v));
}

// ---------------------------------------------------------------------------
// Red-black NGS (eq. iterative / eq. point-update)
// ---------------------------------------------------------------------------

// The scalars of one unknown's local problem (eq. point-update): the
// coefficient c = xi + kappa + m_ii of its own value, the right-hand side f
// (g_i plus the neighbour couplings plus kappa x0) and its root density.
struct PointEq {
    double cc, f, b;
};

// Reduces the stencil of unknown (i, j, k): K*_i, g_i, the old value x0 and
// the K* and current psi of the 2 DIM neighbours (outside the domain: zero
// coefficient, any finite value).  REMARK = false: the caller has excluded the
// Remark's kappa rule.
template <bool SINK, int DIM, bool REMARK = true>
__device__ __forceinline__ PointEq ngs_reduce(const Geo &g, const Law &L, const double *beta,
                                              double lambdaU, const Stencil<DIM> &st, double Ki,
                                              const double *Kn, const double *pn, double f,
                                              double x0, int i, int j, int k, int colour)
{
    double mii = 0.0;
#pragma unroll
    for (int q = 0; q < 2 * DIM; ++q) {
        const double m = st.cf[q] * (Ki + Kn[q]);
        mii += m;
        f += m * pn[q];
    }
    double kap;
    if (L.kappa_rule == kKappaConst) {
        kap = L.kappa;
    } else if (!REMARK || L.kappa_rule == kKappaRel) {
        kap = L.kappa * mii;
    } else if (colour == 0) {
        double usum = 0.0;
#pragma unroll
        for (int q = 0; q < 2 * DIM; ++q) {
            int d[3] = {i, j, k};
            d[q >> 1] += (q & 1) ? 1 : -1;
            if (st.cf[q] != 0.0 && !dirichlet_at(g, d[0], d[1], d[2], nullptr))
                usum += st.cf[q] * (Ki + Kn[q]);
        }
        kap = lambdaU - usum;
    } else {
        kap = lambdaU;
    }
    PointEq e;
    e.f = f + kap * x0;
    e.cc = L.xi + kap + mii;
    const int vk = (DIM == 1) ? i : (DIM == 2 ? j : k);
    e.b = SINK ? beta[vk] : 0.0;
    return e;
}

// The safeguarded Newton solve of a reduced point problem.
template <int MODEL, bool SINK>
__device__ __forceinline__ double ngs_solve(const Geo &g, const Law &L, double a, const PointEq &e,
                                            double x0, long long idx)
{
    if constexpr (MODEL == kMulti) {
        const Law &Ls = L.soils[g.soil[idx]];
        return (L.newton == 3) ? local_solve_soil<SINK, 3>(Ls, a, e.b, e.cc, e.f, x0)
                               : local_solve_soil<SINK, 0>(Ls, a, e.b, e.cc, e.f, x0);
    } else {
        return (L.newton == 3) ? local_solve_t<MODEL, SINK, 3>(L, a, e.b, e.cc, e.f, x0)
                               : local_solve_t<MODEL, SINK, 0>(L, a, e.b, e.cc, e.f, x0);
    }
}

// New value of unknown (i, j, k) from gathered values (eq. point-update).
template <int MODEL, bool SINK, int DIM>
__device__ __forceinline__ double ngs_point(const Geo &g, const Law &L, double a, const double *beta,
                                            double lambdaU, const Stencil<DIM> &st, double Ki,
                                            const double *Kn, const double *pn, double f, double x0,
                                            int i, int j, int k, long long idx, int colour)
{
    const PointEq e = ngs_reduce<SINK, DIM>(g, L, beta, lambdaU, st, Ki, Kn, pn, f, x0, i, j, k,
                                            colour);
    return ngs_solve<MODEL, SINK>(g, L, a, e, x0, idx);
}

// Defect g_i - N_i(psi) of unknown i (column i of its row) at idx from its
// gathered values: x = psi_i, K*_i, g_i, the axis-0 neighbours (pl, kl: i - 1;
// pr, kr: i + 1) and the off-row neighbour values with their coefficients cfo
// (0: no neighbour; the node's own values stand in).  bz: root density of the
// row (2-D, 3-D); in 1-D the row is the vertical axis and beta[i] is used.
template <int MODEL, bool SINK, int DIM>
__device__ __forceinline__ double defect_at(const Geo &g, const Law &L, double a,
                                            const double *beta, double bz, int i, long long idx,
                                            double x, double Ki, double gi, double pl, double pr,
                                            double kl, double kr, const double *po,
                                            const double *ko, const double *cfo)
{
    constexpr int NO = 2 * (DIM - 1);
    double s;
    if constexpr (MODEL == kMulti) s = a * theta_only(L.soils[g.soil[idx]], x);
    else s = a * theta_only_t<MODEL>(L, x);
    if (SINK) {
        double fa, dfa;
        feddes(L, x, fa, dfa);
        s += ((DIM == 1) ? beta[i] : bz) * fa;
    }
    // neighbours in the order of stencil(): axis 0 low/high, then the others
    const double cx = ((i == 0 || i == g.n[0] - 1) ? 1.0 : 0.5) * g.ih2[0];
    const double cm0 = i > 0 ? cx : 0.0, cp0 = i < g.n[0] - 1 ? cx : 0.0;
    double mpsi = 0.0;
    mpsi += cm0 * (Ki + kl) * (x - pl);
    mpsi += cp0 * (Ki + kr) * (x - pr);
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        const bool ok = cfo[o] != 0.0;
        const double pn = ok ? po[o] : x;
        const double kn = ok ? ko[o] : Ki;
        mpsi += cfo[o] * (Ki + kn) * (x - pn);
    }
    return gi - (s + (L.xi * x + mpsi));
}

// Off-row coefficient of direction o (axis 1 + o / 2, low or high side) for a
// node on row coordinate cl of that axis; 0 where the neighbour is missing.
__device__ __forceinline__ double offrow_cf(const Geo &g, int o, int cl)
{
    const int l = 1 + o / 2;
    const bool up = o & 1;
    const bool ok = up ? cl < g.n[l] - 1 : cl > 0;
    return ok ? ((cl == 0 || cl == g.n[l] - 1) ? 1.0 : 0.5) * g.ih2[l] : 0.0;
}

// Update of unknown (i, j, k) stored at idx, its axis-0 neighbours at xl and
// xl + 1 (a grid's levels have parity-split rows, see stencil_split; the
// workspace arrays are padded, so both are always loaded, as one pair).
template <int MODEL, bool SINK, int DIM>
__device__ __forceinline__ bool ngs_cell_at(const Geo &g, const Law &L, double a,
                                            const double *beta, double lambdaU, const double *K,
                                            const double *gv, double *psi, int i, int j, int k,
                                            long long idx, long long xl, int colour)
{
    const Stencil<DIM> st = stencil_split<DIM>(g, i, j, k, idx, xl);
    const double Ki = K[idx];
    const double x0 = psi[idx];
    const double f = gv[idx];
    double Kn[2 * DIM], pn[2 * DIM];
    const double2_u kx = load_pair(K + xl), px = load_pair(psi + xl);
    Kn[0] = kx.x;
    Kn[1] = kx.y;
    pn[0] = px.x;
    pn[1] = px.y;
#pragma unroll
    for (int q = 2; q < 2 * DIM; ++q) {
        Kn[q] = K[st.jn[q]];
        pn[q] = psi[st.jn[q]];
    }
    const double x1 = ngs_point<MODEL, SINK, DIM>(g, L, a, beta, lambdaU, st, Ki, Kn, pn, f, x0, i,
                                                  j, k, idx, colour);
    psi[idx] = x1;
    return fabs(x1 - x0) > 8.8817841970012523e-16 * fabs(x0);   // 4 ulp (2^-50 |x0|)
}

// The update of unknown (i, j, k); true if it moved the stored value by more
// than 4 ulp.
template <int MODEL, bool SINK, int DIM>
__device__ __forceinline__ bool ngs_cell(const Geo &g, const Law &L, double a, const double *beta,
                                         double lambdaU, const double *K, const double *gv,
                                         double *psi, int i, int j, int k, int colour)
{
    const long long idx = lin(g, i, j, k);
    return ngs_cell_at<MODEL, SINK, DIM>(g, L, a, beta, lambdaU, K, gv, psi, i, j, k, idx,
                                         xnb(g, i, idx, -1), colour);
}

// ---------------------------------------------------------------------------
// Fused red-black sweep for 3-D levels, marching along z.  Lane (lx, ly) of a
// work-group owns the node pair x = 2p, 2p+1 of row y and walks up the
// group's z-chunk; at plane z its active column c is the red one
// (c + y + z even).  Step z computes the red value at (c, y, z) from old values,
// then the black value at (c, y, z-1), whose neighbours are all new red values:
// those of plane z-1 from LDS (written in the previous step by the lanes that
// own them), and the lane's own red values of planes z-2 and z.  A ring of
// lanes around the tile recomputes the red values that the tile's black nodes
// need from the neighbouring tiles, and the first step of a chunk recomputes
// the red plane below it; these are not stored.  Old values come from pin and
// new ones go to pout, each node written once by the tile that owns it: no
// ordering between work-groups, and a sweep reads psi, K* and g once (plus the
// halo).  The per-node arithmetic is that of the two-pass sweep (ngs_point),
// so the two agree to rounding (the compiler may fuse multiply-adds
// differently in the two kernels).
// ---------------------------------------------------------------------------

struct FusedMap {
    int LX, LY, ZC;      // lane grid (pairs x rows, ring included), planes per chunk
    int ntx, nty, ntz;
    int nwg, per;        // work-groups, logical groups per XCD
};

template <int MODEL, bool SINK>
__global__ __launch_bounds__(512) void k_sweep_fused(Geo g, Law L, Step st, const double *beta,
                                                     double lambdaU, const double *K,
                                                     const double *gv, const double *pin,
                                                     double *pout, FusedMap fm)
{
    extern __shared__ double red[];   // two planes of LX pairs x LY rows
    const unsigned b = xcd_block((unsigned)fm.per);
    if ((int)b >= fm.nwg) return;
    const int bx = (int)b % fm.ntx;
    const int rest = (int)b / fm.ntx;
    const int by = rest % fm.nty;
    const int bz = rest / fm.nty;
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const int IX = fm.LX - 2, IY = fm.LY - 2;
    const int P0 = bx * IX, Y0 = by * IY, Z0 = bz * fm.ZC;
    const int X0 = 2 * P0;
    const int X1 = min(2 * (P0 + IX), n0), Y1 = min(Y0 + IY, n1), Z1 = min(Z0 + fm.ZC, n2);
    const int tid = threadIdx.x;
    const int lx = tid % fm.LX, ly = tid / fm.LX;
    const int p = P0 - 1 + lx, y = Y0 - 1 + ly;
    const int W = 2 * fm.LX, slot = W * fm.LY;
    for (int q = tid; q < 2 * slot; q += blockDim.x) red[q] = 0.0;

    const bool in_x = lx >= 1 && lx <= IX && 2 * p < n0;
    const bool in_y = ly >= 1 && ly <= IY && y < n1;
    const bool interior = in_x && in_y;
    // ring lanes: the column left or right of the tile, or the row below or
    // above it (ring_col < 0: whichever column of the pair is red)
    bool ring = false;
    int ring_col = -1;
    if (in_y && lx == 0 && X0 > 0) { ring = true; ring_col = X0 - 1; }
    if (in_y && lx == IX + 1 && X1 < n0) { ring = true; ring_col = X1; }
    if (in_x && ((ly == 0 && Y0 > 0) || (ly == IY + 1 && Y1 < n1))) ring = true;
    const int xo = ly * W - (X0 - 2);   // LDS offset of (x, y) is xo + x
    __syncthreads();

    double r1 = 0.0, r2 = 0.0;   // own red values of the last two steps
    for (int z = (Z0 > 0 ? Z0 - 1 : 0); z <= Z1; ++z) {
        const int c = 2 * p + ((y + z) & 1);
        double rz = 0.0;
        const bool do_red = z < n2 && c < n0 &&
                            (interior || (ring && z >= Z0 && z < Z1 && (ring_col < 0 || ring_col == c)));
        if (do_red) {
            const long long idx = lin(g, c, y, z);
            const double x0 = pin[idx];
            rz = x0;
            if (!dirichlet_at(g, c, y, z, nullptr)) {
                const Stencil<3> sn = stencil<3, true>(g, c, y, z, idx);
                const double Ki = K[idx];
                const double f = gv[idx];
                double Kn[6], pn[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    Kn[q] = K[sn.jn[q]];
                    pn[q] = pin[sn.jn[q]];
                }
                rz = ngs_point<MODEL, SINK, 3>(g, L, st.a, beta, lambdaU, sn, Ki, Kn, pn, f, x0, c,
                                               y, z, idx, 0);
            }
            red[(z & 1) * slot + xo + c] = rz;
            if (interior && z >= Z0 && z < Z1) pout[idx] = rz;
        }
        const int zb = z - 1;
        if (interior && zb >= Z0 && zb < Z1 && c < n0) {
            const long long idx = lin(g, c, y, zb);
            const double x0 = pin[idx];
            double v = x0;
            if (!dirichlet_at(g, c, y, zb, nullptr)) {
                const Stencil<3> sn = stencil<3, true>(g, c, y, zb, idx);
                const double Ki = K[idx];
                const double f = gv[idx];
                double Kn[6], pn[6];
#pragma unroll
                for (int q = 0; q < 6; ++q) Kn[q] = K[sn.jn[q]];
                const double *sl = red + (zb & 1) * slot + xo + c;
                pn[0] = sl[-1];
                pn[1] = sl[1];
                pn[2] = sl[-W];
                pn[3] = sl[W];
                pn[4] = r2;
                pn[5] = rz;
                v = ngs_point<MODEL, SINK, 3>(g, L, st.a, beta, lambdaU, sn, Ki, Kn, pn, f, x0, c,
                                              y, zb, idx, 1);
            }
            pout[idx] = v;
        }
        r2 = r1;
        r1 = rz;
        __syncthreads();
    }
}

// The update of unknown (i, j, k) at idx (axis-0 neighbours at xl, xl + 1),
// its stencil gathered through raw buffer loads with 32-bit offsets
// (off-row neighbours outside the level read 0 and have coefficient 0; the
// axis-0 pair reads the padding at the row's end).
template <int MODEL, bool SINK, int DIM>
__device__ __forceinline__ void sweep_node_buf(const Geo &g, const Law &L, double a,
                                               const double *beta, double lambdaU,
                                               __amdgpu_buffer_rsrc_t rP, __amdgpu_buffer_rsrc_t rK,
                                               __amdgpu_buffer_rsrc_t rG, int i, int j, int k,
                                               long long idx, long long xl, int colour)
{
    const int vo = (int)idx * 8, vx = (int)xl * 8;
    const Stencil<DIM> sn = stencil_split<DIM>(g, i, j, k, idx, xl);
    const double Ki = buf_ld<double>(rK, vo), x0 = buf_ld<double>(rP, vo);
    const double f = buf_ld<double>(rG, vo);
    double Kn[2 * DIM], pn[2 * DIM];
    const v2f64 kx = buf_ld2(rK, vx, 0.0), px = buf_ld2(rP, vx, 0.0);
    Kn[0] = kx.x;
    Kn[1] = kx.y;
    pn[0] = px.x;
    pn[1] = px.y;
#pragma unroll
    for (int l = 1; l < DIM; ++l) {
        const int so = g.stride[l] * 8;
        Kn[2 * l] = buf_ld<double>(rK, vo - so);
        pn[2 * l] = buf_ld<double>(rP, vo - so);
        Kn[2 * l + 1] = buf_ld<double>(rK, vo + so);
        pn[2 * l + 1] = buf_ld<double>(rP, vo + so);
    }
    buf_st(rP, vo, ngs_point<MODEL, SINK, DIM>(g, L, a, beta, lambdaU, sn, Ki, Kn, pn, f, x0, i, j,
                                               k, idx, colour));
}

// One colour of a red-black sweep, one node per lane.  BUF (levels whose
// arrays stay below 2 GiB): the stencil is gathered through raw buffer loads
// with 32-bit offsets (off-row neighbours outside the level read 0 and have
// coefficient 0; the axis-0 pair reads the padding at the row's end).
template <int MODEL, bool SINK, int DIM, bool BUF>
__global__ __launch_bounds__(256) void k_sweep(Geo g, Law L, Step st, const double *beta,
                                               double lambdaU, const double *K, const double *gv,
                                               double *psi, int colour, ColourMap cm)
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
    // parity-split row: node i at ih (+ xh if odd); its left neighbour i - 1
    // at ih (i odd) or xh + ih - 1 (i even), the right one just after it
    const long long rb = (long long)j * g.stride[1] + (long long)k * g.stride[2];
    const long long idx = rb + ih + (par ? g.xh : 0);
    const long long xl = rb + ih + (par ? 0 : g.xh - 1);
    if constexpr (BUF) {
        const long long bytes = (g.N + 32) * (long long)sizeof(double);   // + padding
        sweep_node_buf<MODEL, SINK, DIM>(g, L, st.a, beta, lambdaU, buf_rsrc(psi, bytes),
                                         buf_rsrc(K, bytes), buf_rsrc(gv, bytes), i, (int)j,
                                         (int)k, idx, xl, colour);
    } else {
        ngs_cell_at<MODEL, SINK, DIM>(g, L, st.a, beta, lambdaU, K, gv, psi, i, (int)j, (int)k, idx,
                                      xl, colour);
    }
}

// One colour of a red-black sweep, two nodes of that colour per lane: half-row
// positions 2q and 2q + 1 (nodes i and i + 2), through raw buffer loads as in
// k_sweep (levels below 2 GiB).  Own values, g and each off-row direction are
// one 16-byte load per array, the three axis-0 neighbours (in the other half)
// a pair and a single.  Both stencils are reduced to their point problems
// before the first solve starts, so the second node holds three values, not
// its stencil, through the first solve; the solves run one after the other.
// The per-node arithmetic is that of k_sweep; the kappa rule is CONST or REL
// (the launcher sends the Remark's rule to k_sweep).  Slots: (xh + 1) / 2 per
// row.
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(256) void k_sweep_pair(Geo g, Law L, Step st, const double *beta,
                                                    double lambdaU, const double *K,
                                                    const double *gv, double *psi, int colour,
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
    const int len = par ? g.n[0] - g.xh : g.xh;   // nodes of this parity in the row
    if (2 * q >= len) return;
    const bool has_b = 2 * q + 1 < len;
    const int ia = 4 * q + par;                   // nodes ia and ia + 2
    const long long rb = (long long)j * g.stride[1] + (long long)k * g.stride[2];
    const long long idx = rb + (par ? g.xh : 0) + 2 * q;
    const long long xl = rb + (par ? 0 : g.xh - 1) + 2 * q;   // ia - 1, ia + 1, ia + 3
    const bool dir_a = dirichlet_t<DIM>(g, ia, (int)j, (int)k);
    const bool dir_b = !has_b || dirichlet_t<DIM>(g, ia + 2, (int)j, (int)k);
    if (dir_a && dir_b) return;
    const long long bytes = (g.N + 32) * (long long)sizeof(double);   // + padding
    const __amdgpu_buffer_rsrc_t rP = buf_rsrc(psi, bytes), rK = buf_rsrc(K, bytes),
                                 rG = buf_rsrc(gv, bytes);
    const int vo = (int)idx * 8, vx = (int)xl * 8;
    const v2f64 P = buf_ld2(rP, vo, 0.0), KK = buf_ld2(rK, vo, 0.0), G2 = buf_ld2(rG, vo, 0.0);
    const v2f64 PX = buf_ld2(rP, vx, 0.0), KX = buf_ld2(rK, vx, 0.0);
    const double PX2 = buf_ld<double>(rP, vx + 16), KX2 = buf_ld<double>(rK, vx + 16);
    constexpr int NO = 2 * (DIM - 1);
    v2f64 Po[NO > 0 ? NO : 1], Ko[NO > 0 ? NO : 1];
#pragma unroll
    for (int l = 1; l < DIM; ++l) {
        const int so = g.stride[l] * 8;
        Po[2 * l - 2] = buf_ld2(rP, vo - so, 0.0);
        Ko[2 * l - 2] = buf_ld2(rK, vo - so, 0.0);
        Po[2 * l - 1] = buf_ld2(rP, vo + so, 0.0);
        Ko[2 * l - 1] = buf_ld2(rK, vo + so, 0.0);
    }
    const double pw[3] = {PX.x, PX.y, PX2}, kw[3] = {KX.x, KX.y, KX2};
    PointEq e[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int i = ia + 2 * a;
        const Stencil<DIM> sn = stencil_split<DIM>(g, i, (int)j, (int)k, idx + a, xl + a);
        double Kn[2 * DIM], pn[2 * DIM];
        Kn[0] = kw[a];
        Kn[1] = kw[a + 1];
        pn[0] = pw[a];
        pn[1] = pw[a + 1];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            Kn[2 + o] = a ? Ko[o].y : Ko[o].x;
            pn[2 + o] = a ? Po[o].y : Po[o].x;
        }
        e[a] = ngs_reduce<SINK, DIM, false>(g, L, beta, lambdaU, sn, a ? KK.y : KK.x, Kn, pn,
                                     a ? G2.y : G2.x, a ? P.y : P.x, i, (int)j, (int)k, colour);
    }
    const double xa = dir_a ? P.x : ngs_solve<MODEL, SINK>(g, L, st.a, e[0], P.x, idx);
    __builtin_amdgcn_sched_barrier(0);
    if (!has_b) {
        buf_st(rP, vo, xa);
        return;
    }
    const double xb = dir_b ? P.y : ngs_solve<MODEL, SINK>(g, L, st.a, e[1], P.y, idx + 1);
    buf_st2(rP, vo, xa, xb);
}

// The last colour pass of a pre-smoothing (colour 1) fused with the defect of
// the nodes it updates: k_sweep_pair's update, then g - N(psi) at both nodes
// (0 at Dirichlet nodes) from the new values and the neighbours already in
// registers (all of the other colour, unchanged by this pass), stored into d,
// and their max-norm folded into norm_bits.  The defect arithmetic is
// defect_at, as in k_residual_pair.  Every lane reaches the block reduction.
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(256) void k_sweep_pair_defect(Geo g, Law L, Step st,
                                                           const double *beta, const double *K,
                                                           const double *gv, double *psi,
                                                           int colour, ColourMap cm, double *d,
                                                           unsigned long long *norm_bits)
{
    double v = 0.0;
    const unsigned long long t =
        (unsigned long long)xcd_block_dir(gridDim.x / 8u, colour & 1) * blockDim.x + threadIdx.x;
    unsigned row = 0;
    int q = 0;
    unsigned j = 0, k = 0;
    int len = 0;
    if (t < cm.total) {
        row = udiv((unsigned)t, cm.dH);
        q = (int)((unsigned)(t - (unsigned long long)row * cm.H));
        if (DIM == 3) {
            k = udiv(row, cm.dN1);
            j = row - k * cm.n1;
        } else if (DIM == 2) {
            j = row;
        }
        len = ((j + k + colour) & 1) ? g.n[0] - g.xh : g.xh;
    }
    if (2 * q < len) {
        const int par = (int)((j + k + colour) & 1);
        const bool has_b = 2 * q + 1 < len;
        const int ia = 4 * q + par;
        const long long rb = (long long)j * g.stride[1] + (long long)k * g.stride[2];
        const long long idx = rb + (par ? g.xh : 0) + 2 * q;
        const long long xl = rb + (par ? 0 : g.xh - 1) + 2 * q;
        const bool dir_a = dirichlet_t<DIM>(g, ia, (int)j, (int)k);
        const bool dir_b = !has_b || dirichlet_t<DIM>(g, ia + 2, (int)j, (int)k);
        const long long bytes = (g.N + 32) * (long long)sizeof(double);
        const __amdgpu_buffer_rsrc_t rP = buf_rsrc(psi, bytes), rK = buf_rsrc(K, bytes),
                                     rG = buf_rsrc(gv, bytes), rD = buf_rsrc(d, bytes);
        const int vo = (int)idx * 8, vx = (int)xl * 8;
        const v2f64 P = buf_ld2(rP, vo, 0.0), KK = buf_ld2(rK, vo, 0.0),
                    G2 = buf_ld2(rG, vo, 0.0);
        const v2f64 PX = buf_ld2(rP, vx, 0.0), KX = buf_ld2(rK, vx, 0.0);
        const double PX2 = buf_ld<double>(rP, vx + 16), KX2 = buf_ld<double>(rK, vx + 16);
        constexpr int NO = 2 * (DIM - 1);
        v2f64 Po[NO > 0 ? NO : 1], Ko[NO > 0 ? NO : 1];
#pragma unroll
        for (int l = 1; l < DIM; ++l) {
            const int so = g.stride[l] * 8;
            Po[2 * l - 2] = buf_ld2(rP, vo - so, 0.0);
            Ko[2 * l - 2] = buf_ld2(rK, vo - so, 0.0);
            Po[2 * l - 1] = buf_ld2(rP, vo + so, 0.0);
            Ko[2 * l - 1] = buf_ld2(rK, vo + so, 0.0);
        }
        const double pw[3] = {PX.x, PX.y, PX2}, kw[3] = {KX.x, KX.y, KX2};
        double xnew[2] = {P.x, P.y};
        if (!(dir_a && dir_b)) {
            PointEq e[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int i = ia + 2 * a;
                const Stencil<DIM> sn = stencil_split<DIM>(g, i, (int)j, (int)k, idx + a, xl + a);
                double Kn[2 * DIM], pn[2 * DIM];
                Kn[0] = kw[a];
                Kn[1] = kw[a + 1];
                pn[0] = pw[a];
                pn[1] = pw[a + 1];
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    Kn[2 + o] = a ? Ko[o].y : Ko[o].x;
                    pn[2 + o] = a ? Po[o].y : Po[o].x;
                }
                e[a] = ngs_reduce<SINK, DIM, false>(g, L, beta, 0.0, sn, a ? KK.y : KK.x, Kn, pn,
                                                    a ? G2.y : G2.x, a ? P.y : P.x, i, (int)j,
                                                    (int)k, colour);
            }
            if (!dir_a) xnew[0] = ngs_solve<MODEL, SINK>(g, L, st.a, e[0], P.x, idx);
            __builtin_amdgcn_sched_barrier(0);
            if (!dir_b) xnew[1] = ngs_solve<MODEL, SINK>(g, L, st.a, e[1], P.y, idx + 1);
            if (has_b) buf_st2(rP, vo, xnew[0], xnew[1]);
            else buf_st(rP, vo, xnew[0]);
        }
        // the defect of both nodes at their new values
        double bz = 0.0;
        if (SINK && DIM > 1) bz = beta[DIM == 2 ? j : k];
        double cfo[NO > 0 ? NO : 1];
#pragma unroll
        for (int o = 0; o < NO; ++o) cfo[o] = offrow_cf(g, o, o < 2 ? (int)j : (int)k);
        double r[2] = {0.0, 0.0};
        const double gs[2] = {G2.x, G2.y}, Ks_[2] = {KK.x, KK.y};
        const bool dirs[2] = {dir_a, dir_b};
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            if (dirs[a]) continue;
            double po[NO > 0 ? NO : 1], ko[NO > 0 ? NO : 1];
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                po[o] = a ? Po[o].y : Po[o].x;
                ko[o] = a ? Ko[o].y : Ko[o].x;
            }
            r[a] = defect_at<MODEL, SINK, DIM>(g, L, st.a, beta, bz, ia + 2 * a, idx + a, xnew[a],
                                               Ks_[a], gs[a], pw[a], pw[a + 1], kw[a], kw[a + 1],
                                               po, ko, cfo);
        }
        if (has_b) buf_st2(rD, vo, r[0], r[1]);
        else buf_st(rD, vo, r[0]);
        const double a0 = fabs(r[0]), a1 = fabs(r[1]);
        v = (a1 > a0 || a1 != a1) ? a1 : a0;
    }
    v = block_max(v);
    if (threadIdx.x == 0) {
        const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
        if (bits > __hip_atomic_load(norm_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(norm_bits, bits);
    }
}

// The defect of one colour's nodes (the colour the fused pass did not
// update), two per lane with k_sweep_pair's slots; d and the max-norm as in
// k_residual_pair.
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(256) void k_defect_colour(Geo g, Law L, Step st, const double *beta,
                                                       const double *K, const double *gv,
                                                       const double *psi, int colour, ColourMap cm,
                                                       double *d, unsigned long long *norm_bits)
{
    double v = 0.0;
    const unsigned long long t =
        (unsigned long long)xcd_block(gridDim.x / 8u) * blockDim.x + threadIdx.x;
    unsigned j = 0, k = 0;
    int q = 0, len = 0;
    if (t < cm.total) {
        const unsigned row = udiv((unsigned)t, cm.dH);
        q = (int)((unsigned)(t - (unsigned long long)row * cm.H));
        if (DIM == 3) {
            k = udiv(row, cm.dN1);
            j = row - k * cm.n1;
        } else if (DIM == 2) {
            j = row;
        }
        len = ((j + k + colour) & 1) ? g.n[0] - g.xh : g.xh;
    }
    if (2 * q < len) {
        const int par = (int)((j + k + colour) & 1);
        const bool has_b = 2 * q + 1 < len;
        const int ia = 4 * q + par;
        const long long rb = (long long)j * g.stride[1] + (long long)k * g.stride[2];
        const long long idx = rb + (par ? g.xh : 0) + 2 * q;
        const long long xl = rb + (par ? 0 : g.xh - 1) + 2 * q;
        const double2_u P = load_pair(psi + idx), KK = load_pair(K + idx), G2 = load_pair(gv + idx);
        const double2_u PX = load_pair(psi + xl), KX = load_pair(K + xl);
        const double PX2 = psi[xl + 2], KX2 = K[xl + 2];
        constexpr int NO = 2 * (DIM - 1);
        double2_u Po[NO > 0 ? NO : 1], Ko[NO > 0 ? NO : 1];
        double cfo[NO > 0 ? NO : 1];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            const int l = 1 + o / 2;
            const int cl = l == 1 ? (int)j : (int)k;
            cfo[o] = offrow_cf(g, o, cl);
            const long long b = cfo[o] != 0.0 ? ((o & 1) ? g.stride[l] : -(long long)g.stride[l]) : 0;
            Po[o] = load_pair(psi + idx + b);
            Ko[o] = load_pair(K + idx + b);
        }
        double bz = 0.0;
        if (SINK && DIM > 1) bz = beta[DIM == 2 ? j : k];
        const double xs[2] = {P.x, P.y}, Ks_[2] = {KK.x, KK.y}, gs[2] = {G2.x, G2.y};
        const double pw[3] = {PX.x, PX.y, PX2}, kw[3] = {KX.x, KX.y, KX2};
        double r[2] = {0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int i = ia + 2 * a;
            if ((a == 1 && !has_b) || dirichlet_t<DIM>(g, i, (int)j, (int)k)) continue;
            double po[NO > 0 ? NO : 1], ko[NO > 0 ? NO : 1];
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                po[o] = a ? Po[o].y : Po[o].x;
                ko[o] = a ? Ko[o].y : Ko[o].x;
            }
            r[a] = defect_at<MODEL, SINK, DIM>(g, L, st.a, beta, bz, i, idx + a, xs[a], Ks_[a],
                                               gs[a], pw[a], pw[a + 1], kw[a], kw[a + 1], po, ko,
                                               cfo);
        }
        if (has_b) store_pair(d + idx, r[0], r[1]);
        else d[idx] = r[0];
        const double a0 = fabs(r[0]), a1 = fabs(r[1]);
        v = (a1 > a0 || a1 != a1) ? a1 : a0;
    }
    v = block_max(v);
    if (threadIdx.x == 0) {
        const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
        if (bits > __hip_atomic_load(norm_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(norm_bits, bits);
    }
}

// One colour of a red-black sweep of a 3-D level, marching along axis 2 with
// the other colour staged in LDS.  A work-group owns kZmRows rows (axis 1) x
// 128 positions (one segment of the colour's half-rows) x zc planes; lane q of
// row ly updates positions 2q and 2q + 1 of the segment.  Every stencil
// neighbour of a node is of the other colour: its axis-0 neighbours sit in the
// other half of its own row, its axis-1 and axis-2 neighbours at its own
// position in the other-colour half of the adjacent rows.  The LDS ring holds,
// for the planes z - 1, z, z + 1, the other-colour psi and K* of the rows
// j0 - 1 .. j0 + kZmRows over positions -1 .. 128 of the segment, filled with
// coalesced loads; plane z + 2 (and the node's own psi, K*, g of plane z + 1)
// are loaded into registers while plane z is solved.  Each value of the other
// colour is fetched from memory about 1.5 times (rows of the halo), not 6.
// Half-rows of 128 s or 128 s + 1 positions only (n0 = 256 s or 256 s + 1):
// the one position past the last segment (the node n0 - 1) is updated after
// the march by the last segment's group, from global memory.  The per-node
// arithmetic is that of k_sweep; kappa CONST or REL.
constexpr int kZmRows = 4;
constexpr int kZmW = 132;   // LDS row: position -1 at index 1 (pairs 16-byte aligned)

struct ZmMap {
    int nsx, nsy, ncz, zc;   // segments, row stripes, plane chunks, planes per chunk
    int nwg, per;            // work-groups, logical groups per XCD
};

template <int MODEL, bool SINK>
__global__ __launch_bounds__(256) void k_sweep_zm(Geo g, Law L, Step st, const double *beta,
                                                  const double *K, const double *gv, double *psi,
                                                  int colour, ZmMap zm)
{
    __shared__ double sP[3][kZmRows + 2][kZmW], sK[3][kZmRows + 2][kZmW];
    const unsigned b = xcd_block_dir((unsigned)zm.per, colour & 1);
    if ((int)b >= zm.nwg) return;
    const int sx = (int)b % zm.nsx;
    const int rest = (int)b / zm.nsx;
    const int sy = rest % zm.nsy, cz = rest / zm.nsy;
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const int xh = g.xh;
    const int j0 = sy * kZmRows, z0 = cz * zm.zc, z1 = min(z0 + zm.zc, n2);
    const int tid = threadIdx.x, ly = tid >> 6, q = tid & 63;
    const int j = j0 + ly;
    const int p0 = 128 * sx;   // first position of the segment
    const long long bytes = (g.N + 32) * (long long)sizeof(double);
    const __amdgpu_buffer_rsrc_t rP = buf_rsrc(psi, bytes), rK = buf_rsrc(K, bytes),
                                 rG = buf_rsrc(gv, bytes);
    const long long s1 = g.stride[1], s2 = g.stride[2];

    // halo element f < (kZmRows + 2) * 130 of plane z: row j0 - 1 + f / 130,
    // position p0 - 1 + f % 130 of that row's other-colour half
    constexpr int NF = (kZmRows + 2) * 130, NU = (NF + 255) / 256;
    auto fetch = [&](int z, double *vp, double *vk) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int f = tid + 256 * u;
            const int rr = f / 130, e = f - rr * 130;
            const int jj = j0 - 1 + rr, pos = p0 - 1 + e;
            const int par = (jj + z + colour + 1) & 1;   // other colour's parity of i in the row
            const int len = par ? n0 - xh : xh;
            double a = 0.0, c = 0.0;
            if (f < NF && jj >= 0 && jj < n1 && z >= 0 && z < n2 && pos >= 0 && pos < len) {
                const int off = (int)(((long long)jj * s1 + (long long)z * s2 + (par ? xh : 0) + pos) * 8);
                a = buf_ld<double>(rP, off);
                c = buf_ld<double>(rK, off);
            }
            vp[u] = a;
            vk[u] = c;
        }
    };
    auto stash = [&](int slot, const double *vp, const double *vk) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int f = tid + 256 * u;
            if (f < NF) {
                const int rr = f / 130, e = f - rr * 130;
                sP[slot][rr][e + 1] = vp[u];
                sK[slot][rr][e + 1] = vk[u];
            }
        }
    };
    // own values (psi, K*, g pairs) of the lane's two nodes in plane z
    auto own = [&](int z, v2f64 &P, v2f64 &KK, v2f64 &G2) {
        if (j < n1 && z < n2) {
            const int par = (j + z + colour) & 1;
            const int vo = (int)(((long long)j * s1 + (long long)z * s2 + (par ? xh : 0) + p0 + 2 * q) * 8);
            P = buf_ld2(rP, vo, 0.0);
            KK = buf_ld2(rK, vo, 0.0);
            G2 = buf_ld2(rG, vo, 0.0);
        }
    };

    double vp[NU], vk[NU];
    for (int z = z0 - 1; z <= z0 + 1; ++z) {
        fetch(z, vp, vk);
        stash((z + 3) % 3, vp, vk);
    }
    v2f64 P = {0.0, 0.0}, KK = {0.0, 0.0}, G2 = {0.0, 0.0};
    own(z0, P, KK, G2);
    __syncthreads();

    for (int z = z0; z < z1; ++z) {
        const bool more = z + 1 < z1;   // a next plane in the chunk
        if (more) fetch(z + 2, vp, vk);
        v2f64 Pn = P, Kn2 = KK, Gn = G2;
        if (more) own(z + 1, Pn, Kn2, Gn);
        if (j < n1) {
            const int par = (j + z + colour) & 1;
            const int ia = 2 * (p0 + 2 * q) + par;   // nodes ia and ia + 2
            const bool dir_a = dirichlet_at(g, ia, j, z, nullptr);
            const bool dir_b = dirichlet_at(g, ia + 2, j, z, nullptr);
            if (!(dir_a && dir_b)) {
                const int sm = (z + 2) % 3, sc = z % 3, sp = (z + 1) % 3;
                PointEq e[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int i = ia + 2 * a;
                    // LDS index of position p0 - 1 + t is t + 1
                    const int xo = 2 * q + par + a + 1, yo = 2 * q + a + 2;
                    const Stencil<3> sn = stencil_split<3>(g, i, j, z, 0, 0);
                    double Kn[6], pn[6];
                    Kn[0] = sK[sc][ly + 1][xo];
                    pn[0] = sP[sc][ly + 1][xo];
                    Kn[1] = sK[sc][ly + 1][xo + 1];
                    pn[1] = sP[sc][ly + 1][xo + 1];
                    Kn[2] = sK[sc][ly][yo];
                    pn[2] = sP[sc][ly][yo];
                    Kn[3] = sK[sc][ly + 2][yo];
                    pn[3] = sP[sc][ly + 2][yo];
                    Kn[4] = sK[sm][ly + 1][yo];
                    pn[4] = sP[sm][ly + 1][yo];
                    Kn[5] = sK[sp][ly + 1][yo];
                    pn[5] = sP[sp][ly + 1][yo];
                    e[a] = ngs_reduce<SINK, 3, false>(g, L, beta, 0.0, sn, a ? KK.y : KK.x, Kn, pn,
                                                      a ? G2.y : G2.x, a ? P.y : P.x, i, j, z,
                                                      colour);
                    // one node's twelve LDS values live at a time
                    __builtin_amdgcn_sched_barrier(0);
                }
                const long long idx =
                    (long long)j * s1 + (long long)z * s2 + (par ? xh : 0) + p0 + 2 * q;
                const double xa = dir_a ? P.x : ngs_solve<MODEL, SINK>(g, L, st.a, e[0], P.x, idx);
                const double xb =
                    dir_b ? P.y : ngs_solve<MODEL, SINK>(g, L, st.a, e[1], P.y, idx + 1);
                buf_st2(rP, (int)(idx * 8), xa, xb);
            }
        }
        __syncthreads();                        // plane z - 1 no longer read
        if (more) stash((z + 2) % 3, vp, vk);   // its slot takes plane z + 2
        __syncthreads();
        P = Pn;
        KK = Kn2;
        G2 = Gn;
    }

    // the node past the last segment (n0 - 1 when n0 = 256 s + 1)
    if (sx == zm.nsx - 1) {
        const int pe = 128 * zm.nsx;
        for (int t = tid; t < kZmRows * (z1 - z0); t += 256) {
            const int jj = j0 + (t % kZmRows), z = z0 + t / kZmRows;
            if (jj >= n1) continue;
            const int par = (jj + z + colour) & 1;
            if (pe >= (par ? n0 - xh : xh)) continue;
            const int i = 2 * pe + par;
            if (dirichlet_at(g, i, jj, z, nullptr)) continue;
            const long long rb = (long long)jj * s1 + (long long)z * s2;
            sweep_node_buf<MODEL, SINK, 3>(g, L, st.a, beta, 0.0, rP, rK, rG, i, jj, z,
                                           rb + pe + (par ? xh : 0), rb + pe + (par ? 0 : xh - 1),
                                           colour);
        }
    }
}

// Whole sweeps of a tiny level in one work-group (the coarsest levels, where
// launch latency, not work, dominates).
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(256) void k_sweep_small(Geo g, Law L, Step st, const double *beta,
                                                     double lambdaU, const double *K,
                                                     const double *gv, double *psi, int nsweeps)
{
    const int N = (int)g.N;
    for (int s = 0; s < nsweeps; ++s) {
        for (int colour = 0; colour < 2; ++colour) {
            for (int t = threadIdx.x; t < N; t += blockDim.x) {
                int i = t % g.n[0];
                int r = t / g.n[0];
                int j = r % g.n[1];
                int k = r / g.n[1];
                if (((i + j + k) & 1) != colour) continue;
                if (dirichlet_t<DIM>(g, i, j, k)) continue;
                ngs_cell<MODEL, SINK, DIM>(g, L, st.a, beta, lambdaU, K, gv, psi, i, j, k, colour);
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// The cycle on the small levels of a grid in one work-group (levels of at most
// kTailNodes nodes): the same per-node operations as the multi-launch cycle,
// with work-group barriers between the steps instead of launches.
// ---------------------------------------------------------------------------

// n sweeps of a level; with exit set (the coarsest level) the loop stops after
// a sweep that moved no value by more than 4 ulp: the coarse problem is then
// solved to rounding, and further sweeps only move values within rounding.
template <int MODEL, bool SINK, int DIM>
__device__ void tail_sweeps64(const TailLevel &T, const Law &L, double a, int n, bool exit = false)
{
    const ColourMap cm = tail_cm(T);
    for (int sw = 0; sw < n; ++sw) {
        int changed = 0;
        for (int colour = 0; colour < 2; ++colour) {
            for (unsigned long long t = threadIdx.x; t < cm.total; t += blockDim.x) {
                int i, j, k;
                if (!colour_ijk(T.g, cm, t, colour, i, j, k)) continue;
                if (dirichlet_t<DIM>(T.g, i, j, k)) continue;
                changed |= ngs_cell<MODEL, SINK, DIM>(T.g, L, a, T.beta, T.lambdaU, T.K, T.gv,
                                                      T.psi, i, j, k, colour);
            }
            if (colour == 0 || !exit) __syncthreads();
            else if (!__syncthreads_or(changed)) return;
        }
    }
}

// Levels lds_from..last live in LDS for the duration of the cycle (psi, K*, g,
// d, psibar of each, with one zero element before and after every array for
// the padded stencils): K* and, for the top level, psi and g are copied in;
// the top level's psi is copied back (the only result used after the cycle;
// the top level's psibar and beta stay in global memory).
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(512) void k_vcycle_tail(const TailArgs *A, int top, int last, Law L,
                                                     Step st, int nu1, int nu2, int nuc,
                                                     int lds_from)
{
    extern __shared__ double lds[];
    __shared__ TailLevel SL[kMaxLevels];
    for (int l = top + (int)threadIdx.x; l <= last; l += (int)blockDim.x) SL[l] = A->lv[l];
    __syncthreads();
    if (lds_from <= last) {
        if (threadIdx.x == 0) {
            long long off = 0;
            for (int l = lds_from; l <= last; ++l) {
                const long long n = SL[l].g.N + 2;
                double **arr[5] = {&SL[l].psi, &SL[l].K, &SL[l].gv, &SL[l].d, &SL[l].psibar};
                for (int q = 0; q < 5; ++q) {
                    if (l == top && q == 4) continue;   // read-only, stays global
                    *arr[q] = lds + off + 1;
                    off += n;
                }
            }
        }
        __syncthreads();
        for (int l = lds_from; l <= last; ++l) {
            const TailLevel &G = A->lv[l], &S = SL[l];
            const long long N = S.g.N;
            for (long long t = threadIdx.x; t < N + 2; t += blockDim.x) {
                const long long u = t - 1;
                const bool in = u >= 0 && u < N;
                S.K[u] = in ? G.K[u] : 0.0;
                S.psi[u] = (in && l == top) ? G.psi[u] : 0.0;
                S.gv[u] = (in && l == top) ? G.gv[u] : 0.0;
                S.d[u] = 0.0;
                if (l != top) S.psibar[u] = 0.0;
            }
        }
        __syncthreads();
    }
    const double a = st.a;
    for (int l = top; l < last; ++l) {
        const TailLevel &F = SL[l], &C = SL[l + 1];
        tail_sweeps64<MODEL, SINK, DIM>(F, L, a, nu1);
        const NodeMap nf = tail_nm(F), nc = tail_nm(C);
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)F.g.N; t += blockDim.x) {
            int i, j, k;
            node_ijk(nf, t, i, j, k);
            double r = 0.0;
            if (!dirichlet_t<DIM>(F.g, i, j, k))
                r = F.gv[t] - apply_N_t<MODEL, SINK, DIM, true>(F.g, L, a, F.beta, F.K, F.psi, i, j, k,
                                                          (long long)t);
            F.d[t] = r;
        }
        __syncthreads();
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)C.g.N; t += blockDim.x) {
            int i, j, k;
            node_ijk(nc, t, i, j, k);
            restrict_at<DIM, double>(C.g, F.g, F.psi, F.d, C.psibar, C.gv, i, j, k);
        }
        __syncthreads();
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)C.g.N; t += blockDim.x) {
            int i, j, k;
            node_ijk(nc, t, i, j, k);
            if (!dirichlet_t<DIM>(C.g, i, j, k))
                C.gv[t] = apply_N_t<MODEL, SINK, DIM, true>(C.g, L, a, C.beta, C.K, C.psibar, i, j, k,
                                                      (long long)t) +
                          C.gv[t];
            C.psi[t] = C.psibar[t];
        }
        __syncthreads();
    }
    tail_sweeps64<MODEL, SINK, DIM>(SL[last], L, a, nuc, true);
    for (int l = last - 1; l >= top; --l) {
        const TailLevel &F = SL[l], &C = SL[l + 1];
        const NodeMap nf = tail_nm(F);
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)F.g.N; t += blockDim.x) {
            int i, j, k;
            node_ijk(nf, t, i, j, k);
            prolong_at<DIM, double>(F.g, C.g, C.psi, C.psibar, F.psi, i, j, k);
        }
        __syncthreads();
        tail_sweeps64<MODEL, SINK, DIM>(F, L, a, nu2);
    }
    if (top >= lds_from)
        for (long long t = threadIdx.x; t < SL[top].g.N; t += blockDim.x) A->lv[top].psi[t] = SL[top].psi[t];
}

// ---------------------------------------------------------------------------
// Defect d = g - N(psi) and its max-norm (step 2 of the FAS algorithm)
// ---------------------------------------------------------------------------

// Two nodes of the same parity per thread, side by side in one half of a
// parity-split row (positions 2q and 2q + 1 of the half: nodes i and i + 2):
// their own values, g, and each off-row neighbour direction are one 16-byte
// load per array, the three axis-0 neighbours (in the other half) a pair and
// a single load; the two theta chains overlap.  Each node's arithmetic is that
// of apply_N_t.  Slots: H = (n0 + 1) / 2 per row, the first (H + 1) / 2 for
// the even half, the rest for the odd half.
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(256) void k_residual_pair(Geo g, Law L, Step st, const double *beta,
                                                       const double *K, const double *gv,
                                                       const double *psi, double *d,
                                                       unsigned long long *norm_bits, ColourMap cm,
                                                       MpStart mp)
{
    double v = 0.0;
    const unsigned long long t =
        (unsigned long long)xcd_block(gridDim.x / 8u) * blockDim.x + threadIdx.x;
    if (t < cm.total) {
        const unsigned row = udiv((unsigned)t, cm.dH);
        const int slot = (int)((unsigned)(t - (unsigned long long)row * cm.H));
        const int H = g.xh, P0 = (H + 1) / 2;
        const int h = slot < P0 ? 0 : 1;
        const int q = slot - h * P0;
        const int half_len = h ? g.n[0] - H : H;
        const bool has_b = 2 * q + 1 < half_len;
        const int ia = 4 * q + h;                 // nodes ia and ia + 2
        int j = 0, k = 0;
        if (DIM == 3) {
            k = (int)udiv(row, cm.dN1);
            j = (int)row - k * (int)cm.n1;
        } else if (DIM == 2) {
            j = (int)row;
        }
        const long long rb = (long long)j * g.stride[1] + (long long)k * g.stride[2];
        const long long idx = rb + h * H + 2 * q;          // node ia; ia + 2 at idx + 1
        const long long xl = rb + (h ? 0 : H - 1) + 2 * q; // nodes ia - 1, ia + 1, ia + 3
        const double2_u P = load_pair(psi + idx), KK = load_pair(K + idx), G2 = load_pair(gv + idx);
        const double2_u PX = load_pair(psi + xl), KX = load_pair(K + xl);
        const double PX2 = psi[xl + 2], KX2 = K[xl + 2];
        // off-row neighbour pairs (the nodes themselves, coefficient 0, outside)
        constexpr int NO = 2 * (DIM - 1);
        double2_u Po[NO > 0 ? NO : 1], Ko[NO > 0 ? NO : 1];
        double cfo[NO > 0 ? NO : 1];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            const int l = 1 + o / 2;
            const int cl = l == 1 ? j : k;
            const bool up = o & 1;
            const bool ok = up ? cl < g.n[l] - 1 : cl > 0;
            const long long b = ok ? (up ? g.stride[l] : -(long long)g.stride[l]) : 0;
            Po[o] = load_pair(psi + idx + b);
            Ko[o] = load_pair(K + idx + b);
            cfo[o] = ok ? ((cl == 0 || cl == g.n[l] - 1) ? 1.0 : 0.5) * g.ih2[l] : 0.0;
        }
        double bz = 0.0;   // root density of the row (2-D, 3-D)
        if (SINK && DIM > 1) bz = beta[DIM == 2 ? j : k];
        const double xs[2] = {P.x, P.y}, Ks_[2] = {KK.x, KK.y}, gs[2] = {G2.x, G2.y};
        // axis-0 neighbours: left of ia, right of ia = left of ia + 2, right of ia + 2
        const double pw[3] = {PX.x, PX.y, PX2}, kw[3] = {KX.x, KX.y, KX2};
        double r[2] = {0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int i = ia + 2 * a;
            if ((a == 1 && !has_b) || dirichlet_t<DIM>(g, i, j, k)) continue;
            double po[NO > 0 ? NO : 1], ko[NO > 0 ? NO : 1];
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                po[o] = a ? Po[o].y : Po[o].x;
                ko[o] = a ? Ko[o].y : Ko[o].x;
            }
            r[a] = defect_at<MODEL, SINK, DIM>(g, L, st.a, beta, bz, i, idx + a, xs[a], Ks_[a],
                                               gs[a], pw[a], pw[a + 1], kw[a], kw[a + 1], po, ko,
                                               cfo);
        }
        if (d) {
            if (has_b) store_pair(d + idx, r[0], r[1]);
            else d[idx] = r[0];
        }
        if (mp.rhs) {
            if (has_b) {
                store_pair(mp.rhs + idx, (float)r[0], (float)r[1]);
                store_pair(mp.pb + idx, (float)xs[0], (float)xs[1]);
                store_pair(mp.dl + idx, 0.0f, 0.0f);
            } else {
                mp.rhs[idx] = (float)r[0];
                mp.pb[idx] = (float)xs[0];
                mp.dl[idx] = 0.0f;
            }
        }
        const double a0 = fabs(r[0]), a1 = fabs(r[1]);
        v = (a1 > a0 || a1 != a1) ? a1 : a0;
    }
    if (norm_bits) {
        v = block_max(v);
        if (threadIdx.x == 0) {
            const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
            if (bits > __hip_atomic_load(norm_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMax(norm_bits, bits);
        }
    }
}

// Size of the terms the defect of a node and its pointwise solve sum (|g|,
// a |theta|, the sink, xi |psi_i| and m_ij (|psi_i| + |psi_j|) per face),
// maximised over the unknowns: the scale of the defect's rounding floor (a
// one-ulp change of psi_i moves the defect by m_ii ulp(psi_i)).
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(256) void k_defect_scale(Geo g, Law L, Step st, const double *beta,
                                                      const double *K, const double *gv,
                                                      const double *psi, unsigned long long *out,
                                                      NodeMap nm)
{
    double v = 0.0;
    const unsigned long long t =
        (unsigned long long)xcd_block(gridDim.x / 8u) * blockDim.x + threadIdx.x;
    if (t < (unsigned long long)g.N) {
        int i, j, k;
        node_ijk(nm, t, i, j, k);
        if (!dirichlet_at(g, i, j, k, nullptr)) {
            const long long idx = (long long)t;
            const Stencil<DIM> sn = stencil<DIM>(g, i, j, k, idx);
            const double x = psi[idx], Ki = K[idx];
            double th;
            if constexpr (MODEL == kMulti) th = theta_only(L.soils[g.soil[idx]], x);
            else th = theta_only_t<MODEL>(L, x);
            v = fabs(gv[idx]) + fabs(st.a * th) + fabs(L.xi * x);
            if (SINK) {
                double fa, dfa;
                feddes(L, x, fa, dfa);
                v += fabs(beta[(DIM == 1) ? i : (DIM == 2 ? j : k)] * fa);
            }
#pragma unroll
            for (int q = 0; q < 2 * DIM; ++q)
                v += fabs(sn.cf[q] * (Ki + K[sn.jn[q]])) * (fabs(x) + fabs(psi[sn.jn[q]]));
        }
    }
    v = block_max(v);
    if (threadIdx.x == 0) atomicMax(out, (unsigned long long)__double_as_longlong(v));
}

// ---------------------------------------------------------------------------
// Transfers (section 3.2 steps 3, 4 and 6)
// ---------------------------------------------------------------------------

// g_H = N_H(psibar_H) + d_H (g_H holds d_H on entry), psi_H = psibar_H.
template <int MODEL, bool SINK, int DIM>
__global__ __launch_bounds__(256) void k_coarse_rhs(Geo g, Law L, Step st, const double *beta,
                                                    const double *K, const double *psibar,
                                                    double *gv, double *psi, NodeMap nm)
{
    const unsigned long long t =
        (unsigned long long)xcd_block(gridDim.x / 8u) * blockDim.x + threadIdx.x;
    if (t >= (unsigned long long)g.N) return;
    int i, j, k;
    node_ijk(nm, t, i, j, k);
    if (!dirichlet_t<DIM>(g, i, j, k))
        gv[t] = apply_N_t<MODEL, SINK, DIM, true>(g, L, st.a, beta, K, psibar, i, j, k, (long long)t) +
                gv[t];
    psi[t] = psibar[t];
}

// Root density of the Feddes-exponential sink on every level:
// beta(z) = Tp exp(-(Lz - z)/root_len) / Z, Z the trapezoidal integral of the
// exponential over the fine column, so that the column integral is Tp.
struct BetaArgs {
    int nlev;
    int nvert[kMaxLevels];
    double hvert[kMaxLevels];
    double *beta[kMaxLevels];
    double Lz, Tp, rl;
};

__global__ __launch_bounds__(256) void k_root_beta(BetaArgs a)
{
    __shared__ double part[256];
    const int n0 = a.nvert[0];
    const double h0 = a.hvert[0];
    double s = 0.0;
    for (int k = threadIdx.x; k < n0; k += blockDim.x) {
        double w = (k == 0 || k == n0 - 1) ? 0.5 : 1.0;
        s += w * h0 * exp(-(a.Lz - k * h0) / a.rl);
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
        __syncthreads();
    }
    const double Z = part[0];
    for (int l = 0; l < a.nlev; ++l)
        for (int k = threadIdx.x; k < a.nvert[l]; k += blockDim.x)
            a.beta[l][k] = a.Tp * exp(-(a.Lz - k * a.hvert[l]) / a.rl) / Z;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

void launch_root_beta(int nlev, const int *nvert, const double *hvert, double *const *beta,
                      double Lz, double Tp, double root_len, hipStream_t s)
{
    BetaArgs a;
    a.nlev = nlev;
    for (int l = 0; l < nlev; ++l) {
        a.nvert[l] = nvert[l];
        a.hvert[l] = hvert[l];
        a.beta[l] = beta[l];
    }
    a.Lz = Lz;
    a.Tp = Tp;
    a.rl = root_len;
    hipLaunchKernelGGL(k_root_beta, dim3(1), dim3(256), 0, s, a);
}

template <typename T>
static void relayout_t(const Geo &g, const T *src, T *dst, bool to_level, hipStream_t s)
{
    hipLaunchKernelGGL(k_relayout<T>, dim3((unsigned)((g.N + 255) / 256)), dim3(256), 0, s, g, src,
                       dst, to_level ? 1 : 0, make_fastdiv((unsigned)g.n[0]));
}

void launch_relayout(const Geo &g, const double *src, double *dst, bool to_level, hipStream_t s)
{
    relayout_t<double>(g, src, dst, to_level, s);
}

void launch_relayout_u8(const Geo &g, const unsigned char *src, unsigned char *dst, bool to_level,
                        hipStream_t s)
{
    relayout_t<unsigned char>(g, src, dst, to_level, s);
}

void launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u64, dim3((n + 63) / 64), dim3(64), 0, s, p, n, v);
}

void launch_setup_kstar(const Geo &g, const Law &law, const Step &st, const double *psi_n,
                        const double *psi_nm1, const double *Ks_field, double *K, double *psi,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_setup_kstar, node_grid(g), dim3(kBX, kBY), 0, s, g, law, st, psi_n,
                       psi_nm1, Ks_field, K, psi);
}

void launch_setup_g(const Geo &g, const Law &law, const Step &st, const double *psi_n,
                    const double *psi_nm1, const double *K, double *gvec, hipStream_t s)
{
    hipLaunchKernelGGL(k_setup_g, node_grid(g), dim3(kBX, kBY), 0, s, g, law, st, psi_n, psi_nm1,
                       K, gvec);
}

void launch_inject_u8(const Geo &gc, const Geo &gf, const unsigned char *vf, unsigned char *vc,
                      hipStream_t s)
{
    hipLaunchKernelGGL((k_inject_t<unsigned char>), node_grid(gc), dim3(kBX, kBY), 0, s, gc, gf,
                       vf, vc);
}

void launch_inject(const Geo &gc, const Geo &gf, const double *Kf, double *Kc, hipStream_t s)
{
    hipLaunchKernelGGL(k_inject, node_grid(gc), dim3(kBX, kBY), 0, s, gc, gf, Kf, Kc);
}

void launch_fw_coarse(const Geo &gc, const Geo &gf, const double *Kf, double *Kc, hipStream_t s)
{
    const dim3 grid(xcd_grid(((unsigned long long)gc.N + 255) / 256));
    const NodeMap nm = node_map(gc);
    if (gc.dim == 1)
        hipLaunchKernelGGL((k_fw_coarse<1>), grid, dim3(256), 0, s, gc, gf, Kf, Kc, nm);
    else if (gc.dim == 2)
        hipLaunchKernelGGL((k_fw_coarse<2>), grid, dim3(256), 0, s, gc, gf, Kf, Kc, nm);
    else
        hipLaunchKernelGGL((k_fw_coarse<3>), grid, dim3(256), 0, s, gc, gf, Kf, Kc, nm);
}

void launch_lambda_u(const Geo &g, const double *K, unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_lambda_u, node_grid(g), dim3(kBX, kBY), 0, s, g, K, out);
}

// Lane grid and chunk depth of the fused sweep (pairs x rows including the
// one-lane ring, planes per chunk); RS_FUSED_TILE="lx,ly,zc" overrides them.
void fused_tile(int *lx, int *ly, int *zc)
{
    *lx = 16; *ly = 16; *zc = 16;
    if (const char *e = getenv("RS_FUSED_TILE")) {
        int a, b, c;
        if (sscanf(e, "%d,%d,%d", &a, &b, &c) == 3 && a >= 3 && b >= 3 && c >= 1 && a * b <= 512) {
            *lx = a; *ly = b; *zc = c;
        }
    }
}

// The fused sweep is opt-in (RS_SWEEP=fused) until it beats the two-pass one.
bool fused_enabled()
{
    const char *e = getenv("RS_SWEEP");
    return e && strcmp(e, "fused") == 0;
}

// Two nodes per lane in the colour sweeps of the large buffer-path levels
// (at least 2^21 nodes: 129^3 takes 13.9 us per colour with two, 15.1 with
// one; on smaller levels the lane's two solves in sequence cost more than
// they save); RS_SWEEP=single keeps one node per lane on every level,
// RS_SWEEP=pair takes two on every buffer-path level.
bool pair_sweep_level(const Geo &g)
{
    const char *e = getenv("RS_SWEEP");
    if (e && strcmp(e, "single") == 0) return false;
    if (e && strcmp(e, "pair") == 0) return true;
    return g.N >= (1ll << 21);
}

// The z-marching LDS sweep: 3-D levels whose rows are split by parity into
// halves of 128 s and 128 s (+ 1) positions; planes per chunk from RS_ZM_ZC
// (default 16).
bool zm_level(const Geo &g)
{
    if (g.dim != 3 || g.xs != 1) return false;
    const int lo = g.n[0] - g.xh, hi = g.xh;   // odd and even half lengths
    return lo >= 128 && lo % 128 == 0 && hi - lo <= 1;
}

ZmMap zm_map(const Geo &g)
{
    ZmMap m;
    m.zc = 16;
    if (const char *e = getenv("RS_ZM_ZC")) {
        const int v = atoi(e);
        if (v >= 1 && v <= 64) m.zc = v;
    }
    m.nsx = (g.n[0] - g.xh) / 128;
    m.nsy = (g.n[1] + kZmRows - 1) / kZmRows;
    m.ncz = (g.n[2] + m.zc - 1) / m.zc;
    m.nwg = m.nsx * m.nsy * m.ncz;
    m.per = (m.nwg + 7) / 8;
    return m;
}

// Opt-in (RS_SWEEP=zm): at 257^3 it takes 134 / 143 / 165 us per colour with
// 8 / 16 / 32 planes per chunk against 91 us for k_sweep_pair.  The march
// serialises a group's planes behind two barriers each, the lanes of a group
// wait for its slowest Newton solve at every plane, and the 150 VGPRs it holds
// (prefetched plane, own values, two stencils) leave 3 waves per SIMD.
bool zm_enabled()
{
    const char *e = getenv("RS_SWEEP");
    return e && strcmp(e, "zm") == 0;
}

FusedMap fused_map(const Geo &g)
{
    FusedMap m;
    fused_tile(&m.LX, &m.LY, &m.ZC);
    const int pairs = (g.n[0] + 1) / 2;
    m.ntx = (pairs + m.LX - 3) / (m.LX - 2);
    m.nty = (g.n[1] + m.LY - 3) / (m.LY - 2);
    m.ntz = (g.n[2] + m.ZC - 1) / m.ZC;
    m.nwg = m.ntx * m.nty * m.ntz;
    m.per = (m.nwg + 7) / 8;
    return m;
}

struct SweepLaunch {
    const Geo &g; const Law &law; const Step &st; const double *beta; double lambdaU;
    const double *K; const double *gvec; double **psi; double **psi_alt; int nsweeps; hipStream_t s;
    template <int M, bool S, int D>
    void go()
    {
        if (g.N <= 1024) {
            hipLaunchKernelGGL((k_sweep_small<M, S, D>), dim3(1), dim3(256), 0, s, g, law, st,
                               beta, lambdaU, K, gvec, *psi, nsweeps);
            return;
        }
        if (D == 3 && psi_alt && *psi_alt && fused_enabled()) {
            FusedMap fm = fused_map(g);
            const size_t lds = sizeof(double) * 4 * (size_t)fm.LX * fm.LY;
            for (int sw = 0; sw < nsweeps; ++sw) {
                hipLaunchKernelGGL((k_sweep_fused<M, S>), dim3(8 * fm.per), dim3(fm.LX * fm.LY),
                                   lds, s, g,
                                   law, st, beta, lambdaU, K, gvec, *psi, *psi_alt, fm);
                double *t = *psi;
                *psi = *psi_alt;
                *psi_alt = t;
            }
            return;
        }
        ColourMap cm = colour_map(g);
        dim3 grid(xcd_grid((cm.total + 255) / 256));
        const bool buf = buffer_ok(g, sizeof(double));
        if (D == 3 && buf && law.kappa_rule != kKappaRemark && zm_level(g) && zm_enabled()) {
            const ZmMap zm = zm_map(g);
            for (int sw = 0; sw < nsweeps; ++sw)
                for (int colour = 0; colour < 2; ++colour)
                    hipLaunchKernelGGL((k_sweep_zm<M, S>), dim3(8 * zm.per), dim3(256), 0, s, g,
                                       law, st, beta, K, gvec, *psi, colour, zm);
            return;
        }
        if (buf && law.kappa_rule != kKappaRemark && pair_sweep_level(g)) {
            ColourMap pm = cm;
            pm.H = (cm.H + 1) / 2;
            pm.dH = make_fastdiv(pm.H);
            pm.total = (unsigned long long)pm.H * g.n[1] * g.n[2];
            dim3 pgrid(xcd_grid((pm.total + 255) / 256));
            for (int sw = 0; sw < nsweeps; ++sw)
                for (int colour = 0; colour < 2; ++colour)
                    hipLaunchKernelGGL((k_sweep_pair<M, S, D>), pgrid, dim3(256), 0, s, g, law, st,
                                       beta, lambdaU, K, gvec, *psi, colour, pm);
            return;
        }
        for (int sw = 0; sw < nsweeps; ++sw)
            for (int colour = 0; colour < 2; ++colour) {
                if (buf)
                    hipLaunchKernelGGL((k_sweep<M, S, D, true>), grid, dim3(256), 0, s, g, law, st,
                                       beta, lambdaU, K, gvec, *psi, colour, cm);
                else
                    hipLaunchKernelGGL((k_sweep<M, S, D, false>), grid, dim3(256), 0, s, g, law, st,
                                       beta, lambdaU, K, gvec, *psi, colour, cm);
            }
    }
};

// A pre-smoothing of nsweeps sweeps on a level that runs the pair sweep, with
// the defect of the iterate it leaves formed on the way: the last colour pass
// also forms the defect of the nodes it updates (k_sweep_pair_defect), one
// more pass that of the other colour (k_defect_colour); d and norm_bits get
// what k_residual_pair would give after the sweeps.  RS_DEFECT_FUSE=0 turns
// it off.
bool sweep_defect_enabled()
{
    const char *e = getenv("RS_DEFECT_FUSE");
    return !(e && strcmp(e, "0") == 0);
}

struct SweepDefectLaunch {
    const Geo &g; const Law &law; const Step &st; const double *beta; const double *K;
    const double *gvec; double *psi; int nsweeps; double *d; unsigned long long *norm_bits;
    hipStream_t s; int phase;
    template <int M, bool S, int D>
    void go()
    {
        ColourMap pm = colour_map(g);
        pm.H = (pm.H + 1) / 2;
        pm.dH = make_fastdiv(pm.H);
        pm.total = (unsigned long long)pm.H * g.n[1] * g.n[2];
        const dim3 pgrid(xcd_grid((pm.total + 255) / 256));
        if (phase == 0) {   // every colour pass but the last
            for (int p = 0; p + 1 < 2 * nsweeps; ++p)
                hipLaunchKernelGGL((k_sweep_pair<M, S, D>), pgrid, dim3(256), 0, s, g, law, st,
                                   beta, 0.0, K, gvec, psi, p & 1, pm);
            return;
        }
        hipLaunchKernelGGL((k_sweep_pair_defect<M, S, D>), pgrid, dim3(256), 0, s, g, law, st,
                           beta, K, gvec, psi, 1, pm, d, norm_bits);
        hipLaunchKernelGGL((k_defect_colour<M, S, D>), pgrid, dim3(256), 0, s, g, law, st, beta, K,
                           gvec, psi, 0, pm, d, norm_bits);
    }
};

struct CoarseRhsLaunch {
    const Geo &g; const Law &law; const Step &st; const double *beta; const double *K;
    const double *psibar; double *gvec; double *psi; hipStream_t s;
    template <int M, bool S, int D>
    void go()
    {
        hipLaunchKernelGGL((k_coarse_rhs<M, S, D>),
                           dim3(xcd_grid(((unsigned long long)g.N + 255) / 256)), dim3(256), 0, s,
                           g, law, st, beta, K, psibar, gvec, psi, node_map(g));
    }
};

struct ScaleLaunch {
    const Geo &g; const Law &law; const Step &st; const double *beta; const double *K;
    const double *gvec; const double *psi; unsigned long long *out; hipStream_t s;
    template <int M, bool S, int D>
    void go()
    {
        hipLaunchKernelGGL((k_defect_scale<M, S, D>),
                           dim3(xcd_grid(((unsigned long long)g.N + 255) / 256)), dim3(256), 0, s,
                           g, law, st, beta, K, gvec, psi, out, node_map(g));
    }
};

void launch_defect_scale(const Geo &g, const Law &law, const Step &st, const double *beta,
                         const double *K, const double *gvec, const double *psi,
                         unsigned long long *out, hipStream_t s)
{
    dispatch<true>(law, g.dim, ScaleLaunch{g, law, st, beta, K, gvec, psi, out, s});
}

struct ResidualLaunch {
    const Geo &g; const Law &law; const Step &st; const double *beta; const double *K;
    const double *gvec; const double *psi; double *d; unsigned long long *norm_bits; hipStream_t s;
    MpStart mp;
    template <int M, bool S, int D>
    void go()
    {
        const ColourMap cm = colour_map(g);
        hipLaunchKernelGGL((k_residual_pair<M, S, D>), dim3(xcd_grid((cm.total + 255) / 256)),
                           dim3(256), 0, s, g, law, st, beta, K, gvec, psi, d, norm_bits, cm, mp);
    }
};

int launch_sweep_rb(const Geo &g, const Law &law, const Step &st, const double *beta,
                    double lambdaU, const double *K, const double *gvec, double **psi,
                    double **psi_alt, int nsweeps, hipStream_t s)
{
    if (nsweeps <= 0) return 0;
    dispatch<true>(law, g.dim, SweepLaunch{g, law, st, beta, lambdaU, K, gvec, psi, psi_alt, nsweeps, s});
    if (g.N <= 1024) return 1;
    return (g.dim == 3 && psi_alt && *psi_alt && fused_enabled()) ? nsweeps : 2 * nsweeps;
}

bool sweep_defect_level(const Geo &g, const Law &law, int nsweeps)
{
    if (nsweeps <= 0 || g.N <= 1024 || !buffer_ok(g, sizeof(double)) ||
        law.kappa_rule == kKappaRemark || !pair_sweep_level(g) || !sweep_defect_enabled())
        return false;
    return !(g.dim == 3 && zm_level(g) && zm_enabled());
}

void launch_sweep_defect(const Geo &g, const Law &law, const Step &st, const double *beta,
                         const double *K, const double *gvec, double *psi, int nsweeps, double *d,
                         unsigned long long *norm_bits, int phase, hipStream_t s)
{
    dispatch<true>(law, g.dim,
                   SweepDefectLaunch{g, law, st, beta, K, gvec, psi, nsweeps, d, norm_bits, s, phase});
}

bool fused_sweep_level(const Geo &g)
{
    return g.dim == 3 && g.N >= kFusedMinNodes && fused_enabled();
}

void launch_residual(const Geo &g, const Law &law, const Step &st, const double *beta,
                     const double *K, const double *gvec, const double *psi, double *d,
                     unsigned long long *norm_bits, hipStream_t s, MpStart mp)
{
    dispatch<true>(law, g.dim, ResidualLaunch{g, law, st, beta, K, gvec, psi, d, norm_bits, s, mp});
}

void launch_restrict(const Geo &gc, const Geo &gf, const double *psi_f, const double *d_f,
                     double *psibar_c, double *g_c, hipStream_t s)
{
    launch_restrict_t<double>(gc, gf, psi_f, d_f, psibar_c, g_c, s);
}

void launch_coarse_rhs(const Geo &gc, const Law &law, const Step &st, const double *beta,
                       const double *K, const double *psibar, double *gvec, double *psi,
                       hipStream_t s)
{
    dispatch<true>(law, gc.dim, CoarseRhsLaunch{gc, law, st, beta, K, psibar, gvec, psi, s});
}

void launch_prolong(const Geo &gf, const Geo &gc, const double *psi_c, const double *psibar_c,
                    double *psi_f, hipStream_t s)
{
    launch_prolong_t<double>(gf, gc, psi_c, psibar_c, psi_f, s);
}

struct TailLaunch {
    const TailArgs *A; int top, last; const Law &law; const Step &st; int nu1, nu2, nuc;
    int lds_from; size_t lds_bytes; hipStream_t s;
    template <int M, bool S, int D>
    void go()
    {
        hipLaunchKernelGGL((k_vcycle_tail<M, S, D>), dim3(1), dim3(512), lds_bytes, s, A, top, last,
                           law, st, nu1, nu2, nuc, lds_from);
    }
};

size_t tail_lds_bytes(const long long *nodes, int top, int from, int last)
{
    size_t b = 0;
    for (int l = from; l <= last; ++l) b += (l == top ? 4 : 5) * sizeof(double) * (size_t)(nodes[l] + 2);
    return b;
}

void launch_vcycle_tail(const TailArgs *args_dev, int top, int last, const Law &law,
                        const Step &st, int nu1, int nu2, int nuc, int dim, const long long *nodes,
                        hipStream_t s)
{
    // the deepest levels that fit in kTailLds bytes of LDS
    int from = last + 1;
    while (from - 1 >= top && tail_lds_bytes(nodes, top, from - 1, last) <= kTailLds) --from;
    const size_t bytes = from <= last ? tail_lds_bytes(nodes, top, from, last) : 0;
    dispatch<true>(law, dim, TailLaunch{args_dev, top, last, law, st, nu1, nu2, nuc, from, bytes, s});
}

void launch_interp(const Geo &gf, const Geo &gc, const double *psi_c, double *psi_f, hipStream_t s)
{
    launch_prolong_t<double, true>(gf, gc, psi_c, nullptr, psi_f, s);
}

}  // namespace rs
