// Continuous-batching engine (include/richards_serve.h).
//
// Device side.  Every resident request ("slot") owns a static record (law,
// step length, pointers into the arena), a dynamic record written only by the
// device (state machine, step counters, residual norms) and one record per
// multigrid level.  Work is described by lists of (slot, level) items with
// prefix sums of their 256-wide tiles; a batched kernel walks the tiles of its
// list in contiguous per-work-group chunks (XCD-aware numbering) and skips
// items whose slot is not in the state the kernel serves.  One correction
// round for all slots is:
//
//   set-up of slots in BEGIN: history shift, K* (FP64) with its FP32 copy on
//     every level, right-hand side g, FP64 defect + norm, control -> ACTIVE
//   FP32 FAS V-cycle of the correction equation for ACTIVE slots:
//     per depth d of the "wide" levels (more than tail_nodes nodes):
//       nu1 red-black sweeps, inner defect, FW restriction, FAS right-hand side
//     one work-group per slot runs the rest of the cycle on its small levels
//     per depth, back up: prolongation of the correction, nu2 sweeps
//   psi += delta (FP64), FP64 defect + norm, control: convergence, step
//     transition (history update and next step's set-up) or failure.
//
// The sequence has a fixed launch shape (work-group counts do not depend on
// which slots are resident), so it is captured once as a HIP graph and
// replayed.  Each node's arithmetic is that of the single-grid kernels
// (cell64.h, cell32.h, transfer.h) and depends only on its own slot's data, so
// a request's result does not depend on the mix it runs in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <iterator>
#include <map>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/richards.h"
#include "../../include/richards_serve.h"
#include "rs_internal.h"
#include "soil_device.h"
#include "grid_device.h"
#include "transfer.h"
#include "soil_mp.h"
#include "cell64.h"
#include "cell32.h"
#include "mp_internal.h"
#include "host_common.h"

namespace rs {
namespace {

constexpr int kTile = 256;
constexpr int kWideGroups = 2048;   // work-groups of every batched multi-group kernel
constexpr int kEngMaxLevels = 12;   // up to 2^11 + 1 nodes on the shortest axis
constexpr int kMaxSlots = 4096;
constexpr int kMaxWide = 8;
constexpr int kTailThreads = 1024;        // work-group of the small-level cycle
constexpr size_t kTailLdsMax = 152 * 1024;  // LDS the small-level cycle may use

enum : int { kEmpty = 0, kBegin = 1, kActive = 2, kFinished = 3, kFailed = 4 };

struct ELevel {
    Geo geo;
    ColourMap cm;
    NodeMap nm;
    float *dl, *K32, *rhs, *r, *dbar, *pb;
};

// The six FP32 arrays of one level (in HBM, or in LDS for the small levels).
struct Arrs {
    float *dl, *K32, *rhs, *r, *dbar, *pb;
};

__device__ __forceinline__ Arrs arrs_of(const ELevel &L)
{
    return Arrs{L.dl, L.K32, L.rhs, L.r, L.dbar, L.pb};
}

struct ESlot {
    Law law;
    Law32 law32;
    double dt;
    int order, nsteps, nlev, wide;
    double *psi, *psi_n, *psi_nm1, *K, *g;
    double tol_abs, tol_rel;
    int stagnation, max_corr;
    int tail_lds;   // small levels fit in the tail's LDS
};

struct EDyn {
    int state, end_prev, steps_done, corr, corr_total, corr_max, slow, order_eff, status, pad;
    double a, r0, best, res;
    unsigned long long norm_bits;
    unsigned long long scale_bits;   // max over nodes of the magnitudes of the defect's terms
                                     // (|g|, a |theta|, xi |psi|, m_ij (|psi_i| + |psi_j|))
};

// A stall counts as the rounding floor when the defect norm of the iterate
// kept is within 16 ulp of the defect's term scale (the rule of rs_bdf_step).
constexpr double kEngFloorRel = 16.0 * 2.220446049250313e-16;

// Work list: count items (slot, level) and three tile prefix sums:
// kind 0 = colour-packed cells of the level, 1 = nodes of the level,
// 2 = nodes of the next coarser level.
struct EList {
    int count;
    unsigned total[3];
    const int *slot;
    const int *lev;
    const unsigned *pre[3];
};

__device__ __forceinline__ unsigned sgpr(unsigned v) { return __builtin_amdgcn_readfirstlane(v); }

// Index of the item whose tile range holds virtual tile v (pre is ascending,
// pre[0] = 0, pre[count] = total).
__device__ __forceinline__ int find_item(const unsigned *pre, int count, unsigned v)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Walk this work-group's contiguous chunk of the list's virtual tiles:
// body(item, tile-within-item).  flush(item) runs when the chunk leaves an item
// (and at its end); every call is uniform over the work-group.
template <typename Body, typename Flush>
__device__ __forceinline__ void tile_loop(const EList &L, int kind, Body &&body, Flush &&flush)
{
    const unsigned total = L.total[kind];
    if (total == 0) return;
    const unsigned per = (total + gridDim.x - 1) / gridDim.x;
    const unsigned lb = xcd_block(gridDim.x / 8u);
    const unsigned v0 = lb * per;
    const unsigned v1 = min(v0 + per, total);
    if (v0 >= v1) return;
    const unsigned *pre = L.pre[kind];
    int it = (int)sgpr((unsigned)find_item(pre, L.count, v0));
    for (unsigned v = v0; v < v1; ++v) {
        while (v >= pre[it + 1]) {
            flush(it);
            ++it;
        }
        body(it, v - pre[it]);
    }
    flush(it);
}

struct NoFlush {
    __device__ void operator()(int) const {}
};

template <typename Fn>
__device__ __forceinline__ void law_dim(int model, int dim, Fn &&fn)
{
    using std::integral_constant;
#define RS_E_DIMS(M)                                                            \
    do {                                                                        \
        if (dim == 1) fn(integral_constant<int, M>{}, integral_constant<int, 1>{}); \
        else if (dim == 2) fn(integral_constant<int, M>{}, integral_constant<int, 2>{}); \
        else fn(integral_constant<int, M>{}, integral_constant<int, 3>{});     \
    } while (0)
    if (model == kVgm) RS_E_DIMS(kVgm);
    else if (model == kHaverkamp) RS_E_DIMS(kHaverkamp);
    else RS_E_DIMS(kLinear);
#undef RS_E_DIMS
}

template <typename Fn>
__device__ __forceinline__ void dim_switch(int dim, Fn &&fn)
{
    using std::integral_constant;
    if (dim == 1) fn(integral_constant<int, 1>{});
    else if (dim == 2) fn(integral_constant<int, 2>{});
    else fn(integral_constant<int, 3>{});
}

__device__ __forceinline__ Step slot_step(const ESlot &S, const EDyn &D)
{
    Step st;
    st.a = D.a;
    st.dt = S.dt;
    st.order = D.order_eff;
    st.lag_extrap = 0;   // the engine lags K* at psi^n
    return st;
}

// ---------------------------------------------------------------------------
// Step set-up (slots in BEGIN)
// ---------------------------------------------------------------------------

// History shift after a finished step (psi^{n-1} <- psi^n <- psi), first
// iterate, K* (FP64) and its FP32 copy on every level where the node is a
// coarse-grid node (injection).
__global__ __launch_bounds__(256) void e_kstar(const EList *FL, const ESlot *slots, EDyn *dyn,
                                               const ELevel *levels)
{
    const EList L = *FL;
    tile_loop(L, 1, [&](int it, unsigned tile) {
        const int s = L.slot[it];
        if (dyn[s].state != kBegin) return;
        const ESlot &S = slots[s];
        const EDyn &D = dyn[s];
        const ELevel &L0 = levels[s * kEngMaxLevels];
        const unsigned long long t = (unsigned long long)tile * kTile + threadIdx.x;
        if (t >= (unsigned long long)L0.geo.N) return;
        int i, j, k;
        node_ijk(L0.nm, t, i, j, k);
        if (D.end_prev) {
            const double p = S.psi[t];
            S.psi_nm1[t] = S.psi_n[t];
            S.psi_n[t] = p;
        }
        const Step st = slot_step(S, D);
        double p0;
        const double Kv = kstar_at(L0.geo, S.law, st, S.psi_n, S.psi_nm1, S.law.Ks, i, j, k,
                                   (long long)t, &p0);
        S.K[t] = Kv;
        S.psi[t] = p0;
        for (int l = 0; l < S.nlev; ++l) {
            const int m = (1 << l) - 1;
            if ((i | j | k) & m) break;
            const ELevel &Lv = levels[s * kEngMaxLevels + l];
            Lv.K32[lin(Lv.geo, i >> l, j >> l, k >> l)] = (float)Kv;
        }
    }, NoFlush{});
}

__global__ __launch_bounds__(256) void e_gvec(const EList *FL, const ESlot *slots,
                                              const EDyn *dyn, const ELevel *levels)
{
    const EList L = *FL;
    tile_loop(L, 1, [&](int it, unsigned tile) {
        const int s = L.slot[it];
        if (dyn[s].state != kBegin) return;
        const ESlot &S = slots[s];
        const ELevel &L0 = levels[s * kEngMaxLevels];
        const unsigned long long t = (unsigned long long)tile * kTile + threadIdx.x;
        if (t >= (unsigned long long)L0.geo.N) return;
        int i, j, k;
        node_ijk(L0.nm, t, i, j, k);
        const Step st = slot_step(S, dyn[s]);
        S.g[t] = g_at(L0.geo, S.law, st, S.psi_n, S.psi_nm1, S.K, i, j, k, (long long)t);
    }, NoFlush{});
}

// FP64 defect d = g - N(psi) of slots in state `want`: its max-norm into the
// slot's norm bits, and the start of the next correction: rhs = fl32(d) and
// delta = 0 on the finest level, base state psi_b = fl32(psi) on every level.
__global__ __launch_bounds__(256) void e_defect(const EList *FL, const ESlot *slots, EDyn *dyn,
                                                const ELevel *levels, int want)
{
    const EList L = *FL;
    double v = 0.0, vs = 0.0;
    tile_loop(L, 1, [&](int it, unsigned tile) {
        const int s = L.slot[it];
        if (dyn[s].state != want) return;
        const ESlot &S = slots[s];
        const ELevel &L0 = levels[s * kEngMaxLevels];
        const unsigned long long t = (unsigned long long)tile * kTile + threadIdx.x;
        if (t >= (unsigned long long)L0.geo.N) return;
        int i, j, k;
        node_ijk(L0.nm, t, i, j, k);
        const double a = dyn[s].a;
        const double x = S.psi[t];
        double r = 0.0;
        law_dim(S.law.model, L0.geo.dim, [&](auto M, auto Dm) {
            if (dirichlet_t<decltype(Dm)::value>(L0.geo, i, j, k)) return;
            double terms = 0.0;
            r = S.g[t] - apply_N_t<decltype(M)::value, false, decltype(Dm)::value, true>(
                             L0.geo, S.law, a, nullptr, S.K, S.psi, i, j, k, (long long)t, &terms);
            const double sc = fabs(S.g[t]) + terms;
            vs = sc > vs ? sc : vs;
        });
        const double ar = fabs(r);
        v = (ar > v || ar != ar) ? ar : v;
        L0.rhs[t] = (float)r;
        L0.dl[t] = 0.0f;
        for (int l = 0; l < S.nlev; ++l) {
            const int m = (1 << l) - 1;
            if ((i | j | k) & m) break;
            const ELevel &Lv = levels[s * kEngMaxLevels + l];
            Lv.pb[lin(Lv.geo, i >> l, j >> l, k >> l)] = (float)x;
        }
    }, [&](int it) {
        const int s = L.slot[it];
        if (dyn[s].state != want) return;   // uniform: same item for the whole group
        const double m = block_max(v);
        if (threadIdx.x == 0) atomicMax(&dyn[s].norm_bits, (unsigned long long)__double_as_longlong(m));
        __syncthreads();
        const double ms = block_max(vs);
        if (threadIdx.x == 0) atomicMax(&dyn[s].scale_bits, (unsigned long long)__double_as_longlong(ms));
        __syncthreads();
        v = 0.0;
        vs = 0.0;
    });
}

// Per-slot control after a defect.  mode 0: slots in BEGIN become ACTIVE with
// r0 = best = the defect norm.  mode 1: ACTIVE slots count the correction and
// test convergence (norm <= max(tol_abs, tol_rel r0), or the rounding floor);
// a converged step either finishes the request or starts the next step.
__global__ __launch_bounds__(256) void e_control(const ESlot *slots, EDyn *dyn, int nslots,
                                                 int mode)
{
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nslots; s += gridDim.x * blockDim.x) {
        EDyn D = dyn[s];
        const ESlot &S = slots[s];
        double res = __longlong_as_double((long long)D.norm_bits);
        const double scale = __longlong_as_double((long long)D.scale_bits);
        if (mode == 0) {
            if (D.state != kBegin) continue;
            D.norm_bits = 0ull;
            D.scale_bits = 0ull;
            D.res = res;
            D.r0 = res;
            D.best = res;
            D.slow = 0;
            D.corr = 0;
            if (!(res == res) || isinf(res)) {
                D.state = kFailed;
                D.status = RS_ENONFINITE;
            } else {
                D.state = kActive;
            }
            dyn[s] = D;
            continue;
        }
        if (D.state != kActive) continue;
        D.norm_bits = 0ull;
        D.scale_bits = 0ull;
        D.res = res;
        D.corr += 1;
        D.corr_total += 1;
        if (!(res == res) || isinf(res)) {
            D.state = kFailed;
            D.status = RS_ENONFINITE;
            dyn[s] = D;
            continue;
        }
        bool done = res <= fmax(S.tol_abs, S.tol_rel * D.r0);
        if (S.stagnation) {
            if (res < D.best) {
                D.best = res;
                D.slow = 0;
            } else if (++D.slow >= 2 && !done) {
                // two corrections without a new minimum: the rounding floor if
                // the norm of the iterate kept (the last one) is near the
                // defect's scale, else the iteration diverges or stalls
                if (res <= kEngFloorRel * scale) {
                    done = true;
                } else {
                    D.state = kFailed;
                    D.status = RS_ENOTCONV;
                    dyn[s] = D;
                    continue;
                }
            }
        }
        if (done) {
            D.corr_max = max(D.corr_max, D.corr);
            D.steps_done += 1;
            if (D.steps_done >= S.nsteps) {
                D.state = kFinished;
                D.status = RS_OK;
            } else {
                D.state = kBegin;
                D.end_prev = 1;
                D.order_eff = S.order;
                D.a = S.order == 1 ? 1.0 / S.dt : 1.5 / S.dt;
            }
        } else if (D.corr >= S.max_corr) {
            D.state = kFailed;
            D.status = RS_ENOTCONV;
        }
        dyn[s] = D;
    }
}

// ---------------------------------------------------------------------------
// FP32 V-cycle of the correction equation, wide levels (slots in ACTIVE)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void e_sweep32(const EList *DL, const ESlot *slots,
                                                 const EDyn *dyn, const ELevel *levels, int colour)
{
    const EList L = *DL;
    tile_loop(L, 0, [&](int it, unsigned tile) {
        const int s = L.slot[it];
        if (dyn[s].state != kActive) return;
        const ESlot &S = slots[s];
        const ELevel &Lv = levels[s * kEngMaxLevels + L.lev[it]];
        int i, j, k;
        if (!colour_ijk(Lv.geo, Lv.cm, (unsigned long long)tile * kTile + threadIdx.x, colour, i,
                        j, k))
            return;
        const float a = (float)dyn[s].a;
        law_dim(S.law.model, Lv.geo.dim, [&](auto M, auto Dm) {
            if (dirichlet_t<decltype(Dm)::value>(Lv.geo, i, j, k)) return;
            ngs_cell32<decltype(M)::value, false, decltype(Dm)::value, true>(
                Lv.geo, S.law32, a, nullptr, 0.0f, Lv.K32, Lv.rhs, Lv.pb, Lv.dl, i, j, k, colour);
        });
    }, NoFlush{});
}

__device__ __forceinline__ void resid32_node(const ESlot &S, float a, const ELevel &Lv,
                                             const Arrs &A, unsigned long long t)
{
    int i, j, k;
    node_ijk(Lv.nm, t, i, j, k);
    float v = 0.0f;
    law_dim(S.law.model, Lv.geo.dim, [&](auto M, auto Dm) {
        if (dirichlet_t<decltype(Dm)::value>(Lv.geo, i, j, k)) return;
        v = A.rhs[t] - apply_Nd<decltype(M)::value, false, decltype(Dm)::value>(
                           Lv.geo, S.law32, a, nullptr, A.K32, A.pb, A.dl, i, j, k, (long long)t);
    });
    A.r[t] = v;
}

__device__ __forceinline__ void restrict32_node(const ELevel &F, const ELevel &C, const Arrs &AF,
                                                const Arrs &AC, unsigned long long t)
{
    int i, j, k;
    node_ijk(C.nm, t, i, j, k);
    dim_switch(C.geo.dim, [&](auto Dm) {
        restrict_at<decltype(Dm)::value, float>(C.geo, F.geo, AF.dl, AF.r, AC.dbar, AC.rhs, i, j,
                                                k);
    });
}

__device__ __forceinline__ void crhs32_node(const ESlot &S, float a, const ELevel &C,
                                            const Arrs &AC, unsigned long long t)
{
    int i, j, k;
    node_ijk(C.nm, t, i, j, k);
    law_dim(S.law.model, C.geo.dim, [&](auto M, auto Dm) {
        if (dirichlet_t<decltype(Dm)::value>(C.geo, i, j, k)) return;
        AC.rhs[t] = apply_Nd<decltype(M)::value, false, decltype(Dm)::value>(
                        C.geo, S.law32, a, nullptr, AC.K32, AC.pb, AC.dbar, i, j, k,
                        (long long)t) +
                    AC.rhs[t];
    });
    AC.dl[t] = AC.dbar[t];
}

__device__ __forceinline__ void prolong32_node(const ELevel &F, const ELevel &C, const Arrs &AF,
                                               const Arrs &AC, unsigned long long t)
{
    int i, j, k;
    node_ijk(F.nm, t, i, j, k);
    dim_switch(F.geo.dim, [&](auto Dm) {
        prolong_at<decltype(Dm)::value, float>(F.geo, C.geo, AC.dl, AC.dbar, AF.dl, i, j, k);
    });
}

// op 0: inner defect on level d; 1: restriction d -> d+1; 2: FAS right-hand
// side on d+1; 3: prolongation d+1 -> d.
__global__ __launch_bounds__(256) void e_transfer32(const EList *DL, const ESlot *slots,
                                                    const EDyn *dyn, const ELevel *levels, int op)
{
    const EList L = *DL;
    const int kind = (op == 1 || op == 2) ? 2 : 1;
    tile_loop(L, kind, [&](int it, unsigned tile) {
        const int s = L.slot[it];
        if (dyn[s].state != kActive) return;
        const ESlot &S = slots[s];
        const ELevel &F = levels[s * kEngMaxLevels + L.lev[it]];
        const ELevel &C = levels[s * kEngMaxLevels + L.lev[it] + 1];
        const unsigned long long t = (unsigned long long)tile * kTile + threadIdx.x;
        const float a = (float)dyn[s].a;
        const Arrs AF = arrs_of(F), AC = arrs_of(C);
        if (kind == 1) {
            if (t >= (unsigned long long)F.geo.N) return;
            if (op == 0) resid32_node(S, a, F, AF, t);
            else prolong32_node(F, C, AF, AC, t);
        } else {
            if (t >= (unsigned long long)C.geo.N) return;
            if (op == 1) restrict32_node(F, C, AF, AC, t);
            else crhs32_node(S, a, C, AC, t);
        }
    }, NoFlush{});
}

// ---------------------------------------------------------------------------
// Small levels: one work-group per slot runs the cycle from level `wide` down
// to the coarsest and back, with work-group barriers between the steps.  Its
// helpers are inlined: as calls they took a stack frame and the call ABI's
// register budget (248 VGPRs against 127), and the array pointers of the LDS
// variant lost their address space (flat instead of LDS loads).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void tail_sweeps(const ESlot &S, float a, const ELevel &Lv,
                                            const Arrs &A, int n, bool exit)
{
    for (int sw = 0; sw < n; ++sw) {
        int changed = 0;
        for (int colour = 0; colour < 2; ++colour) {
            for (unsigned long long t = threadIdx.x; t < Lv.cm.total; t += blockDim.x) {
                int i, j, k;
                if (!colour_ijk(Lv.geo, Lv.cm, t, colour, i, j, k)) continue;
                law_dim(S.law.model, Lv.geo.dim, [&](auto M, auto Dm) {
                    if (dirichlet_t<decltype(Dm)::value>(Lv.geo, i, j, k)) return;
                    changed |= ngs_cell32<decltype(M)::value, false, decltype(Dm)::value>(
                        Lv.geo, S.law32, a, nullptr, 0.0f, A.K32, A.rhs, A.pb, A.dl, i, j, k,
                        colour);
                });
            }
            // a sweep that moved no value by more than FP32 rounding (4 ulp)
            // has converged in FP32 (the correction solve only sets the outer
            // FP64 iteration's contraction): the sweeps left would shuffle
            // rounding
            if (colour == 0 || !exit) __syncthreads();
            else if (!__syncthreads_or(changed)) return;
        }
    }
}

// The V-cycle from level top down to the coarsest and back, one work-group;
// arrs(l) gives the arrays of level l the cycle works on.
template <typename Arr>
__device__ __forceinline__ void tail_cycle(const ESlot &S, float a, const ELevel *LV, int top,
                                           int last, int nu1, int nu2, int nuc, Arr &&arrs)
{
    for (int l = top; l < last; ++l) {
        const ELevel &F = LV[l], &C = LV[l + 1];
        const Arrs AF = arrs(l), AC = arrs(l + 1);
        tail_sweeps(S, a, F, AF, nu1, false);
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)F.geo.N; t += blockDim.x)
            resid32_node(S, a, F, AF, t);
        __syncthreads();
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)C.geo.N; t += blockDim.x)
            restrict32_node(F, C, AF, AC, t);
        __syncthreads();
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)C.geo.N; t += blockDim.x)
            crhs32_node(S, a, C, AC, t);
        __syncthreads();
    }
    tail_sweeps(S, a, LV[last], arrs(last), nuc, true);
    for (int l = last - 1; l >= top; --l) {
        const ELevel &F = LV[l], &C = LV[l + 1];
        const Arrs AF = arrs(l), AC = arrs(l + 1);
        for (unsigned long long t = threadIdx.x; t < (unsigned long long)F.geo.N; t += blockDim.x)
            prolong32_node(F, C, AF, AC, t);
        __syncthreads();
        tail_sweeps(S, a, F, AF, nu2, false);
    }
}

// Arrays of level l of a request whose small levels live in LDS: levels
// top..last one after another, each as dl, K32, rhs, r, dbar, pb (N_l floats).
__device__ __forceinline__ Arrs lds_arrs(const ELevel *LV, int top, int l, float *smem)
{
    size_t off = 0;
    for (int q = top; q < l; ++q) off += 6 * (size_t)LV[q].geo.N;
    const size_t N = (size_t)LV[l].geo.N;
    float *p = smem + off;
    return Arrs{p, p + N, p + 2 * N, p + 3 * N, p + 4 * N, p + 5 * N};
}

__device__ __forceinline__ void block_copy(float *dst, const float *src, long long n)
{
    for (long long t = threadIdx.x; t < n; t += blockDim.x) dst[t] = src[t];
}

// One work-group per request runs its small levels.  A request whose small
// levels fit in LDS (ESlot::tail_lds) works there: K32 and psi_b of every small
// level and delta, rhs of the top one are staged in, the cycle runs on LDS,
// and delta of the top level is written back (the wide levels' prolongation
// reads it).
__global__ __launch_bounds__(1024) void e_tail(const EList *TL, const ESlot *slots,
                                              const EDyn *dyn, const ELevel *levels, int nu1,
                                              int nu2, int nuc)
{
    extern __shared__ float smem[];
    const int b = blockIdx.x;
    if (b >= TL->count) return;
    const int s = TL->slot[b];
    if (dyn[s].state != kActive) return;
    const ESlot &S = slots[s];
    const ELevel *LV = levels + s * kEngMaxLevels;
    const float a = (float)dyn[s].a;
    const int top = S.wide, last = S.nlev - 1;
    if (!S.tail_lds) {
        tail_cycle(S, a, LV, top, last, nu1, nu2, nuc, [&](int l) { return arrs_of(LV[l]); });
        return;
    }
    for (int l = top; l <= last; ++l) {
        const Arrs A = lds_arrs(LV, top, l, smem);
        const long long N = LV[l].geo.N;
        block_copy(A.K32, LV[l].K32, N);
        block_copy(A.pb, LV[l].pb, N);
        if (l == top) {
            block_copy(A.dl, LV[l].dl, N);
            block_copy(A.rhs, LV[l].rhs, N);
        }
    }
    __syncthreads();
    tail_cycle(S, a, LV, top, last, nu1, nu2, nuc,
               [&](int l) { return lds_arrs(LV, top, l, smem); });
    const Arrs T = lds_arrs(LV, top, top, smem);
    block_copy(LV[top].dl, T.dl, LV[top].geo.N);
}

// psi += delta in FP64 on the finest level (delta is 0 at Dirichlet nodes).
__global__ __launch_bounds__(256) void e_apply(const EList *FL, const ESlot *slots,
                                               const EDyn *dyn, const ELevel *levels)
{
    const EList L = *FL;
    tile_loop(L, 1, [&](int it, unsigned tile) {
        const int s = L.slot[it];
        if (dyn[s].state != kActive) return;
        const ELevel &L0 = levels[s * kEngMaxLevels];
        const unsigned long long t = (unsigned long long)tile * kTile + threadIdx.x;
        if (t >= (unsigned long long)L0.geo.N) return;
        slots[s].psi[t] += (double)L0.dl[t];
    }, NoFlush{});
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// First-fit allocator over [0, size) with coalescing of freed ranges.
class Arena {
public:
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
        free_bytes_ = size;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            size_t rest = it->second - bytes;
            size_t start = it->first + bytes;
            free_.erase(it);
            if (rest) free_[start] = rest;
            free_bytes_ -= bytes;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        free_bytes_ += bytes;
        auto nx = free_.lower_bound(off);
        if (nx != free_.end() && off + bytes == nx->first) {
            bytes += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == off) {
                pv->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    size_t free_bytes() const { return free_bytes_; }

private:
    std::map<size_t, size_t> free_;
    size_t free_bytes_ = 0;
};

// Byte layout of the control region (device arena start, mirrored in pinned
// host memory).
struct CtrlLayout {
    size_t slots, dyn, levels, lists, arrays, total;
    int nlists;
    size_t list_stride;   // bytes of one list's arrays
};

CtrlLayout ctrl_layout(const rs_engine_opts &o)
{
    CtrlLayout c;
    const size_t S = (size_t)o.max_slots;
    c.nlists = o.max_wide_levels + 2;   // fine, depth 0..W-1, tail
    size_t off = 0;
    c.slots = off;  off = align_up(off + sizeof(ESlot) * S);
    c.dyn = off;    off = align_up(off + sizeof(EDyn) * S);
    c.levels = off; off = align_up(off + sizeof(ELevel) * S * kEngMaxLevels);
    c.lists = off;  off = align_up(off + sizeof(EList) * c.nlists);
    c.list_stride = align_up(sizeof(int) * 2 * S + sizeof(unsigned) * 3 * (S + 1));
    c.arrays = off; off = align_up(off + c.list_stride * c.nlists);
    c.total = off;
    return c;
}

constexpr size_t kReqPad = 256;

struct ReqPlan {
    int nlev, wide;
    Geo geo[kEngMaxLevels];
    size_t fine_off[5];                 // psi, psi_n, psi_nm1, K, g
    size_t lev_off[kEngMaxLevels][6];   // dl, K32, rhs, r, dbar, pb
    size_t bytes;
};

int plan_request(const rs_engine_opts &o, const rs_grid_desc *d, ReqPlan *p)
{
    int e = validate_desc(d);
    if (e) return e;
    for (int f = 0; f < 2 * d->dim; ++f)
        if (d->face_bc[f] == RS_BC_DIRICHLET_STATE)
            return fail(RS_EINVAL, "the engine serves faces with constant boundary values");
    p->nlev = level_count(d);
    if (p->nlev > kEngMaxLevels)
        return fail(RS_EINVAL, "grid needs %d levels; the engine handles %d", p->nlev,
                    kEngMaxLevels);
    p->wide = 0;
    for (int l = 0; l < p->nlev; ++l) {
        p->geo[l] = make_geo(d, l);
        if (p->geo[l].N > (long long)o.tail_nodes) p->wide = l + 1;
    }
    if (p->wide >= p->nlev)
        return fail(RS_EINVAL, "coarsest level has %lld nodes, above tail_nodes %d",
                     p->geo[p->nlev - 1].N, o.tail_nodes);
    if (p->wide > o.max_wide_levels)
        return fail(RS_EINVAL, "request has %d levels above tail_nodes; the engine runs %d",
                    p->wide, o.max_wide_levels);
    // every array with kReqPad zeroed bytes before and after it (the region is
    // cleared at admission), so the wide-level stencils can load the row
    // neighbours idx -/+ 1 unconditionally
    size_t off = 0;
    auto place = [&](size_t bytes) {
        off = align_up(off + kReqPad);
        const size_t at = off;
        off = align_up(off + bytes + kReqPad);
        return at;
    };
    const size_t N0 = (size_t)p->geo[0].N;
    for (int a = 0; a < 5; ++a) p->fine_off[a] = place(sizeof(double) * N0);
    for (int l = 0; l < p->nlev; ++l)
        for (int a = 0; a < 6; ++a) p->lev_off[l][a] = place(sizeof(float) * (size_t)p->geo[l].N);
    p->bytes = off;
    return RS_OK;
}

int validate_opts(const rs_engine_opts *o)
{
    if (!o) return fail(RS_EINVAL, "null options");
    if (o->struct_size != sizeof(rs_engine_opts))
        return fail(RS_EINVAL, "rs_engine_opts.struct_size %zu != %zu", o->struct_size,
                    sizeof(rs_engine_opts));
    if (o->max_slots < 1 || o->max_slots > kMaxSlots) return fail(RS_EINVAL, "max_slots out of range");
    if (o->max_wide_levels < 0 || o->max_wide_levels > kMaxWide)
        return fail(RS_EINVAL, "max_wide_levels out of range");
    if (o->tail_nodes < 27) return fail(RS_EINVAL, "tail_nodes must be >= 27");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu_coarse < 1) return fail(RS_EINVAL, "bad smoothing counts");
    if (o->max_corrections < 1) return fail(RS_EINVAL, "max_corrections must be >= 1");
    if (!(o->tol_abs >= 0.0) || !(o->tol_rel >= 0.0)) return fail(RS_EINVAL, "tolerances must be >= 0");
    if (o->rounds_per_tick < 1) return fail(RS_EINVAL, "rounds_per_tick must be >= 1");
    return RS_OK;
}

}  // namespace
}  // namespace rs

using namespace rs;

struct rs_engine {
    rs_engine_opts o;
    hipStream_t stream;
    int device;
    char *base;
    size_t bytes;
    CtrlLayout cl;
    char *host;   // pinned mirror of the control region
    ESlot *d_slots, *h_slots;
    EDyn *d_dyn, *h_dyn;
    ELevel *d_levels, *h_levels;
    EList *d_lists, *h_lists;
    Arena arena;
    size_t data_base;   // arena offset where request data starts
    std::vector<int> ticket;          // per slot, -1 if free
    std::vector<size_t> mem_off, mem_len;
    std::vector<char> reported;
    std::vector<ReqPlan> plans;
    std::unordered_map<int, int> slot_of;
    int next_ticket;
    int hi_slot;                      // one past the highest slot ever used
    bool lists_dirty;
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool graph_ready;
    size_t tail_lds_bytes;            // dynamic LDS of the small-level cycle
};

namespace {

template <typename T>
T *dev_at(rs_engine *E, size_t off) { return reinterpret_cast<T *>(E->base + off); }
template <typename T>
T *host_at(rs_engine *E, size_t off) { return reinterpret_cast<T *>(E->host + off); }

// Rebuild the fine, per-depth and tail lists from the resident slots and copy
// them to the device.
int upload_lists(rs_engine *E)
{
    const int S = E->o.max_slots;
    const int W = E->o.max_wide_levels;
    for (int q = 0; q < E->cl.nlists; ++q) {
        const size_t aoff = E->cl.arrays + (size_t)q * E->cl.list_stride;
        int *slot = host_at<int>(E, aoff);
        int *lev = slot + S;
        unsigned *pre0 = reinterpret_cast<unsigned *>(lev + S);
        unsigned *pre[3] = {pre0, pre0 + (S + 1), pre0 + 2 * (S + 1)};
        int n = 0;
        unsigned tot[3] = {0, 0, 0};
        pre[0][0] = pre[1][0] = pre[2][0] = 0;
        for (int s = 0; s < E->hi_slot; ++s) {
            if (E->ticket[s] < 0) continue;
            const ReqPlan &P = E->plans[s];
            int l;
            if (q == 0) l = 0;
            else if (q == W + 1) l = P.wide;
            else {
                l = q - 1;
                if (l >= P.wide) continue;
            }
            const Geo &g = P.geo[l];
            unsigned t0 = (unsigned)((colour_map(g).total + kTile - 1) / kTile);
            unsigned t1 = (unsigned)((g.N + kTile - 1) / kTile);
            unsigned t2 = l + 1 < P.nlev ? (unsigned)((P.geo[l + 1].N + kTile - 1) / kTile) : 0u;
            slot[n] = s;
            lev[n] = l;
            tot[0] += t0;
            tot[1] += t1;
            tot[2] += t2;
            ++n;
            pre[0][n] = tot[0];
            pre[1][n] = tot[1];
            pre[2][n] = tot[2];
        }
        EList &h = E->h_lists[q];
        h.count = n;
        for (int k = 0; k < 3; ++k) h.total[k] = tot[k];
        const size_t doff = aoff;
        h.slot = dev_at<int>(E, doff);
        h.lev = h.slot + S;
        const unsigned *dpre0 = reinterpret_cast<const unsigned *>(h.lev + S);
        for (int k = 0; k < 3; ++k) h.pre[k] = dpre0 + k * (S + 1);
        HIPCALL(hipMemcpyAsync(E->base + aoff, E->host + aoff, E->cl.list_stride,
                               hipMemcpyHostToDevice, E->stream));
    }
    HIPCALL(hipMemcpyAsync(E->base + E->cl.lists, E->host + E->cl.lists,
                           sizeof(EList) * E->cl.nlists, hipMemcpyHostToDevice, E->stream));
    E->lists_dirty = false;
    return RS_OK;
}

// One correction round for every resident slot (the captured sequence).
void enqueue_round(rs_engine *E)
{
    const rs_engine_opts &o = E->o;
    const int W = o.max_wide_levels;
    const dim3 wg(kWideGroups), blk(256);
    hipStream_t s = E->stream;
    const EList *fine = E->d_lists;
    const EList *tail = E->d_lists + W + 1;
    const int ctl_groups = (o.max_slots + 255) / 256;
    hipLaunchKernelGGL(e_kstar, wg, blk, 0, s, fine, E->d_slots, E->d_dyn, E->d_levels);
    hipLaunchKernelGGL(e_gvec, wg, blk, 0, s, fine, E->d_slots, E->d_dyn, E->d_levels);
    hipLaunchKernelGGL(e_defect, wg, blk, 0, s, fine, E->d_slots, E->d_dyn, E->d_levels,
                       (int)kBegin);
    hipLaunchKernelGGL(e_control, dim3(ctl_groups), blk, 0, s, E->d_slots, E->d_dyn,
                       o.max_slots, 0);
    for (int d = 0; d < W; ++d) {
        const EList *dl = E->d_lists + 1 + d;
        for (int sw = 0; sw < o.nu1; ++sw)
            for (int c = 0; c < 2; ++c)
                hipLaunchKernelGGL(e_sweep32, wg, blk, 0, s, dl, E->d_slots, E->d_dyn,
                                   E->d_levels, c);
        for (int op = 0; op < 3; ++op)
            hipLaunchKernelGGL(e_transfer32, wg, blk, 0, s, dl, E->d_slots, E->d_dyn,
                               E->d_levels, op);
    }
    hipLaunchKernelGGL(e_tail, dim3(o.max_slots), dim3(kTailThreads), E->tail_lds_bytes, s, tail,
                       E->d_slots, E->d_dyn, E->d_levels, o.nu1, o.nu2, o.nu_coarse);
    for (int d = W - 1; d >= 0; --d) {
        const EList *dl = E->d_lists + 1 + d;
        hipLaunchKernelGGL(e_transfer32, wg, blk, 0, s, dl, E->d_slots, E->d_dyn, E->d_levels, 3);
        for (int sw = 0; sw < o.nu2; ++sw)
            for (int c = 0; c < 2; ++c)
                hipLaunchKernelGGL(e_sweep32, wg, blk, 0, s, dl, E->d_slots, E->d_dyn,
                                   E->d_levels, c);
    }
    hipLaunchKernelGGL(e_apply, wg, blk, 0, s, fine, E->d_slots, E->d_dyn, E->d_levels);
    hipLaunchKernelGGL(e_defect, wg, blk, 0, s, fine, E->d_slots, E->d_dyn, E->d_levels,
                       (int)kActive);
    hipLaunchKernelGGL(e_control, dim3(ctl_groups), blk, 0, s, E->d_slots, E->d_dyn,
                       o.max_slots, 1);
}

int capture_graph(rs_engine *E)
{
    HIPCALL(hipStreamBeginCapture(E->stream, hipStreamCaptureModeThreadLocal));
    enqueue_round(E);
    hipGraph_t g = nullptr;
    hipError_t e1 = hipStreamEndCapture(E->stream, &g);
    if (e1 != hipSuccess) return fail(RS_EHIP, "graph capture: %s", hipGetErrorString(e1));
    E->graph = g;
    HIPCALL(hipGraphInstantiate(&E->exec, g, nullptr, nullptr, 0));
    E->graph_ready = true;
    return RS_OK;
}

}  // namespace

extern "C" {

void rs_engine_default_opts(rs_engine_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof *o);
    o->struct_size = sizeof(rs_engine_opts);
    o->max_slots = 1024;
    o->max_wide_levels = 4;
    o->tail_nodes = 8192;
    o->nu1 = 2;
    o->nu2 = 2;
    o->nu_coarse = 32;
    o->max_corrections = 100;
    o->tol_abs = 0.0;
    o->tol_rel = 0.0;
    o->stagnation = 1;
    o->rounds_per_tick = 4;
    o->use_graph = 1;
}

int rs_engine_control_bytes(const rs_engine_opts *o, size_t *out)
{
    int e = validate_opts(o);
    if (e) return e;
    if (!out) return fail(RS_EINVAL, "null out");
    *out = ctrl_layout(*o).total;
    return RS_OK;
}

int rs_engine_request_bytes(const rs_engine_opts *o, const rs_grid_desc *d, size_t *out)
{
    int e = validate_opts(o);
    if (e) return e;
    if (!out) return fail(RS_EINVAL, "null out");
    ReqPlan p;
    e = plan_request(*o, d, &p);
    if (e) return e;
    *out = p.bytes;
    return RS_OK;
}

int rs_engine_create(const rs_engine_opts *o, void *arena_dev, size_t arena_bytes, void *stream,
                     rs_engine **out)
{
    int e = validate_opts(o);
    if (e) return e;
    if (!out || !arena_dev) return fail(RS_EINVAL, "null argument");
    if (!stream) return fail(RS_EINVAL, "the engine needs a non-null stream");
    if ((uintptr_t)arena_dev % kAlign) return fail(RS_EINVAL, "arena must be 256-byte aligned");
    CtrlLayout cl = ctrl_layout(*o);
    if (arena_bytes < cl.total + kAlign)
        return fail(RS_ENOMEM, "arena of %zu bytes below the control region (%zu)", arena_bytes,
                    cl.total);
    rs_engine *E = new rs_engine();
    E->o = *o;
    E->stream = (hipStream_t)stream;
    E->base = (char *)arena_dev;
    E->bytes = arena_bytes;
    E->cl = cl;
    E->host = nullptr;
    E->graph = nullptr;
    E->exec = nullptr;
    E->graph_ready = false;
    E->tail_lds_bytes = 0;
    if (hipGetDevice(&E->device) != hipSuccess ||
        hipHostMalloc((void **)&E->host, cl.total, hipHostMallocDefault) != hipSuccess) {
        delete E;
        return fail(RS_EHIP, "pinned control mirror of %zu bytes", cl.total);
    }
    memset(E->host, 0, cl.total);
    {
        int lds_max = 0;
        if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, E->device) !=
            hipSuccess)
            lds_max = 0;
        size_t want = std::min(kTailLdsMax, (size_t)std::max(lds_max, 0));
        if (want >= 64 * 1024 &&
            hipFuncSetAttribute((const void *)e_tail, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)want) == hipSuccess)
            E->tail_lds_bytes = want;
    }
    E->d_slots = dev_at<ESlot>(E, cl.slots);
    E->h_slots = host_at<ESlot>(E, cl.slots);
    E->d_dyn = dev_at<EDyn>(E, cl.dyn);
    E->h_dyn = host_at<EDyn>(E, cl.dyn);
    E->d_levels = dev_at<ELevel>(E, cl.levels);
    E->h_levels = host_at<ELevel>(E, cl.levels);
    E->d_lists = dev_at<EList>(E, cl.lists);
    E->h_lists = host_at<EList>(E, cl.lists);
    E->data_base = cl.total;
    E->arena.reset(arena_bytes - cl.total);
    const int S = o->max_slots;
    E->ticket.assign(S, -1);
    E->mem_off.assign(S, 0);
    E->mem_len.assign(S, 0);
    E->reported.assign(S, 0);
    E->plans.resize(S);
    E->next_ticket = 1;
    E->hi_slot = 0;
    // zeroed control region (all slots EMPTY, empty lists)
    if (hipMemcpyAsync(E->base, E->host, cl.total, hipMemcpyHostToDevice, E->stream) !=
        hipSuccess) {
        (void)hipHostFree(E->host);
        delete E;
        return fail(RS_EHIP, "control region upload");
    }
    E->lists_dirty = true;
    e = upload_lists(E);
    if (e == RS_OK && o->use_graph) e = capture_graph(E);
    if (e == RS_OK && hipStreamSynchronize(E->stream) != hipSuccess)
        e = fail(RS_EHIP, "engine set-up");
    if (e) {
        (void)hipStreamSynchronize(E->stream);   // pending copies read the pinned mirror
        if (E->exec) (void)hipGraphExecDestroy(E->exec);
        if (E->graph) (void)hipGraphDestroy(E->graph);
        (void)hipHostFree(E->host);
        delete E;
        return e;
    }
    *out = E;
    return RS_OK;
}

int rs_engine_submit(rs_engine *E, const rs_grid_desc *d, const rs_constitutive *c,
                     const double *psi0_dev, double dt, int order, int nsteps, int *ticket)
{
    if (!E || !psi0_dev || !ticket) return fail(RS_EINVAL, "null argument");
    int e = validate_law(c);
    if (e) return e;
    if (c->sink != RS_SINK_NONE) return fail(RS_EINVAL, "the engine serves requests without a sink");
    if (c->n_soils > 0 || c->model == RS_GARDNER)
        return fail(RS_EINVAL, "the engine serves the vGM, Haverkamp and linear laws, one per request");
    if (c->kappa_rule == RS_KAPPA_REMARK)
        return fail(RS_EINVAL, "the engine serves kappa rules CONST and REL");
    if (c->Ks_field) return fail(RS_EINVAL, "the engine serves uniform Ks");
    if (c->lag_extrap) return fail(RS_EINVAL, "the engine lags K at psi^n");
    if (c->coarse_kstar != RS_COARSE_INJECT) return fail(RS_EINVAL, "the engine injects K* to coarse levels");
    if (!(dt > 0.0)) return fail(RS_EINVAL, "dt must be positive");
    if (order != 1 && order != 2) return fail(RS_EINVAL, "order must be 1 or 2");
    if (nsteps < 1) return fail(RS_EINVAL, "nsteps must be >= 1");
    ReqPlan P;
    e = plan_request(E->o, d, &P);
    if (e) return e;
    if (P.bytes > E->bytes - E->data_base)
        return fail(RS_EINVAL, "request needs %zu bytes; the arena holds %zu", P.bytes,
                    E->bytes - E->data_base);
    int s = -1;
    for (int q = 0; q < E->o.max_slots; ++q)
        if (E->ticket[q] < 0) { s = q; break; }
    if (s < 0) return fail(RS_EBUSY, "no free slot");
    size_t off;
    if (!E->arena.alloc(P.bytes, &off)) return fail(RS_EBUSY, "arena full");
    char *mem = E->base + E->data_base + off;
    ESlot &S = E->h_slots[s];
    memset(&S, 0, sizeof S);
    S.law = make_law(c);
    S.law32 = make_law32(S.law);
    S.dt = dt;
    S.order = order;
    S.nsteps = nsteps;
    S.nlev = P.nlev;
    S.wide = P.wide;
    double **fp[5] = {&S.psi, &S.psi_n, &S.psi_nm1, &S.K, &S.g};
    for (int a = 0; a < 5; ++a) *fp[a] = (double *)(mem + P.fine_off[a]);
    S.tol_abs = E->o.tol_abs;
    S.tol_rel = E->o.tol_rel;
    S.stagnation = E->o.stagnation;
    S.max_corr = E->o.max_corrections;
    {
        size_t tb = 0;
        for (int l = P.wide; l < P.nlev; ++l) tb += 6 * sizeof(float) * (size_t)P.geo[l].N;
        S.tail_lds = (E->tail_lds_bytes > 0 && tb <= E->tail_lds_bytes) ? 1 : 0;
    }
    for (int l = 0; l < P.nlev; ++l) {
        ELevel &Lv = E->h_levels[s * kEngMaxLevels + l];
        memset(&Lv, 0, sizeof Lv);
        Lv.geo = P.geo[l];
        Lv.cm = colour_map(P.geo[l]);
        Lv.nm = node_map(P.geo[l]);
        float **lp[6] = {&Lv.dl, &Lv.K32, &Lv.rhs, &Lv.r, &Lv.dbar, &Lv.pb};
        for (int a = 0; a < 6; ++a) *lp[a] = (float *)(mem + P.lev_off[l][a]);
    }
    EDyn &D = E->h_dyn[s];
    memset(&D, 0, sizeof D);
    D.state = kBegin;
    D.end_prev = 0;
    D.order_eff = 1;
    D.a = 1.0 / dt;
    const size_t nb = sizeof(double) * (size_t)P.geo[0].N;
    // zero padding around every array (and the arrays themselves)
    HIPCALL(hipMemsetAsync(mem, 0, P.bytes, E->stream));
    HIPCALL(hipMemcpyAsync(S.psi_n, psi0_dev, nb, hipMemcpyDeviceToDevice, E->stream));
    HIPCALL(hipMemcpyAsync(S.psi_nm1, psi0_dev, nb, hipMemcpyDeviceToDevice, E->stream));
    HIPCALL(hipMemcpyAsync(E->d_slots + s, &S, sizeof S, hipMemcpyHostToDevice, E->stream));
    HIPCALL(hipMemcpyAsync(E->d_levels + s * kEngMaxLevels, &E->h_levels[s * kEngMaxLevels],
                           sizeof(ELevel) * P.nlev, hipMemcpyHostToDevice, E->stream));
    HIPCALL(hipMemcpyAsync(E->d_dyn + s, &D, sizeof D, hipMemcpyHostToDevice, E->stream));
    E->plans[s] = P;
    E->ticket[s] = E->next_ticket++;
    E->mem_off[s] = off;
    E->mem_len[s] = P.bytes;
    E->reported[s] = 0;
    E->slot_of[E->ticket[s]] = s;
    E->hi_slot = std::max(E->hi_slot, s + 1);
    E->lists_dirty = true;
    *ticket = E->ticket[s];
    return RS_OK;
}

int rs_engine_tick(rs_engine *E, int *done, int max_done, int *n_done, int *n_active)
{
    if (!E || !n_done || !n_active || (max_done > 0 && !done)) return fail(RS_EINVAL, "null argument");
    *n_done = 0;
    *n_active = 0;
    if (E->lists_dirty) {
        int e = upload_lists(E);
        if (e) return e;
    }
    bool any = false;
    for (int s = 0; s < E->hi_slot; ++s) any = any || E->ticket[s] >= 0;
    if (any) {
        for (int r = 0; r < E->o.rounds_per_tick; ++r) {
            if (E->graph_ready) HIPCALL(hipGraphLaunch(E->exec, E->stream));
            else enqueue_round(E);
        }
        HIPCALL(hipGetLastError());
        if (E->hi_slot > 0)
            HIPCALL(hipMemcpyAsync(E->h_dyn, E->d_dyn, sizeof(EDyn) * E->hi_slot,
                                   hipMemcpyDeviceToHost, E->stream));
    }
    HIPCALL(hipStreamSynchronize(E->stream));
    for (int s = 0; s < E->hi_slot; ++s) {
        if (E->ticket[s] < 0) continue;
        const int st = E->h_dyn[s].state;
        if (st == kBegin || st == kActive) {
            *n_active += 1;
        } else if ((st == kFinished || st == kFailed) && !E->reported[s] && *n_done < max_done) {
            done[(*n_done)++] = E->ticket[s];
            E->reported[s] = 1;
        }
    }
    return RS_OK;
}

int rs_engine_fetch(rs_engine *E, int ticket, double *psi_dev, rs_request_stats *st)
{
    if (!E) return fail(RS_EINVAL, "null engine");
    if (st && st->struct_size != sizeof(rs_request_stats))
        return fail(RS_EINVAL, "rs_request_stats.struct_size");
    auto it = E->slot_of.find(ticket);
    if (it == E->slot_of.end()) return fail(RS_EINVAL, "unknown ticket %d", ticket);
    const int s = it->second;
    const EDyn &D = E->h_dyn[s];
    if (D.state != kFinished && D.state != kFailed)
        return fail(RS_ESTATE, "request %d is still running", ticket);
    if (psi_dev)
        HIPCALL(hipMemcpyAsync(psi_dev, E->h_slots[s].psi,
                               sizeof(double) * (size_t)E->plans[s].geo[0].N,
                               hipMemcpyDeviceToDevice, E->stream));
    if (st) {
        st->state = D.state == kFinished ? RS_REQ_FINISHED : RS_REQ_FAILED;
        st->status = D.status;
        st->steps = D.steps_done;
        st->corrections = D.corr_total;
        st->max_step_corrections = std::max(D.corr_max, D.corr);
        st->res = D.res;
    }
    E->arena.release(E->mem_off[s], E->mem_len[s]);
    E->ticket[s] = -1;
    E->slot_of.erase(it);
    E->h_dyn[s].state = kEmpty;
    HIPCALL(hipMemcpyAsync(E->d_dyn + s, &E->h_dyn[s], sizeof(EDyn), hipMemcpyHostToDevice,
                           E->stream));
    E->lists_dirty = true;
    return RS_OK;
}

int rs_engine_capacity(const rs_engine *E, size_t *free_bytes, int *free_slots)
{
    if (!E) return fail(RS_EINVAL, "null engine");
    if (free_bytes) *free_bytes = E->arena.free_bytes();
    if (free_slots) {
        int n = 0;
        for (int s = 0; s < E->o.max_slots; ++s) n += E->ticket[s] < 0;
        *free_slots = n;
    }
    return RS_OK;
}

void rs_engine_destroy(rs_engine *E)
{
    if (!E) return;
    (void)hipStreamSynchronize(E->stream);
    if (E->exec) (void)hipGraphExecDestroy(E->exec);
    if (E->graph) (void)hipGraphDestroy(E->graph);
    if (E->host) (void)hipHostFree(E->host);
    delete E;
}

}  // extern "C"
