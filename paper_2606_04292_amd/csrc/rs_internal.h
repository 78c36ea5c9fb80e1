// Internal structures shared by the kernels and the host orchestration of
// the richards library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

constexpr int kMaxLevels = 16;
constexpr int kBcDirichlet = 1;
constexpr int kBcNoflux = 2;
constexpr int kBcFreedrain = 3;
constexpr int kVgm = 1;
constexpr int kHaverkamp = 2;
constexpr int kLinear = 3;
constexpr int kGardner = 4;
constexpr int kMulti = 5;      // a soil per node (Law::soils), FP64 path only
constexpr int kMaxSoils = 16;
constexpr int kSinkFeddes = 1;
constexpr int kKappaConst = 1;
constexpr int kKappaRel = 2;
constexpr int kKappaRemark = 3;

// Geometry of one level, passed by value to every kernel.
struct Geo {
    int n[3];        // nodes per axis (1 beyond dim)
    int dim;
    int vert;        // vertical axis = dim - 1
    int stride[3];   // 1, n0, n0*n1 (rows of n0 values)
    // Order of the n0 values of a row in memory: node i at position
    // (i >> xs) + (i & 1) xh.  xs = xh = 0: lexicographic (axis 0 fastest);
    // xs = 1, xh = (n0 + 1) / 2: the row split by parity, even nodes first,
    // then odd ones, so that one colour of the red-black ordering fills whole
    // cache lines.
    int xs, xh;
    long long N;     // total nodes
    double h[3];
    double ih2[3];   // 1 / h^2
    int bc[6];       // face kinds
    int state_mask;  // bit f: face f's Dirichlet values come from the state psi^n
    double bcval[6];
    int pface;       // patch face or -1
    int pax, pat;    // the patch face's axis and its coordinate on that axis (0 or n - 1)
    int plo[2], phi[2];
    double pval;
    const unsigned char *soil;   // soil index per node (read only under kMulti)
};

// Soil law and smoother parameters (by value).
struct Law {
    int model;
    double ts, tr, Ks;
    double dT;               // theta_s - theta_r
    double vg_alpha, vg_n, vg_m;
    double hk_alpha, hk_beta, hk_A, hk_gamma, unit;
    double lin_c;
    int sink;
    double h1, h2, h3, h4;
    double xi;
    int kappa_rule;
    double kappa;
    int newton;
    double newton_tol;   // a Newton step of at most newton_tol |x| ends the pointwise solve
    double gd_alpha;     // Gardner exponent (per law unit of psi)
    const Law *soils;    // kMulti: device table of per-soil laws, indexed by Geo::soil
    // binomial coefficients binom(e, k), k = 1..7, of (1 + u)^e - 1: e = hk_beta
    // (Haverkamp) or vg_n (vGM) in bin1, e = -vg_m (vGM) in bin2; the series is
    // used while |u| < series_u (2^-8, or 0 when an exponent lies outside
    // [-1, 7], where the truncation bound below does not hold)
    double bin1[7], bin2[7];
    double series_u;
};

// Step coefficients (by value).
struct Step {
    double a;        // BDF leading coefficient: 1/dt or 3/(2 dt)
    double dt;
    int order;       // effective order (1 or 2)
    int lag_extrap;  // BDF2 lag 2 psi^n - psi^{n-1}
};

// ---------------------------------------------------------------------------
// Small levels in one work-group: per-level records of a grid, kept in its
// workspace (written at creation, lambdaU refreshed at step set-up).
// ---------------------------------------------------------------------------
constexpr long long kTailNodes = 2049;   // levels of at most this many nodes

struct TailLevel {
    Geo g;
    long long cm_total;
    unsigned H, n1;
    unsigned dH_m, dH_s, dN1_m, dN1_s;    // colour-slot division (FastDiv parts)
    unsigned n0, nn1;
    unsigned d0_m, d0_s, d1_m, d1_s;      // node division
    double *psi, *K, *gv, *d, *psibar;
    const double *beta;
    double lambdaU;
    // FP32 correction cycle (mixed grids; null otherwise): delta, K*, rhs,
    // base state, inner defect, restricted delta
    float *dl, *K32, *rhs32, *pb32, *r32, *dbar32;
    float lambdaU32;
};

struct TailArgs {
    TailLevel lv[kMaxLevels];
};

// ---------------------------------------------------------------------------
// Kernel launchers (kernels_fp64.hip)
// ---------------------------------------------------------------------------
// The V-cycle from level top (all of whose levels hold at most kTailNodes
// nodes) down to level last and back, in one work-group.
// nodes[l]: node count of level l (sizes the LDS copy of the deepest levels).
void launch_vcycle_tail(const TailArgs *args_dev, int top, int last, const Law &law,
                        const Step &st, int nu1, int nu2, int nuc, int dim, const long long *nodes,
                        hipStream_t s);
constexpr size_t kTailLds = 56 * 1024;   // LDS for the deepest levels of that cycle
void launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t s);
// Lexicographic (C ABI) order <-> the level's row layout; src and dst must not overlap.
void launch_relayout(const Geo &g, const double *src, double *dst, bool to_level, hipStream_t s);
void launch_relayout_u8(const Geo &g, const unsigned char *src, unsigned char *dst, bool to_level,
                        hipStream_t s);
void launch_setup_kstar(const Geo &g, const Law &law, const Step &st, const double *psi_n,
                        const double *psi_nm1, const double *Ks_field, double *K, double *psi,
                        hipStream_t s);
void launch_setup_g(const Geo &g, const Law &law, const Step &st, const double *psi_n,
                    const double *psi_nm1, const double *K, double *gvec, hipStream_t s);
void launch_inject(const Geo &gc, const Geo &gf, const double *Kf, double *Kc, hipStream_t s);
// Kc = full-weighting average of Kf around each coarse node (mirrored at the ends)
void launch_fw_coarse(const Geo &gc, const Geo &gf, const double *Kf, double *Kc, hipStream_t s);
void launch_inject_u8(const Geo &gc, const Geo &gf, const unsigned char *vf, unsigned char *vc,
                      hipStream_t s);
void launch_lambda_u(const Geo &g, const double *K, unsigned long long *out, hipStream_t s);
// Red-black sweeps; 3-D levels with a second psi buffer use the fused kernel
// and swap *psi / *psi_alt after every sweep.  Returns the kernel launches made.
int launch_sweep_rb(const Geo &g, const Law &law, const Step &st, const double *beta,
                    double lambdaU, const double *K, const double *gvec, double **psi,
                    double **psi_alt, int nsweeps, hipStream_t s);
// Levels that get a second psi buffer for the fused sweep (3-D levels of at
// least kFusedMinNodes nodes, when the fused sweep is selected at grid
// creation).
constexpr long long kFusedMinNodes = 33LL * 33 * 33;
bool fused_sweep_level(const Geo &g);
// Start of an FP32 correction (mixed precision) written by the defect kernel:
// rhs = fl32(defect), psi_b = fl32(psi), delta = 0 on every node.
struct MpStart {
    float *rhs, *pb, *dl;
};
// nsweeps red-black sweeps of a level whose sweeps run two nodes per lane
// (sweep_defect_level), leaving the defect of the swept iterate in d and its
// max-norm folded into norm_bits (the caller zeroes it): phase 0 launches
// every colour pass but the last, phase 1 the last one fused with the defect
// of its nodes and the defect of the other colour.
bool sweep_defect_level(const Geo &g, const Law &law, int nsweeps);
void launch_sweep_defect(const Geo &g, const Law &law, const Step &st, const double *beta,
                         const double *K, const double *gvec, double *psi, int nsweeps, double *d,
                         unsigned long long *norm_bits, int phase, hipStream_t s);
void launch_residual(const Geo &g, const Law &law, const Step &st, const double *beta,
                     const double *K, const double *gvec, const double *psi, double *d,
                     unsigned long long *norm_bits, hipStream_t s, MpStart mp = {});
// max over the unknowns of the summed magnitudes of the defect's terms, as
// the bits of a non-negative double, atomically max-ed into *out
void launch_defect_scale(const Geo &g, const Law &law, const Step &st, const double *beta,
                         const double *K, const double *gvec, const double *psi,
                         unsigned long long *out, hipStream_t s);
void launch_restrict(const Geo &gc, const Geo &gf, const double *psi_f, const double *d_f,
                     double *psibar_c, double *g_c, hipStream_t s);
void launch_coarse_rhs(const Geo &gc, const Law &law, const Step &st, const double *beta,
                       const double *K, const double *psibar, double *gvec, double *psi,
                       hipStream_t s);
void launch_prolong(const Geo &gf, const Geo &gc, const double *psi_c, const double *psibar_c,
                    double *psi_f, hipStream_t s);
// psi_f = linear interpolation of psi_c at fine unknowns (FMG interpolation)
void launch_interp(const Geo &gf, const Geo &gc, const double *psi_c, double *psi_f, hipStream_t s);

}  // namespace rs
