// Host side of the richards library: descriptor validation, workspace
// planning, the multigrid level hierarchy, V-cycle orchestration and the
// C ABI declared in include/richards.h.  All arithmetic on solver data runs
// in the kernels; the host only sequences launches and reads back norms.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/richards.h"
#include "rs_internal.h"
#include "mp_internal.h"
#include "host_common.h"
#include "grid_device.h"

namespace rs {
void launch_root_beta(int nlev, const int *nvert, const double *hvert, double *const *beta,
                      double Lz, double Tp, double root_len, hipStream_t s);
}

using namespace rs;

namespace rs {

thread_local char g_err[512];

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

static bool pow2p1(int n)
{
    if (n < 3) return false;
    int m = n - 1;
    return (m & (m - 1)) == 0;
}

int validate_desc(const rs_grid_desc *d)
{
    if (!d) return fail(RS_EINVAL, "null grid descriptor");
    if (d->struct_size != sizeof(rs_grid_desc))
        return fail(RS_EINVAL, "rs_grid_desc.struct_size %zu != %zu", d->struct_size,
                    sizeof(rs_grid_desc));
    if (d->dim < 1 || d->dim > 3) return fail(RS_EINVAL, "dim must be 1, 2 or 3");
    for (int l = 0; l < d->dim; ++l) {
        if (!pow2p1(d->n[l])) return fail(RS_EINVAL, "n[%d]=%d is not 2^k+1 >= 3", l, d->n[l]);
        if (!(d->L[l] > 0.0)) return fail(RS_EINVAL, "L[%d] must be positive", l);
    }
    for (int f = 0; f < 2 * d->dim; ++f) {
        int b = d->face_bc[f];
        if (b != RS_BC_DIRICHLET && b != RS_BC_NOFLUX && b != RS_BC_FREEDRAIN &&
            b != RS_BC_DIRICHLET_STATE)
            return fail(RS_EINVAL, "face_bc[%d]=%d invalid", f, b);
        if (b == RS_BC_FREEDRAIN && f != 2 * (d->dim - 1))
            return fail(RS_EINVAL, "free drainage is only allowed on the bottom face");
        if (!std::isfinite(d->face_value[f])) return fail(RS_EINVAL, "face_value[%d] not finite", f);
    }
    {
        long long N = 1;
        for (int l = 0; l < d->dim; ++l) N *= d->n[l];
        if (N >= (1ll << 31)) return fail(RS_EINVAL, "grid of %lld nodes; at most 2^31 - 1", N);
    }
    if (d->patch_face >= 0) {
        if (d->patch_face >= 2 * d->dim) return fail(RS_EINVAL, "patch_face out of range");
        if (d->dim < 2) return fail(RS_EINVAL, "a face patch needs dim >= 2");
        int ax = d->patch_face / 2, t = 0;
        for (int l = 0; l < d->dim; ++l) {
            if (l == ax) continue;
            if (d->patch_lo[t] < 0 || d->patch_hi[t] >= d->n[l] || d->patch_lo[t] > d->patch_hi[t])
                return fail(RS_EINVAL, "patch range invalid on axis %d", l);
            ++t;
        }
    }
    return RS_OK;
}

int level_count(const rs_grid_desc *d)
{
    int m = d->n[0];
    for (int l = 1; l < d->dim; ++l) m = d->n[l] < m ? d->n[l] : m;
    int k = 1;
    while (m > 3) { m = (m - 1) / 2 + 1; ++k; }
    return k;
}

Geo make_geo(const rs_grid_desc *d, int lev)
{
    Geo g;
    memset(&g, 0, sizeof g);
    g.dim = d->dim;
    g.vert = d->dim - 1;
    long long N = 1;
    for (int l = 0; l < 3; ++l) {
        if (l < d->dim) {
            g.n[l] = ((d->n[l] - 1) >> lev) + 1;
            g.h[l] = d->L[l] / (g.n[l] - 1);
            g.ih2[l] = 1.0 / (g.h[l] * g.h[l]);
        } else {
            g.n[l] = 1;
            g.h[l] = 1.0;
            g.ih2[l] = 0.0;
        }
        N *= g.n[l];
    }
    g.N = N;
    g.stride[0] = 1;
    g.stride[1] = g.n[0];
    g.stride[2] = g.n[0] * g.n[1];
    for (int f = 0; f < 6; ++f) {
        // a state-valued Dirichlet face is a Dirichlet face whose values come
        // from the state: the kernels see kBcDirichlet plus its bit in state_mask
        const int b = f < 2 * d->dim ? d->face_bc[f] : 0;
        g.bc[f] = b == RS_BC_DIRICHLET_STATE ? kBcDirichlet : b;
        if (b == RS_BC_DIRICHLET_STATE) g.state_mask |= 1 << f;
        g.bcval[f] = f < 2 * d->dim ? d->face_value[f] : 0.0;
    }
    g.pface = d->patch_face;
    if (g.pface >= 0) {
        g.pax = g.pface >> 1;
        g.pat = (g.pface & 1) ? g.n[g.pax] - 1 : 0;
    }
    int s = 1 << lev;
    for (int t = 0; t < 2; ++t) {
        g.plo[t] = (d->patch_lo[t] + s - 1) / s;
        g.phi[t] = d->patch_hi[t] / s;
    }
    g.pval = d->patch_value;
    return g;
}

}  // namespace rs

namespace {

// Workspace layout: per level psi, K, g, d, psibar (FP64) and the root
// density table; fine-level history psi^n, psi^{n-1}, the Ks field; scratch.
struct Layout {
    int nlev;
    size_t lev_off[kMaxLevels][6];   // psi, K, g, d, psibar, psi_alt (fused levels)
    size_t mp_off[kMaxLevels][6];    // RS_MIXED: delta, K32, rhs, r, dbar, psi_b (FP32)
    size_t beta_off[kMaxLevels];
    size_t soil_off[kMaxLevels];     // soil index per node (layered media)
    size_t psi_n, psi_nm1, ks, scratch, tail, soil_tab;
    size_t total;
};

constexpr int kScratchWords = 64;

// Every array is placed with at least kPad zeroed bytes before and after it
// (the workspace is cleared at creation): the single-grid stencils load the
// axis-0 neighbours idx -/+ 1 unconditionally (see stencil<DIM, true>).
constexpr size_t kPad = 256;

void plan(const rs_grid_desc *d, int precision, Layout *L)
{
    size_t off = 0;
    auto place = [&](size_t bytes) {
        off = align_up(off + kPad);
        const size_t at = off;
        off = align_up(off + bytes + kPad);
        return at;
    };
    L->nlev = level_count(d);
    for (int l = 0; l < L->nlev; ++l) {
        Geo g = make_geo(d, l);
        for (int a = 0; a < 5; ++a) L->lev_off[l][a] = place(sizeof(double) * (size_t)g.N);
        L->lev_off[l][5] = fused_sweep_level(g) ? place(sizeof(double) * (size_t)g.N) : 0;
        L->beta_off[l] = place(sizeof(double) * (size_t)g.n[g.vert]);
        L->soil_off[l] = place((size_t)g.N);
        for (int a = 0; a < 6; ++a)
            L->mp_off[l][a] = precision == RS_MIXED ? place(sizeof(float) * (size_t)g.N) : 0;
    }
    size_t N0 = (size_t)make_geo(d, 0).N;
    L->psi_n = place(sizeof(double) * N0);
    L->psi_nm1 = place(sizeof(double) * N0);
    L->ks = place(sizeof(double) * N0);
    L->scratch = place(sizeof(unsigned long long) * kScratchWords);
    L->tail = place(sizeof(TailArgs));
    L->soil_tab = place(sizeof(Law) * kMaxSoils);
    L->total = off;
}

struct LevelData {
    Geo geo;
    double *psi, *K, *g, *d, *psibar, *beta;
    double *psi_alt;   // second psi buffer of the fused sweep (or null)
    float *dl, *K32, *rhs32, *r32, *dbar32, *pb32;   // RS_MIXED correction cycles
    double lambdaU;
    long long unknowns;
};

}  // namespace

namespace rs {

// Unknown (non-Dirichlet) nodes of a level, counted on the host from the same
// index rules the kernels use.
long long count_unknowns(const Geo &g)
{
    long long dirichlet = 0;
    for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j) {
            // a row off the boundary of axes 1 and 2 has only its two end nodes
            // on the domain boundary
            bool row_on_boundary = (g.dim > 1 && (j == 0 || j == g.n[1] - 1)) ||
                                   (g.dim > 2 && (k == 0 || k == g.n[2] - 1));
            int step = row_on_boundary ? 1 : (g.n[0] - 1);
            for (int i = 0; i < g.n[0]; i += step) {
                int c[3] = {i, j, k};
                bool dir = false;
                for (int l = 0; l < g.dim; ++l) {
                    if (c[l] == 0 && g.bc[2 * l] == kBcDirichlet) dir = true;
                    if (c[l] == g.n[l] - 1 && g.bc[2 * l + 1] == kBcDirichlet) dir = true;
                }
                if (g.pface >= 0) {
                    int ax = g.pface >> 1;
                    int at = (g.pface & 1) ? g.n[ax] - 1 : 0;
                    if (c[ax] == at) {
                        bool in = true;
                        int t = 0;
                        for (int l = 0; l < g.dim; ++l) {
                            if (l == ax) continue;
                            if (c[l] < g.plo[t] || c[l] > g.phi[t]) in = false;
                            ++t;
                        }
                        if (in) dir = true;
                    }
                }
                dirichlet += dir ? 1 : 0;
            }
        }
    return g.N - dirichlet;
}

}  // namespace rs

struct rs_grid {
    rs_grid_desc desc;
    int precision;
    hipStream_t stream;
    int device;
    int nlev;
    LevelData lev[kMaxLevels];
    double *psi_n, *psi_nm1, *ks;
    bool has_ks;
    int coarse_k;                     // RS_COARSE_INJECT or RS_COARSE_FW
    unsigned long long *scratch;
    unsigned long long *host_bits;   // pinned readback
    Law *soil_tab;                    // device table of per-soil laws (layered media)
    TailArgs *tail_dev;               // per-level records of the one-work-group cycle
    TailArgs *tail_host;              // pinned copy
    int tail_top;                     // first level run by it (nlev: none)
    Law law;
    Law32 law32;
    bool law_set;
    Step step;
    bool in_step;
    int nstep;
    double t;
    int nu_coarse;
    double updates;                   // pointwise updates since the step began
    bool prof_on;
    std::vector<hipEvent_t> prof_ev;  // start/stop pairs of finest-level sweeps
    std::vector<int> prof_sweeps;
    std::vector<int> prof_launch;
    size_t prof_used;
    double prof_ms;
    long long prof_launches;
    double prof_cells;
    // Graphs of the part of a V-cycle below the finest level ([0] FP64 cycle,
    // [1] FP32 correction cycle): captured on the private stream cap when the
    // kernel arguments they bake in (key) change, replayed on the grid's
    // stream.  cap null: plain launches (grids of rs_bdf_step_static, the
    // fused sweep, RS_GRAPH=0).
    hipStream_t cap;
    hipGraphExec_t cg[2];
    unsigned char cg_key[2][512];
    double cg_updates[2];
    int law_version;
};

namespace rs {

Law make_law(const rs_constitutive *c)
{
    Law L;
    memset(&L, 0, sizeof L);
    L.model = c->model;
    L.ts = c->theta_s;
    L.tr = c->theta_r;
    L.Ks = c->Ks;
    L.dT = c->theta_s - c->theta_r;
    L.vg_alpha = c->vg_alpha;
    L.vg_n = c->vg_n;
    L.vg_m = c->model == RS_VGM ? 1.0 - 1.0 / c->vg_n : 0.0;
    L.hk_alpha = c->hk_alpha;
    L.hk_beta = c->hk_beta;
    L.hk_A = c->hk_A;
    L.hk_gamma = c->hk_gamma;
    L.unit = c->psi_unit > 0.0 ? c->psi_unit : 1.0;
    L.lin_c = c->lin_c;
    L.sink = c->sink;
    L.h1 = c->h1;
    L.h2 = c->h2;
    L.h3 = c->h3;
    L.h4 = c->h4;
    L.xi = c->xi;
    L.kappa_rule = c->kappa_rule;
    L.kappa = c->kappa;
    L.newton = c->newton_iters;
    L.newton_tol = c->newton_tol;
    L.gd_alpha = c->gd_alpha;
    L.soils = nullptr;
    // binom(e, k) = binom(e, k - 1) (e - k + 1) / k
    auto binom = [](double e, double *b) {
        double v = 1.0;
        for (int k = 1; k <= 7; ++k) {
            v *= (e - (k - 1)) / k;
            b[k - 1] = v;
        }
    };
    const double e1 = c->model == RS_HAVERKAMP ? L.hk_beta : L.vg_n;
    binom(e1, L.bin1);
    binom(-L.vg_m, L.bin2);
    L.series_u = (e1 >= -1.0 && e1 <= 7.0 && -L.vg_m >= -1.0) ? 0.00390625 : 0.0;
    if (c->n_soils > 0) L.model = kMulti;   // the table is attached by the grid
    return L;
}

// The constitutive record of one soil of a layered medium: the soil's law
// fields over the shared ones.
rs_constitutive soil_constitutive(const rs_constitutive *c, const rs_soil &s)
{
    rs_constitutive q = *c;
    q.model = s.model;
    q.theta_s = s.theta_s;
    q.theta_r = s.theta_r;
    q.Ks = s.Ks;
    q.vg_alpha = s.vg_alpha;
    q.vg_n = s.vg_n;
    q.hk_alpha = s.hk_alpha;
    q.hk_beta = s.hk_beta;
    q.hk_A = s.hk_A;
    q.hk_gamma = s.hk_gamma;
    q.psi_unit = s.psi_unit;
    q.lin_c = s.lin_c;
    q.gd_alpha = s.gd_alpha;
    q.Ks_field = nullptr;
    q.n_soils = 0;
    q.soils = nullptr;
    q.soil_id = nullptr;
    return q;
}

int validate_law(const rs_constitutive *c)
{
    if (!c) return fail(RS_EINVAL, "null constitutive");
    if (c->struct_size != sizeof(rs_constitutive))
        return fail(RS_EINVAL, "rs_constitutive.struct_size %zu != %zu", c->struct_size,
                    sizeof(rs_constitutive));
    if (c->coarse_kstar != RS_COARSE_INJECT && c->coarse_kstar != RS_COARSE_FW)
        return fail(RS_EINVAL, "coarse_kstar must be RS_COARSE_INJECT or RS_COARSE_FW");
    if (c->n_soils != 0) {
        if (c->n_soils < 0 || c->n_soils > RS_MAX_SOILS)
            return fail(RS_EINVAL, "n_soils must be in 0..%d", RS_MAX_SOILS);
        if (!c->soils || !c->soil_id) return fail(RS_EINVAL, "layered medium needs soils and soil_id");
        if (c->Ks_field) return fail(RS_EINVAL, "a layered medium takes Ks from its soils");
        for (int s = 0; s < c->n_soils; ++s) {
            rs_constitutive q = soil_constitutive(c, c->soils[s]);
            int e = validate_law(&q);
            if (e) return e;
        }
        return RS_OK;
    }
    if (c->model != RS_VGM && c->model != RS_HAVERKAMP && c->model != RS_LINEAR &&
        c->model != RS_GARDNER)
        return fail(RS_EINVAL, "unknown model %d", c->model);
    if (c->model == RS_GARDNER && !(c->gd_alpha > 0.0))
        return fail(RS_EINVAL, "Gardner needs alpha > 0");
    if (c->model != RS_LINEAR && !(c->theta_s > c->theta_r && c->theta_r >= 0.0))
        return fail(RS_EINVAL, "need theta_s > theta_r >= 0");
    if (!(c->Ks > 0.0) && !c->Ks_field) return fail(RS_EINVAL, "Ks must be positive");
    if (c->model == RS_VGM && !(c->vg_n > 1.0 && c->vg_alpha > 0.0))
        return fail(RS_EINVAL, "vGM needs n > 1 and alpha > 0");
    if (c->model == RS_HAVERKAMP &&
        !(c->hk_alpha > 0.0 && c->hk_beta > 0.0 && c->hk_A > 0.0 && c->hk_gamma > 0.0))
        return fail(RS_EINVAL, "Haverkamp parameters must be positive");
    if (c->model == RS_LINEAR && !(c->lin_c >= 0.0)) return fail(RS_EINVAL, "lin_c must be >= 0");
    if (c->sink != RS_SINK_NONE && c->sink != RS_SINK_FEDDES_EXP)
        return fail(RS_EINVAL, "unknown sink %d", c->sink);
    if (c->sink == RS_SINK_FEDDES_EXP &&
        !(c->h4 < c->h3 && c->h3 < c->h2 && c->h2 < c->h1 && c->root_len > 0.0 && c->Tp >= 0.0))
        return fail(RS_EINVAL, "Feddes parameters need h4 < h3 < h2 < h1, root_len > 0, Tp >= 0");
    if (!(c->xi >= 0.0)) return fail(RS_EINVAL, "xi must be >= 0");
    if (c->kappa_rule != RS_KAPPA_CONST && c->kappa_rule != RS_KAPPA_REL &&
        c->kappa_rule != RS_KAPPA_REMARK)
        return fail(RS_EINVAL, "unknown kappa rule %d", c->kappa_rule);
    if (c->kappa_rule != RS_KAPPA_REMARK && !(c->kappa >= 0.0))
        return fail(RS_EINVAL, "kappa must be >= 0");
    if (c->newton_iters < 1 || c->newton_iters > 64)
        return fail(RS_EINVAL, "newton_iters must be in 1..64");
    if (!(c->newton_tol >= 0.0 && c->newton_tol <= 1e-3))
        return fail(RS_EINVAL, "newton_tol must be in 0..1e-3");
    return RS_OK;
}

}  // namespace rs

namespace {

int harvest_profile(rs_grid *G)
{
    for (size_t q = 0; q < G->prof_used; ++q) {
        float ms = 0.f;
        HIPCALL(hipEventElapsedTime(&ms, G->prof_ev[2 * q], G->prof_ev[2 * q + 1]));
        G->prof_ms += ms;
        G->prof_launches += G->prof_launch[q];
        // prof_sweeps counts colour passes: half the unknowns each
        G->prof_cells += 0.5 * (double)G->prof_sweeps[q] * (double)G->lev[0].unknowns;
    }
    G->prof_used = 0;
    return RS_OK;
}

// A free pair of profiling events (created on first use).
hipError_t prof_slot(rs_grid *G)
{
    if (2 * (G->prof_used + 1) <= G->prof_ev.size()) return hipSuccess;
    for (int e = 0; e < 2; ++e) {
        hipEvent_t ev;
        const hipError_t r = hipEventCreate(&ev);
        if (r != hipSuccess) return r;
        G->prof_ev.push_back(ev);
    }
    G->prof_sweeps.push_back(0);
    G->prof_launch.push_back(0);
    return hipSuccess;
}

// nsweeps red-black sweeps on level l, counted, and timed on the finest level
// when profiling is on.
int sweep_level(rs_grid *G, int l, int nsweeps)
{
    LevelData &f = G->lev[l];
    bool timed = G->prof_on && l == 0 && nsweeps > 0;
    if (timed) {
        if (2 * (G->prof_used + 1) > G->prof_ev.size()) {
            for (int e = 0; e < 2; ++e) {
                hipEvent_t ev;
                HIPCALL(hipEventCreate(&ev));
                G->prof_ev.push_back(ev);
            }
            G->prof_sweeps.push_back(0);
            G->prof_launch.push_back(0);
        }
        HIPCALL(hipEventRecord(G->prof_ev[2 * G->prof_used], G->stream));
    }
    int launches = launch_sweep_rb(f.geo, G->law, G->step, f.beta, f.lambdaU, f.K, f.g, &f.psi,
                                   &f.psi_alt, nsweeps, G->stream);
    if (timed) {
        HIPCALL(hipEventRecord(G->prof_ev[2 * G->prof_used + 1], G->stream));
        G->prof_sweeps[G->prof_used] = 2 * nsweeps;
        G->prof_launch[G->prof_used] = launches;
        G->prof_used += 1;
    }
    G->updates += (double)nsweeps * (double)f.unknowns;
    return RS_OK;
}

int read_norm(rs_grid *G, double *out)
{
    HIPCALL(hipMemcpyAsync(G->host_bits, G->scratch, sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, G->stream));
    HIPCALL(hipStreamSynchronize(G->stream));
    if (G->prof_used) {
        int e = harvest_profile(G);
        if (e) return e;
    }
    unsigned long long b = G->host_bits[0];
    double v;
    memcpy(&v, &b, sizeof v);
    *out = v;
    return RS_OK;
}

// FP64 defect max-norm of the finest level (and the defect vector into d; or,
// with mp_start, the start of an FP32 correction: rhs = fl32(defect),
// psi_b = fl32(psi), delta = 0).
int fine_norm(rs_grid *G, double *out, double *d = nullptr, bool mp_start = false)
{
    LevelData &f = G->lev[0];
    launch_fill_u64(G->scratch, 1, 0ull, G->stream);
    MpStart mp{};
    if (mp_start) mp = MpStart{f.rhs32, f.pb32, f.dl};
    launch_residual(f.geo, G->law, G->step, f.beta, f.K, f.g, f.psi, d, G->scratch, G->stream, mp);
    HIPCALL(hipGetLastError());
    return read_norm(G, out);
}

// The pre-smoothing of an FP64 cycle on the finest level and the max-norm of
// the defect it leaves (the defect vector into d): where the level runs the
// pair sweep, the last colour pass forms the defect of its nodes on the way
// and one more pass that of the others; otherwise the sweeps, then the defect
// kernel.  The same d and norm either way.
int presmooth_norm(rs_grid *G, int nu1, double *out)
{
    LevelData &f = G->lev[0];
    if (f.psi_alt || !sweep_defect_level(f.geo, G->law, nu1)) {
        int e = sweep_level(G, 0, nu1);
        if (e) return e;
        return fine_norm(G, out, f.d);
    }
    launch_fill_u64(G->scratch, 1, 0ull, G->stream);
    // the plain colour passes are timed like any sweep batch of the level
    const bool timed = G->prof_on;
    if (timed) {
        HIPCALL(prof_slot(G));
        HIPCALL(hipEventRecord(G->prof_ev[2 * G->prof_used], G->stream));
    }
    launch_sweep_defect(f.geo, G->law, G->step, f.beta, f.K, f.g, f.psi, nu1, f.d, G->scratch, 0,
                        G->stream);
    if (timed) {
        HIPCALL(hipEventRecord(G->prof_ev[2 * G->prof_used + 1], G->stream));
        G->prof_sweeps[G->prof_used] = 2 * nu1 - 1;
        G->prof_launch[G->prof_used] = 2 * nu1 - 1;
        G->prof_used += 1;
    }
    launch_sweep_defect(f.geo, G->law, G->step, f.beta, f.K, f.g, f.psi, nu1, f.d, G->scratch, 1,
                        G->stream);
    HIPCALL(hipGetLastError());
    G->updates += (double)nu1 * (double)f.unknowns;
    return read_norm(G, out);
}

// Scale of the defect's rounding floor on the finest level: the largest sum
// of the magnitudes of the terms one node's defect adds up.
int defect_scale(rs_grid *G, double *out)
{
    LevelData &f = G->lev[0];
    unsigned long long *w = G->scratch + (kScratchWords - 1);
    launch_fill_u64(w, 1, 0ull, G->stream);
    launch_defect_scale(f.geo, G->law, G->step, f.beta, f.K, f.g, f.psi, w, G->stream);
    HIPCALL(hipGetLastError());
    HIPCALL(hipMemcpyAsync(G->host_bits + (kScratchWords - 1), w, sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, G->stream));
    HIPCALL(hipStreamSynchronize(G->stream));
    memcpy(out, &G->host_bits[kScratchWords - 1], sizeof(double));
    return RS_OK;
}

// A stall of the cycle counts as the rounding floor when the residual of the
// iterate that is kept is within 16 ulp of the defect's term scale (the
// largest per-node sum of the magnitudes of the terms that the defect and the
// pointwise solve of that node add up).
constexpr double kFloorRel = 16.0 * 2.220446049250313e-16;

// FP32 red-black sweeps of the correction equation on level l.
void sweep32_level(rs_grid *G, int l, int nsweeps)
{
    LevelData &f = G->lev[l];
    bool timed = G->prof_on && l == 0 && nsweeps > 0;
    if (timed && 2 * (G->prof_used + 1) > G->prof_ev.size()) {
        for (int e = 0; e < 2; ++e) {
            hipEvent_t ev;
            if (hipEventCreate(&ev) != hipSuccess) { timed = false; break; }
            G->prof_ev.push_back(ev);
        }
        G->prof_sweeps.push_back(0);
        G->prof_launch.push_back(0);
    }
    if (timed) timed = hipEventRecord(G->prof_ev[2 * G->prof_used], G->stream) == hipSuccess;
    launch_sweep32(f.geo, G->law32, (float)G->step.a, f.beta, (float)f.lambdaU, f.K32, f.rhs32,
                   f.pb32, f.dl, nsweeps, G->stream);
    if (timed && hipEventRecord(G->prof_ev[2 * G->prof_used + 1], G->stream) == hipSuccess) {
        G->prof_sweeps[G->prof_used] = 2 * nsweeps;
        G->prof_launch[G->prof_used] = f.geo.N <= 1024 ? 1 : 2 * nsweeps;
        G->prof_used += 1;
    }
    G->updates += (double)nsweeps * (double)f.unknowns;
}

int vcycle_level(rs_grid *G, int l, int nu1, int nu2);
void vcycle32_level(rs_grid *G, int l, int nu1, int nu2);

// The part of a V-cycle below the finest level, as plain launches: the
// restriction of the fine iterate and of its defect (FP64: already in the
// level's d), the coarse right-hand side, the cycle on level 1 and below, the
// prolongation.  which = 1: the FP32 correction cycle, which first forms its
// inner defect (the coarse levels hold the injected base state psi_b).
void coarse_cycle_plain(rs_grid *G, int which, int nu1, int nu2)
{
    LevelData &f = G->lev[0], &c = G->lev[1];
    if (which == 0) {
        launch_restrict(c.geo, f.geo, f.psi, f.d, c.psibar, c.g, G->stream);
        launch_coarse_rhs(c.geo, G->law, G->step, c.beta, c.K, c.psibar, c.g, c.psi, G->stream);
        vcycle_level(G, 1, nu1, nu2);
        launch_prolong(f.geo, c.geo, c.psi, c.psibar, f.psi, G->stream);
        return;
    }
    const float a = (float)G->step.a;
    launch_residual32(f.geo, G->law32, a, f.beta, f.K32, f.rhs32, f.pb32, f.dl, f.r32, G->stream);
    launch_restrict32(c.geo, f.geo, f.dl, f.r32, c.dbar32, c.rhs32, G->stream);
    launch_coarse_rhs32(c.geo, G->law32, a, c.beta, c.K32, c.pb32, c.dbar32, c.rhs32, c.dl, G->stream);
    vcycle32_level(G, 1, nu1, nu2);
    launch_prolong32(f.geo, c.geo, c.dl, c.dbar32, f.dl, G->stream);
}

// What the coarse-cycle graph bakes into its kernel arguments.
struct CycleKey {
    double a, dt;
    int order, lag_extrap, nu1, nu2, nu_coarse, law_version;
    double lambdaU[kMaxLevels];
};

// The coarse part of a V-cycle: replays its graph (captured again when the
// step coefficients, the law, the cycle counts or the shift change), or
// launches it plainly on grids without graphs.  A capture that fails turns
// the graphs off for the grid.
int coarse_cycle(rs_grid *G, int which, int nu1, int nu2)
{
    if (!G->cap) {
        coarse_cycle_plain(G, which, nu1, nu2);
        return RS_OK;
    }
    CycleKey k;
    static_assert(sizeof(CycleKey) <= sizeof(G->cg_key[0]), "key size");
    memset(&k, 0, sizeof k);
    k.a = G->step.a;
    k.dt = G->step.dt;
    k.order = G->step.order;
    k.lag_extrap = G->step.lag_extrap;
    k.nu1 = nu1;
    k.nu2 = nu2;
    k.nu_coarse = G->nu_coarse;
    k.law_version = G->law_version;
    for (int l = 0; l < G->nlev; ++l) k.lambdaU[l] = G->lev[l].lambdaU;
    if (!G->cg[which] || memcmp(&k, G->cg_key[which], sizeof k) != 0) {
        if (G->cg[which]) {
            HIPCALL(hipStreamSynchronize(G->stream));   // a replay may still run
            HIPCALL(hipGraphExecDestroy(G->cg[which]));
            G->cg[which] = nullptr;
        }
        hipStream_t s = G->stream;
        const bool prof = G->prof_on;
        const double u = G->updates;
        hipGraph_t gr = nullptr;
        bool ok = hipStreamBeginCapture(G->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            G->stream = G->cap;
            G->prof_on = false;
            coarse_cycle_plain(G, which, nu1, nu2);
            ok = hipStreamEndCapture(G->cap, &gr) == hipSuccess && gr;
            G->stream = s;
            G->prof_on = prof;
        }
        G->cg_updates[which] = G->updates - u;
        G->updates = u;
        if (ok) ok = hipGraphInstantiate(&G->cg[which], gr, nullptr, nullptr, 0) == hipSuccess;
        if (gr) (void)hipGraphDestroy(gr);
        (void)hipGetLastError();
        if (!ok) {
            // no graphs for this grid from now on
            G->cg[which] = nullptr;
            coarse_cycle_plain(G, which, nu1, nu2);
            HIPCALL(hipGetLastError());
            (void)hipStreamDestroy(G->cap);
            G->cap = nullptr;
            return RS_OK;
        }
        memcpy(G->cg_key[which], &k, sizeof k);
    }
    HIPCALL(hipGraphLaunch(G->cg[which], G->stream));
    G->updates += G->cg_updates[which];
    return RS_OK;
}

// FP32 FAS V-cycle on the correction equation (same structure as the FP64 one).
void vcycle32_level(rs_grid *G, int l, int nu1, int nu2)
{
    LevelData &f = G->lev[l];
    const float a = (float)G->step.a;
    if (l >= 1 && l >= G->tail_top && l < G->nlev - 1) {
        // the rest of the correction cycle on small levels: one work-group
        launch_vcycle_tail32(G->tail_dev, l, G->nlev - 1, G->law32, a, nu1, nu2, G->nu_coarse,
                             G->desc.dim, G->stream);
        for (int q = l; q < G->nlev - 1; ++q)
            G->updates += (double)(nu1 + nu2) * (double)G->lev[q].unknowns;
        // the coarsest level's loop may stop after its first sweep (4-ulp exit):
        // counted as one sweep
        G->updates += (double)G->lev[G->nlev - 1].unknowns;
        return;
    }
    if (l == G->nlev - 1) {
        sweep32_level(G, l, G->nu_coarse);
        return;
    }
    if (l == 0) {
        sweep32_level(G, 0, nu1);
        (void)coarse_cycle(G, 1, nu1, nu2);
        sweep32_level(G, 0, nu2);
        return;
    }
    LevelData &c = G->lev[l + 1];
    sweep32_level(G, l, nu1);
    launch_residual32(f.geo, G->law32, a, f.beta, f.K32, f.rhs32, f.pb32, f.dl, f.r32, G->stream);
    launch_restrict32(c.geo, f.geo, f.dl, f.r32, c.dbar32, c.rhs32, G->stream);
    launch_coarse_rhs32(c.geo, G->law32, a, c.beta, c.K32, c.pb32, c.dbar32, c.rhs32, c.dl, G->stream);
    vcycle32_level(G, l + 1, nu1, nu2);
    launch_prolong32(f.geo, c.geo, c.dl, c.dbar32, f.dl, G->stream);
    sweep32_level(G, l, nu2);
}

// One outer defect correction: the defect kernel has already written the FP32
// right-hand side fl32(r), the base state fl32(psi) and delta = 0 on the finest
// level (fine_norm with mp_start); psi_b is injected into the coarse levels
// once, FP32 cycles solve the correction equation and psi += delta in FP64.
void mp_correction(rs_grid *G, int inner, int nu1, int nu2)
{
    LevelData &f = G->lev[0];
    Geo geo[kMaxLevels];
    float *pb[kMaxLevels];
    for (int l = 0; l < G->nlev; ++l) {
        geo[l] = G->lev[l].geo;
        pb[l] = G->lev[l].pb32;
    }
    launch_inject_base32(geo, pb, G->nlev, G->stream);
    for (int c = 0; c < inner; ++c) vcycle32_level(G, 0, nu1, nu2);
    launch_apply_delta(f.geo.N, f.dl, f.psi, G->stream);
}

int vcycle_level(rs_grid *G, int l, int nu1, int nu2)
{
    LevelData &f = G->lev[l];
    if (l >= G->tail_top && l < G->nlev - 1) {
        // the rest of the cycle on small levels: one work-group, one launch
        long long nodes[kMaxLevels];
        for (int q = 0; q < G->nlev; ++q) nodes[q] = G->lev[q].geo.N;
        launch_vcycle_tail(G->tail_dev, l, G->nlev - 1, G->law, G->step, nu1, nu2, G->nu_coarse,
                           G->desc.dim, nodes, G->stream);
        for (int q = l; q < G->nlev - 1; ++q)
            G->updates += (double)(nu1 + nu2) * (double)G->lev[q].unknowns;
        // the coarsest level's loop may stop after its first sweep (4-ulp exit):
        // counted as one sweep
        G->updates += (double)G->lev[G->nlev - 1].unknowns;
        return RS_OK;
    }
    if (l == G->nlev - 1) return sweep_level(G, l, G->nu_coarse);
    if (l == 0) {
        int e = sweep_level(G, 0, nu1);
        if (e) return e;
        launch_residual(f.geo, G->law, G->step, f.beta, f.K, f.g, f.psi, f.d, nullptr, G->stream);
        e = coarse_cycle(G, 0, nu1, nu2);
        if (!e) e = sweep_level(G, 0, nu2);
        return e;
    }
    LevelData &c = G->lev[l + 1];
    int e = sweep_level(G, l, nu1);
    if (e) return e;
    launch_residual(f.geo, G->law, G->step, f.beta, f.K, f.g, f.psi, f.d, nullptr, G->stream);
    launch_restrict(c.geo, f.geo, f.psi, f.d, c.psibar, c.g, G->stream);
    launch_coarse_rhs(c.geo, G->law, G->step, c.beta, c.K, c.psibar, c.g, c.psi, G->stream);
    e = vcycle_level(G, l + 1, nu1, nu2);
    if (e) return e;
    launch_prolong(f.geo, c.geo, c.psi, c.psibar, f.psi, G->stream);
    return sweep_level(G, l, nu2);
}

// Full multigrid (FMG): right-hand side restricted down the hierarchy by full
// weighting (zero at Dirichlet nodes), iterate injected; nu_coarse sweeps on
// the coarsest level; then per finer level the linear interpolation of the
// coarser solution and one FAS V-cycle with that level's right-hand side.
int fmg_cycle(rs_grid *G, int nu1, int nu2)
{
    for (int l = 0; l + 1 < G->nlev; ++l) {
        LevelData &f = G->lev[l], &c = G->lev[l + 1];
        launch_restrict(c.geo, f.geo, f.psi, f.g, c.psibar, c.g, G->stream);
        launch_inject(c.geo, f.geo, f.psi, c.psi, G->stream);
    }
    int e = sweep_level(G, G->nlev - 1, G->nu_coarse);
    if (e) return e;
    for (int l = G->nlev - 2; l >= 0; --l) {
        launch_interp(G->lev[l].geo, G->lev[l + 1].geo, G->lev[l + 1].psi, G->lev[l].psi,
                      G->stream);
        e = vcycle_level(G, l, nu1, nu2);
        if (e) return e;
    }
    return RS_OK;
}

double *field_ptr(const rs_grid *G, int level, int field)
{
    const LevelData &L = G->lev[level];
    switch (field) {
    case RS_FIELD_PSI: return L.psi;
    case RS_FIELD_KSTAR: return L.K;
    case RS_FIELD_G: return L.g;
    case RS_FIELD_PSIBAR: return L.psibar;
    default: return nullptr;
    }
}

// Fill G (a value-initialised rs_grid) as a view of a planned workspace at
// base: level arrays, history, scratch words, the one-work-group cycle's
// records; host_bits (kScratchWords words) and tail_host are the host-side
// read-back and staging buffers.  Allocates nothing; queues the copy of the
// cycle records on the stream.
int grid_view(rs_grid *G, const rs_grid_desc *d, int precision, const Layout &L, char *base,
              hipStream_t stream, unsigned long long *host_bits, TailArgs *tail_host)
{
    G->desc = *d;
    G->precision = precision;
    G->stream = stream;
    if (hipGetDevice(&G->device) != hipSuccess) G->device = -1;
    G->nlev = L.nlev;
    for (int l = 0; l < L.nlev; ++l) {
        LevelData &v = G->lev[l];
        v.geo = make_geo(d, l);
        // rows split by parity: a colour pass reads and writes whole cache
        // lines of its own colour (the C ABI exchanges lexicographic arrays)
        v.geo.xs = 1;
        v.geo.xh = (v.geo.n[0] + 1) / 2;
        v.geo.soil = (const unsigned char *)(base + L.soil_off[l]);
        v.psi = (double *)(base + L.lev_off[l][0]);
        v.K = (double *)(base + L.lev_off[l][1]);
        v.g = (double *)(base + L.lev_off[l][2]);
        v.d = (double *)(base + L.lev_off[l][3]);
        v.psibar = (double *)(base + L.lev_off[l][4]);
        v.psi_alt = L.lev_off[l][5] ? (double *)(base + L.lev_off[l][5]) : nullptr;
        float **mp[6] = {&v.dl, &v.K32, &v.rhs32, &v.r32, &v.dbar32, &v.pb32};
        for (int a = 0; a < 6; ++a)
            *mp[a] = L.mp_off[l][a] ? (float *)(base + L.mp_off[l][a]) : nullptr;
        v.beta = (double *)(base + L.beta_off[l]);
        v.lambdaU = 0.0;
        v.unknowns = count_unknowns(v.geo);
    }
    G->psi_n = (double *)(base + L.psi_n);
    G->psi_nm1 = (double *)(base + L.psi_nm1);
    G->ks = (double *)(base + L.ks);
    G->scratch = (unsigned long long *)(base + L.scratch);
    G->soil_tab = (Law *)(base + L.soil_tab);
    G->has_ks = false;
    G->law_set = false;
    G->in_step = false;
    G->nstep = 0;
    G->t = 0.0;
    G->nu_coarse = 32;
    G->coarse_k = RS_COARSE_INJECT;
    G->updates = 0.0;
    G->prof_on = false;
    G->prof_used = 0;
    G->prof_ms = 0.0;
    G->prof_launches = 0;
    G->prof_cells = 0.0;
    G->host_bits = host_bits;
    G->tail_dev = (TailArgs *)(base + L.tail);
    G->tail_host = tail_host;
    memset(G->tail_host, 0, sizeof(TailArgs));
    G->tail_top = G->nlev;
    for (int l = G->nlev - 1; l >= 0 && G->lev[l].geo.N <= kTailNodes && !G->lev[l].psi_alt; --l)
        G->tail_top = l;
    for (int l = 0; l < G->nlev; ++l) {
        const LevelData &v = G->lev[l];
        TailLevel &T = G->tail_host->lv[l];
        const ColourMap cm = colour_map(v.geo);
        const NodeMap nm = node_map(v.geo);
        T.g = v.geo;
        T.cm_total = (long long)cm.total;
        T.H = cm.H;
        T.n1 = cm.n1;
        T.dH_m = cm.dH.m;
        T.dH_s = cm.dH.s;
        T.dN1_m = cm.dN1.m;
        T.dN1_s = cm.dN1.s;
        T.n0 = nm.n0;
        T.nn1 = nm.n1;
        T.d0_m = nm.d0.m;
        T.d0_s = nm.d0.s;
        T.d1_m = nm.d1.m;
        T.d1_s = nm.d1.s;
        T.psi = v.psi;
        T.K = v.K;
        T.gv = v.g;
        T.d = v.d;
        T.psibar = v.psibar;
        T.beta = v.beta;
        T.lambdaU = 0.0;
        T.dl = v.dl;
        T.K32 = v.K32;
        T.rhs32 = v.rhs32;
        T.pb32 = v.pb32;
        T.r32 = v.r32;
        T.dbar32 = v.dbar32;
        T.lambdaU32 = 0.0f;
    }
    HIPCALL(hipMemcpyAsync(G->tail_dev, G->tail_host, sizeof(TailArgs), hipMemcpyHostToDevice,
                           G->stream));
    return RS_OK;
}

// Device memory of rs_bdf_step_static: the whole FP64 workspace of one grid
// (level arrays, history, norm words, cycle records), so that the call needs
// no allocation.  Each device holds its own copy for the life of the process.
static __device__ __align__(256) unsigned char scratch[RS_STATIC_WORKSPACE_BYTES];

// Per device: the device address of that copy (hipGetSymbolAddress, once, on
// the first call with the device current) and the host-side read-back and
// staging words of its grid.
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices];
unsigned long long g_static_bits[kMaxDevices][kScratchWords];
TailArgs g_static_tail[kMaxDevices];

}  // namespace

extern "C" {

const char *rs_last_error(void) { return g_err; }

int rs_workspace_bytes(const rs_grid_desc *d, int precision, size_t *out)
{
    int e = validate_desc(d);
    if (e) return e;
    if (precision != RS_FP64 && precision != RS_MIXED) return fail(RS_EINVAL, "bad precision");
    if (!out) return fail(RS_EINVAL, "null out");
    Layout L;
    plan(d, precision, &L);
    *out = L.total;
    return RS_OK;
}

int rs_create_grid(const rs_grid_desc *d, int precision, void *ws_dev, size_t ws_bytes,
                   void *stream, rs_grid **out)
{
    int e = validate_desc(d);
    if (e) return e;
    if (precision != RS_FP64 && precision != RS_MIXED) return fail(RS_EINVAL, "bad precision");
    if (!out) return fail(RS_EINVAL, "null out");
    if (!ws_dev) return fail(RS_EINVAL, "null workspace");
    if (((uintptr_t)ws_dev) % kAlign) return fail(RS_EINVAL, "workspace must be 256-byte aligned");
    Layout L;
    plan(d, precision, &L);
    if (ws_bytes < L.total)
        return fail(RS_ENOMEM, "workspace %zu bytes < required %zu", ws_bytes, L.total);
    // the padding around every array must hold finite values (zeros)
    HIPCALL(hipMemsetAsync(ws_dev, 0, L.total, (hipStream_t)stream));
    rs_grid *G = new (std::nothrow) rs_grid();
    if (!G) return fail(RS_ENOMEM, "host allocation failed");
    unsigned long long *bits = nullptr;
    TailArgs *tail = nullptr;
    if (hipHostMalloc((void **)&bits, kScratchWords * sizeof(unsigned long long),
                      hipHostMallocDefault) != hipSuccess) {
        delete G;
        return fail(RS_EHIP, "hipHostMalloc failed");
    }
    if (hipHostMalloc((void **)&tail, sizeof(TailArgs), hipHostMallocDefault) != hipSuccess) {
        (void)hipHostFree(bits);
        delete G;
        return fail(RS_EHIP, "hipHostMalloc failed");
    }
    e = grid_view(G, d, precision, L, (char *)ws_dev, (hipStream_t)stream, bits, tail);
    const char *gv = getenv("RS_GRAPH");
    const bool fused = G->nlev > 0 && G->lev[0].psi_alt;
    if (!e && !(gv && gv[0] == '0') && !fused && hipStreamCreate(&G->cap) != hipSuccess) {
        (void)hipGetLastError();
        G->cap = nullptr;
    }
    if (e) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        (void)hipHostFree(tail);
        (void)hipHostFree(bits);
        delete G;
        return e;
    }
    *out = G;
    return RS_OK;
}

void rs_destroy_grid(rs_grid *G)
{
    if (!G) return;
    (void)hipStreamSynchronize(G->stream);   // queued copies read the pinned buffers
    for (int w = 0; w < 2; ++w)
        if (G->cg[w]) (void)hipGraphExecDestroy(G->cg[w]);
    if (G->cap) (void)hipStreamDestroy(G->cap);
    for (hipEvent_t ev : G->prof_ev) (void)hipEventDestroy(ev);
    if (G->host_bits) (void)hipHostFree(G->host_bits);
    if (G->tail_host) (void)hipHostFree(G->tail_host);
    delete G;
}

int rs_set_constitutive(rs_grid *G, const rs_constitutive *c)
{
    if (!G) return fail(RS_EINVAL, "null grid");
    int e = validate_law(c);
    if (e) return e;
    if (G->precision == RS_MIXED && (c->n_soils > 0 || c->model == RS_GARDNER))
        return fail(RS_EINVAL, "layered media and the Gardner law need an RS_FP64 grid");
    if (c->n_soils > 0) {
        const long long N = G->lev[0].geo.N;
        for (long long i = 0; i < N; ++i)
            if (c->soil_id[i] >= c->n_soils)
                return fail(RS_EINVAL, "soil_id[%lld] = %d >= n_soils", i, (int)c->soil_id[i]);
        Law tab[kMaxSoils];
        for (int s = 0; s < c->n_soils; ++s) {
            rs_constitutive q = soil_constitutive(c, c->soils[s]);
            tab[s] = make_law(&q);
        }
        HIPCALL(hipMemcpyAsync(G->soil_tab, tab, sizeof(Law) * (size_t)c->n_soils,
                               hipMemcpyHostToDevice, G->stream));
        // staged in the level's defect array, then reordered to the row layout
        unsigned char *stage = (unsigned char *)G->lev[0].d;
        HIPCALL(hipMemcpyAsync(stage, c->soil_id, (size_t)N, hipMemcpyHostToDevice, G->stream));
        launch_relayout_u8(G->lev[0].geo, stage, (unsigned char *)G->lev[0].geo.soil, true,
                           G->stream);
        for (int l = 1; l < G->nlev; ++l)
            launch_inject_u8(G->lev[l].geo, G->lev[l - 1].geo, G->lev[l - 1].geo.soil,
                             (unsigned char *)G->lev[l].geo.soil, G->stream);
        HIPCALL(hipGetLastError());
        HIPCALL(hipStreamSynchronize(G->stream));   // the host table and ids are the caller's
    }
    G->law = make_law(c);
    if (c->n_soils > 0) G->law.soils = G->soil_tab;
    G->law32 = make_law32(G->law);
    G->step.lag_extrap = c->lag_extrap ? 1 : 0;
    G->coarse_k = c->coarse_kstar;
    if (c->Ks_field) {
        size_t bytes = sizeof(double) * (size_t)G->lev[0].geo.N;
        HIPCALL(hipMemcpyAsync(G->lev[0].d, c->Ks_field, bytes, hipMemcpyHostToDevice, G->stream));
        launch_relayout(G->lev[0].geo, G->lev[0].d, G->ks, true, G->stream);
        HIPCALL(hipGetLastError());
        HIPCALL(hipStreamSynchronize(G->stream));
        G->has_ks = true;
    } else {
        G->has_ks = false;
    }
    if (c->sink == RS_SINK_FEDDES_EXP) {
        int nv[kMaxLevels];
        double hv[kMaxLevels];
        double *bp[kMaxLevels];
        for (int l = 0; l < G->nlev; ++l) {
            const Geo &g = G->lev[l].geo;
            nv[l] = g.n[g.vert];
            hv[l] = g.h[g.vert];
            bp[l] = G->lev[l].beta;
        }
        int v = G->desc.dim - 1;
        launch_root_beta(G->nlev, nv, hv, bp, G->desc.L[v], c->Tp, c->root_len, G->stream);
        HIPCALL(hipGetLastError());
    }
    G->law_set = true;
    G->law_version += 1;
    return RS_OK;
}

int rs_set_state(rs_grid *G, const double *psi_n, const double *psi_nm1, int nstep, double t)
{
    if (!G || !psi_n) return fail(RS_EINVAL, "null argument");
    const Geo &g0 = G->lev[0].geo;
    launch_relayout(g0, psi_n, G->psi_n, true, G->stream);
    launch_relayout(g0, psi_nm1 ? psi_nm1 : psi_n, G->psi_nm1, true, G->stream);
    HIPCALL(hipGetLastError());
    G->nstep = nstep;
    G->t = t;
    G->in_step = false;
    return RS_OK;
}

int rs_get_state(const rs_grid *G, double *psi_n, double *psi_nm1, int *nstep, double *t)
{
    if (!G) return fail(RS_EINVAL, "null grid");
    const Geo &g0 = G->lev[0].geo;
    if (psi_n) launch_relayout(g0, G->psi_n, psi_n, false, G->stream);
    if (psi_nm1) launch_relayout(g0, G->psi_nm1, psi_nm1, false, G->stream);
    HIPCALL(hipGetLastError());
    if (nstep) *nstep = G->nstep;
    if (t) *t = G->t;
    return RS_OK;
}

int rs_begin_step(rs_grid *G, double dt, int order)
{
    if (!G) return fail(RS_EINVAL, "null grid");
    if (!G->law_set) return fail(RS_ESTATE, "rs_set_constitutive must come first");
    if (!(dt > 0.0)) return fail(RS_EINVAL, "dt must be positive");
    if (order != 1 && order != 2) return fail(RS_EINVAL, "order must be 1 or 2");
    G->step.dt = dt;
    G->step.order = (order == 2 && G->nstep > 0) ? 2 : 1;
    G->step.a = (G->step.order == 1) ? 1.0 / dt : 1.5 / dt;
    LevelData &f = G->lev[0];
    launch_setup_kstar(f.geo, G->law, G->step, G->psi_n, G->psi_nm1, G->has_ks ? G->ks : nullptr,
                       f.K, f.psi, G->stream);
    launch_setup_g(f.geo, G->law, G->step, G->psi_n, G->psi_nm1, f.K, f.g, G->stream);
    for (int l = 1; l < G->nlev; ++l) {
        if (G->coarse_k == RS_COARSE_FW)
            launch_fw_coarse(G->lev[l].geo, G->lev[l - 1].geo, G->lev[l - 1].K, G->lev[l].K, G->stream);
        else
            launch_inject(G->lev[l].geo, G->lev[l - 1].geo, G->lev[l - 1].K, G->lev[l].K, G->stream);
    }
    if (G->precision == RS_MIXED)
        for (int l = 0; l < G->nlev; ++l)
            launch_to_f32(G->lev[l].geo.N, G->lev[l].K, G->lev[l].K32, G->stream);
    HIPCALL(hipGetLastError());
    if (G->law.kappa_rule == kKappaRemark) {
        launch_fill_u64(G->scratch + 1, G->nlev, 0ull, G->stream);
        for (int l = 0; l < G->nlev; ++l)
            launch_lambda_u(G->lev[l].geo, G->lev[l].K, G->scratch + 1 + l, G->stream);
        HIPCALL(hipMemcpyAsync(G->host_bits + 1, G->scratch + 1,
                               sizeof(unsigned long long) * G->nlev, hipMemcpyDeviceToHost,
                               G->stream));
        HIPCALL(hipStreamSynchronize(G->stream));
        for (int l = 0; l < G->nlev; ++l) {
            double v;
            memcpy(&v, &G->host_bits[1 + l], sizeof v);
            G->lev[l].lambdaU = v;
            G->tail_host->lv[l].lambdaU = v;   // the stream is idle: the last copy is done
            G->tail_host->lv[l].lambdaU32 = (float)v;
        }
        if (G->tail_top < G->nlev)
            HIPCALL(hipMemcpyAsync(G->tail_dev, G->tail_host, sizeof(TailArgs),
                                   hipMemcpyHostToDevice, G->stream));
    }
    G->in_step = true;
    return RS_OK;
}

int rs_sweep(rs_grid *G, int level, int nsweeps)
{
    if (!G) return fail(RS_EINVAL, "null grid");
    if (!G->in_step) return fail(RS_ESTATE, "no active step (call rs_begin_step)");
    if (level < 0 || level >= G->nlev) return fail(RS_EINVAL, "level out of range");
    if (nsweeps < 0) return fail(RS_EINVAL, "nsweeps < 0");
    int e = sweep_level(G, level, nsweeps);
    if (e) return e;
    HIPCALL(hipGetLastError());
    return RS_OK;
}

int rs_vcycle(rs_grid *G, int nu1, int nu2, double *res)
{
    if (!G) return fail(RS_EINVAL, "null grid");
    if (!G->in_step) return fail(RS_ESTATE, "no active step (call rs_begin_step)");
    if (nu1 < 0 || nu2 < 0) return fail(RS_EINVAL, "negative smoothing count");
    int e = vcycle_level(G, 0, nu1, nu2);
    if (e) return e;
    HIPCALL(hipGetLastError());
    if (res) return fine_norm(G, res);
    return RS_OK;
}

int rs_fmg(rs_grid *G, int nu1, int nu2, double *res)
{
    if (!G) return fail(RS_EINVAL, "null grid");
    if (!G->in_step) return fail(RS_ESTATE, "no active step (call rs_begin_step)");
    if (nu1 < 0 || nu2 < 0) return fail(RS_EINVAL, "negative smoothing count");
    int e = fmg_cycle(G, nu1, nu2);
    if (e) return e;
    HIPCALL(hipGetLastError());
    if (res) return fine_norm(G, res);
    return RS_OK;
}

int rs_correction_cycle(rs_grid *G, int inner_cycles, int nu1, int nu2, double *res)
{
    if (!G) return fail(RS_EINVAL, "null grid");
    if (G->precision != RS_MIXED) return fail(RS_ESTATE, "grid was not created with RS_MIXED");
    if (!G->in_step) return fail(RS_ESTATE, "no active step (call rs_begin_step)");
    if (inner_cycles < 1 || nu1 < 0 || nu2 < 0) return fail(RS_EINVAL, "bad cycle counts");
    double r;
    int e = fine_norm(G, &r, nullptr, true);
    if (e) return e;
    mp_correction(G, inner_cycles, nu1, nu2);
    HIPCALL(hipGetLastError());
    if (res) return fine_norm(G, res);
    return RS_OK;
}

int rs_residual_norm(rs_grid *G, double *out)
{
    if (!G || !out) return fail(RS_EINVAL, "null argument");
    if (!G->in_step) return fail(RS_ESTATE, "no active step (call rs_begin_step)");
    int e = fine_norm(G, out);
    if (e) return e;
    if (!std::isfinite(*out)) return fail(RS_ENONFINITE, "residual is not finite");
    return RS_OK;
}

int rs_residual(rs_grid *G, double *d_dev)
{
    if (!G || !d_dev) return fail(RS_EINVAL, "null argument");
    if (!G->in_step) return fail(RS_ESTATE, "no active step (call rs_begin_step)");
    LevelData &f = G->lev[0];
    launch_residual(f.geo, G->law, G->step, f.beta, f.K, f.g, f.psi, f.d, nullptr, G->stream);
    launch_relayout(f.geo, f.d, d_dev, false, G->stream);
    HIPCALL(hipGetLastError());
    return RS_OK;
}

int rs_end_step(rs_grid *G)
{
    if (!G) return fail(RS_EINVAL, "null grid");
    if (!G->in_step) return fail(RS_ESTATE, "no active step");
    double *tmp = G->psi_nm1;
    G->psi_nm1 = G->psi_n;
    G->psi_n = tmp;
    size_t bytes = sizeof(double) * (size_t)G->lev[0].geo.N;
    HIPCALL(hipMemcpyAsync(G->psi_n, G->lev[0].psi, bytes, hipMemcpyDeviceToDevice, G->stream));
    G->nstep += 1;
    G->t += G->step.dt;
    G->in_step = false;
    return RS_OK;
}

int rs_bdf_step(rs_grid *G, double dt, int order, const rs_solve_opts *o, rs_step_stats *st)
{
    if (!G || !o) return fail(RS_EINVAL, "null argument");
    if (o->struct_size != sizeof(rs_solve_opts)) return fail(RS_EINVAL, "rs_solve_opts.struct_size");
    if (st && st->struct_size != sizeof(rs_step_stats)) return fail(RS_EINVAL, "rs_step_stats.struct_size");
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu_coarse < 1 || o->max_cycles < 0)
        return fail(RS_EINVAL, "bad solve options");
    G->nu_coarse = o->nu_coarse;
    int e = rs_begin_step(G, dt, order);
    if (e) return e;
    double r;
    e = fine_norm(G, &r);
    if (e) return e;
    double r0 = r;
    int cycles = 0, slow = 0, nh = 0;
    double best = r;
    double hist[64];
    hist[nh++] = r;
    bool stagnated = false;
    G->updates = 0.0;
    const bool mixed = G->precision == RS_MIXED;
    if (mixed) {
        e = fine_norm(G, &r, nullptr, true);   // defect vector for the first correction
        if (e) return e;
    }
    // FP64 V-cycles on grids whose finest level is not part of the
    // one-work-group cycle take the stopping test where the cycle forms the
    // fine defect anyway, after the pre-smoothing: a step ends there, with
    // that iterate, once its defect meets the test (one fine defect pass per
    // cycle instead of two).
    const bool test_in_cycle = !mixed && G->nlev > 1 && G->tail_top > 0;
    // The stagnation test compares the norms the cycles measure with each
    // other: the first norm taken inside a cycle (after its pre-smoothing,
    // before any coarse correction) and the norm after an FMG cycle (which
    // replaces the iterate) start the comparison afresh.
    bool fresh = true;
    while (std::isfinite(r) && r > o->tol_abs && cycles < o->max_cycles) {
        if (test_in_cycle && !(o->fmg && cycles == 0)) {
            double rn;
            e = presmooth_norm(G, o->nu1, &rn);
            if (e) return e;
            ++cycles;
            if (nh < 64) hist[nh++] = rn;
            r = rn;
            if (o->stagnation) {
                if (fresh || rn < best) {
                    best = rn;
                    slow = 0;
                } else if (++slow >= 2) {
                    stagnated = true;
                    break;
                }
            }
            fresh = false;
            if (!(std::isfinite(rn) && rn > o->tol_abs) || cycles >= o->max_cycles) break;
            e = coarse_cycle(G, 0, o->nu1, o->nu2);
            if (!e) e = sweep_level(G, 0, o->nu2);
            if (e) return e;
            HIPCALL(hipGetLastError());
            continue;
        }
        const bool after_fmg = o->fmg && cycles == 0;
        if (after_fmg) {
            e = fmg_cycle(G, o->nu1, o->nu2);
            if (e) return e;
        } else if (mixed) {
            mp_correction(G, o->mp_inner_cycles > 0 ? o->mp_inner_cycles : 1, o->nu1, o->nu2);
        } else {
            e = vcycle_level(G, 0, o->nu1, o->nu2);
            if (e) return e;
        }
        HIPCALL(hipGetLastError());
        double rn;
        e = fine_norm(G, &rn, nullptr, mixed);
        if (e) return e;
        ++cycles;
        if (nh < 64) hist[nh++] = rn;
        r = rn;
        if (o->stagnation) {
            if (after_fmg || rn < best) {
                best = rn;
                slow = 0;
            } else if (++slow >= 2) {
                stagnated = true;
                break;
            }
        }
        if (after_fmg) fresh = true;
    }
    int status = RS_OK;
    bool stalled = false;
    if (!std::isfinite(r)) status = RS_ENONFINITE;
    else if (r > o->tol_abs && !stagnated) status = RS_ENOTCONV;
    else if (stagnated && r > o->tol_abs) {
        // two cycles without a new minimum: the rounding floor, unless the
        // residual of the iterate kept (the last one) is above the rounding
        // of the defect's terms (a cycle that diverges or stalls)
        double sc;
        e = defect_scale(G, &sc);
        if (e) return e;
        if (!(r <= kFloorRel * sc)) {
            status = RS_ENOTCONV;
            stalled = true;
        }
    }
    if (st) {
        st->cycles = cycles;
        st->status = status;
        st->res0 = r0;
        st->res = r;
        st->n_hist = nh;
        memcpy(st->res_hist, hist, sizeof(double) * nh);
        st->cell_updates = G->updates;
    }
    if (status != RS_OK) {
        return fail(status, status == RS_ENONFINITE ? "residual is not finite"
                            : stalled ? "the cycle stalled far above the rounding floor (it diverges)"
                                      : "tolerance not reached in max_cycles");
    }
    return rs_end_step(G);
}

int rs_copy_field(const rs_grid *G, int level, int field, double *dst)
{
    if (!G || !dst) return fail(RS_EINVAL, "null argument");
    if (level < 0 || level >= G->nlev) return fail(RS_EINVAL, "level out of range");
    double *p = field_ptr(G, level, field);
    if (!p) return fail(RS_EINVAL, "unknown field %d", field);
    launch_relayout(G->lev[level].geo, p, dst, false, G->stream);
    HIPCALL(hipGetLastError());
    return RS_OK;
}

int rs_set_field(rs_grid *G, int level, int field, const double *src)
{
    if (!G || !src) return fail(RS_EINVAL, "null argument");
    if (level < 0 || level >= G->nlev) return fail(RS_EINVAL, "level out of range");
    double *p = field_ptr(G, level, field);
    if (!p) return fail(RS_EINVAL, "unknown field %d", field);
    launch_relayout(G->lev[level].geo, src, p, true, G->stream);
    HIPCALL(hipGetLastError());
    return RS_OK;
}

int rs_profile_enable(rs_grid *G, int on)
{
    if (!G) return fail(RS_EINVAL, "null grid");
    G->prof_on = on != 0;
    return RS_OK;
}

int rs_profile_read(rs_grid *G, double *sweep_ms, long long *launches, double *cells, int reset)
{
    if (!G) return fail(RS_EINVAL, "null grid");
    HIPCALL(hipStreamSynchronize(G->stream));
    int e = harvest_profile(G);
    if (e) return e;
    if (sweep_ms) *sweep_ms = G->prof_ms;
    if (launches) *launches = G->prof_launches;
    if (cells) *cells = G->prof_cells;
    if (reset) {
        G->prof_ms = 0.0;
        G->prof_launches = 0;
        G->prof_cells = 0.0;
    }
    return RS_OK;
}

int rs_bdf_step_static(const rs_grid_desc *d, const rs_constitutive *c, const double *psi_n,
                       const double *psi_nm1, int nstep, double dt, int order,
                       const rs_solve_opts *o, double *psi_out, rs_step_stats *st, void *stream)
{
    int e = validate_desc(d);
    if (e) return e;
    if (!c || !psi_n || !psi_out || !o) return fail(RS_EINVAL, "null argument");
    if (nstep < 0) return fail(RS_EINVAL, "nstep < 0");
    Layout L;
    plan(d, RS_FP64, &L);
    if (L.total > sizeof(scratch))
        return fail(RS_ENOMEM, "grid needs %zu bytes of workspace; the static scratch holds %zu",
                    L.total, sizeof(scratch));
    int dev = -1;
    HIPCALL(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(RS_EINVAL, "device %d out of range", dev);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_static_mu);
        if (!g_static_ptr[dev]) {
            void *p = nullptr;
            HIPCALL(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            if (!p) return fail(RS_EHIP, "no device address for the static scratch");
            g_static_ptr[dev] = p;
        }
        base = g_static_ptr[dev];
    }
    hipStream_t s = (hipStream_t)stream;
    // the previous call's contents stay in the array: clear this grid's part
    // (the padding around every array must hold zeros) with a kernel
    launch_fill_u64((unsigned long long *)base, (int)(L.total / sizeof(unsigned long long)), 0ull, s);
    HIPCALL(hipGetLastError());
    rs_grid G{};
    e = grid_view(&G, d, RS_FP64, L, (char *)base, s, g_static_bits[dev], &g_static_tail[dev]);
    if (!e) e = rs_set_constitutive(&G, c);
    if (!e) e = rs_set_state(&G, psi_n, psi_nm1, nstep, 0.0);
    if (e) {
        (void)hipStreamSynchronize(s);
        return e;
    }
    const int code = rs_bdf_step(&G, dt, order, o, st);
    if (code != RS_OK && code != RS_ENOTCONV && code != RS_ENONFINITE) {
        (void)hipStreamSynchronize(s);
        return code;
    }
    char msg[sizeof g_err];
    memcpy(msg, g_err, sizeof msg);
    launch_relayout(G.lev[0].geo, code == RS_OK ? G.psi_n : G.lev[0].psi, psi_out, false, s);
    HIPCALL(hipGetLastError());
    HIPCALL(hipStreamSynchronize(s));
    if (code != RS_OK) memcpy(g_err, msg, sizeof msg);
    return code;
}

int rs_num_levels(const rs_grid *G) { return G ? G->nlev : 0; }

int rs_level_shape(const rs_grid *G, int level, int *n_out)
{
    if (!G || !n_out) return fail(RS_EINVAL, "null argument");
    if (level < 0 || level >= G->nlev) return fail(RS_EINVAL, "level out of range");
    for (int a = 0; a < 3; ++a) n_out[a] = G->lev[level].geo.n[a];
    return RS_OK;
}

}  // extern "C"
