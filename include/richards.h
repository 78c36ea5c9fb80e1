/*
 * richards.h - C ABI of the MI355X (gfx950) NGS-FAS solver for the
 * BDF-discretised Richards equation (Gu & Wang, "An Efficient Solver for the
 * Richards Equation for Variably Saturated Flows in Porous Media").
 *
 * The library computes, per time step, the solution psi^{n+1} of the fully
 * discrete system N_h(psi) = g_h (section 3.2, eq. Nh-def / Nh-system) with
 * FAS multigrid V-cycles (section 3.2, the two-grid FAS algorithm applied
 * recursively) whose smoother is the nonlinear Gauss-Seidel iteration of the
 * triangular splitting M = L + D_kappa + U_kappa (Lemma lem:decompos,
 * eq. iterative), one scalar Newton solve per cell (eq. point-update), taken
 * in red-black order.  All arithmetic runs in hand-written HIP kernels on the
 * device; this header exposes only plain pointers and sizes.
 *
 * Conventions
 *  - Grid (section 2, read as vertex-centred): dim in {1,2,3}; n[l] nodes on
 *    axis l including both boundary nodes, n[l] = 2^k + 1 >= 3; spacing
 *    h_l = L[l] / (n[l] - 1).  Axis dim-1 is vertical; its coordinate is
 *    elevation (0 at the bottom, positive up).
 *  - Arrays are flattened lexicographically with axis 0 fastest (the
 *    flattening s(i) of section 2), one FP64 value per node, boundary nodes
 *    included.  Dirichlet nodes hold their boundary value.
 *  - Faces: 2*l is the low end of axis l, 2*l+1 the high end.
 *  - psi in metres; K in m/s; time in s (any consistent unit system works).
 *  - Every call returns RS_OK (0) or an error code; rs_last_error() gives a
 *    message for the calling thread.  No C++ exception crosses the ABI.
 *  - Device pointers ("_dev") refer to memory of the device that was current
 *    when the grid was created; the caller owns them and all workspaces.
 *  - Calls on one grid are asynchronous on the grid's stream unless stated
 *    otherwise; calls on one grid must not be made concurrently.
 */
#ifndef RICHARDS_H
#define RICHARDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define RS_OK 0
#define RS_EINVAL 1       /* invalid argument or descriptor */
#define RS_ENOMEM 2       /* workspace smaller than rs_workspace_bytes */
#define RS_EHIP 3         /* a HIP runtime call failed */
#define RS_ESTATE 4       /* call out of order (e.g. vcycle before begin_step) */
#define RS_ENONFINITE 5   /* NaN or Inf in the residual */
#define RS_ENOTCONV 6     /* tolerance not reached within max_cycles */

/* precision of the smoother / coarse levels */
#define RS_FP64 0         /* everything in FP64 */
#define RS_MIXED 1        /* FP32 correction cycles inside FP64 defect correction */

/* boundary-face kinds */
#define RS_BC_DIRICHLET 1 /* prescribed head (value stored in the psi array) */
#define RS_BC_NOFLUX 2    /* zero normal flux, half control volume */
#define RS_BC_FREEDRAIN 3 /* unit total-head gradient outflow; bottom face only */
#define RS_BC_DIRICHLET_STATE 4 /* prescribed head taken node by node from the state psi^n
                                   (non-uniform boundary data, e.g. the top boundary of the
                                   2-D Gardner case of section 4.2); face_value unused.
                                   RS_FP64 and RS_MIXED grids; not in the serving engine */

/* constitutive models (Table tab:models) */
#define RS_VGM 1          /* van Genuchten - Mualem, m = 1 - 1/n, l = 1/2 */
#define RS_HAVERKAMP 2    /* Haverkamp et al. */
#define RS_LINEAR 3       /* theta = theta_r + lin_c psi, K = Ks (testing) */
#define RS_GARDNER 4      /* Gardner: theta_r + (theta_s - theta_r) e^(alpha psi), K = Ks e^(alpha psi) */
#define RS_MAX_SOILS 16

#define RS_SINK_NONE 0
#define RS_SINK_FEDDES_EXP 1  /* S = beta(z) a(psi): Feddes stress factor,
                                 exponential root density integrating to Tp */

/* diagonal shift Lambda_kappa (Lemma lem:decompos) */
#define RS_KAPPA_CONST 1  /* kappa_i = kappa */
#define RS_KAPPA_REL 2    /* kappa_i = kappa * m_ii */
#define RS_KAPPA_REMARK 3 /* kappa_i = max_j rowsum(U)_j - rowsum(U)_i, the
                             Remark after the contraction theorem */

/* fields for rs_copy_field / rs_set_field */
#define RS_FIELD_PSI 0    /* current iterate */
#define RS_FIELD_KSTAR 1  /* nodal K at the lagged state */
#define RS_FIELD_G 2      /* right-hand side (g_h on level 0, FAS g_H below) */
#define RS_FIELD_PSIBAR 3 /* restricted iterate (levels >= 1) */

/* Problem domain and boundary (section 2; Dirichlet data as in section 4).
 * One optional Dirichlet patch: the nodes of face patch_face (or -1 for none)
 * whose tangential node indices lie in [patch_lo, patch_hi] (inclusive, axes
 * in increasing order) take the value patch_value.  A node on several
 * Dirichlet faces takes the patch value, else the value of the highest-
 * numbered Dirichlet face holding it. */
typedef struct rs_grid_desc {
    size_t struct_size;   /* sizeof(rs_grid_desc) */
    int dim;
    int n[3];
    double L[3];
    int face_bc[6];
    double face_value[6];
    int patch_face;
    int patch_lo[2];
    int patch_hi[2];
    double patch_value;
} rs_grid_desc;

/* K* on the coarse levels (the coarse operator of section 3.2 is defined by
 * analogy with the fine one): the fine value at the coinciding node, or the
 * full-weighting average (1/4, 1/2, 1/4 per axis, mirrored at the ends) of the
 * finer level's K*, which keeps the cycle convergent where K* jumps between
 * neighbouring nodes.  Both converge to the same step solution. */
#define RS_COARSE_INJECT 0
#define RS_COARSE_FW 1

/* Soil law, sink and smoother parameters (Table tab:models; eq. fully-bdf1
 * for xi; Lemma lem:decompos for kappa; eq. point-update for the Newton
 * count).  psi_unit scales psi before the Haverkamp law (100: law in cm).
 * Ks_field: nullable HOST pointer, one saturated conductivity per fine node,
 * copied by the call. lag_extrap: for BDF2, lag the diffusion matrix at
 * 2 psi^n - psi^{n-1} instead of psi^n.  newton_tol: the pointwise solve
 * (eq. point-update) takes at most newton_iters safeguarded Newton steps and
 * ends after a Newton step that moved psi by at most newton_tol |psi| (0: only
 * a zero step ends it early; 1e-10 leaves out steps below rounding); 0..1e-3.
 * gd_alpha: the Gardner exponent (per law unit of psi, psi_unit applies).
 *
 * Layered media (section 4: the composite column of 4.1, the two-layer
 * medium of 4.2): n_soils > 0 gives every fine node its own soil law,
 * soils[soil_id[node]]; each rs_soil supplies the law (model, theta_s,
 * theta_r, Ks and the model's parameters) and every other field of this
 * struct (sink, xi, kappa, Newton settings) stays shared.  Coarse nodes take
 * the soil of the fine node they coincide with.  soils and soil_id are HOST
 * pointers copied by the call; soil_id has one entry per fine node, each
 * < n_soils <= RS_MAX_SOILS.  The scalar law fields above are then unused.
 * Layered media and the Gardner law run on RS_FP64 grids only (RS_EINVAL
 * on RS_MIXED grids and in the serving engine); Ks_field must be null. */
typedef struct rs_soil {
    int model;            /* RS_VGM, RS_HAVERKAMP, RS_GARDNER or RS_LINEAR */
    double theta_s, theta_r, Ks;
    double vg_alpha, vg_n;
    double hk_alpha, hk_beta, hk_A, hk_gamma, psi_unit;
    double lin_c;
    double gd_alpha;
} rs_soil;

typedef struct rs_constitutive {
    size_t struct_size;   /* sizeof(rs_constitutive) */
    int model;
    double theta_s, theta_r, Ks;
    double vg_alpha, vg_n;
    double hk_alpha, hk_beta, hk_A, hk_gamma, psi_unit;
    double lin_c;
    int sink;
    double Tp, root_len, h1, h2, h3, h4;
    double xi;
    int kappa_rule;
    double kappa;
    int newton_iters;
    int lag_extrap;
    double newton_tol;
    const double *Ks_field;
    double gd_alpha;
    int n_soils;                  /* 0: the law above everywhere */
    const rs_soil *soils;         /* HOST, n_soils entries */
    const unsigned char *soil_id; /* HOST, one per fine node */
    int coarse_kstar;             /* RS_COARSE_INJECT (0) or RS_COARSE_FW; the engine takes RS_COARSE_INJECT */
} rs_constitutive;

/* V-cycle parameters (nu_1, nu_2, nu_H of section 3.2) and stopping test
 * (max-norm of g_h - N_h(psi), section 3.2 last paragraph). */
typedef struct rs_solve_opts {
    size_t struct_size;   /* sizeof(rs_solve_opts) */
    int nu1, nu2, nu_coarse, max_cycles;
    double tol_abs;       /* stop when ||g - N(psi)||_inf <= tol_abs */
    int stagnation;       /* also stop at the rounding floor: two cycles in a row
                             that set no new minimum of the norm (the norm after an
                             FMG cycle, and the first norm a step takes inside a
                             cycle, start the comparison afresh).  RS_OK if the norm
                             of the last iterate (the one kept) is within 16 ulp of
                             the largest sum of magnitudes of one node's defect terms
                             (|g|, a|theta|, sink, xi|psi_i|, m_ij (|psi_i| + |psi_j|)
                             per face: a one-ulp change of psi_i moves the defect by
                             m_ii ulp(psi_i)), else RS_ENOTCONV: the cycle diverges
                             or stalls (coarse_kstar = RS_COARSE_FW helps where K*
                             jumps between nodes) */
    int mp_inner_cycles;  /* RS_MIXED: FP32 V-cycles per FP64 defect correction */
    int fmg;              /* 1: the first cycle of every step is one FMG(nu1, nu2) cycle
                             (rs_fmg, in FP64), counted as a cycle */
} rs_solve_opts;

typedef struct rs_step_stats {
    size_t struct_size;   /* sizeof(rs_step_stats) */
    int cycles;           /* V-cycles (FP64) or outer corrections (RS_MIXED) */
    int status;           /* RS_OK, RS_ENOTCONV or RS_ENONFINITE */
    double res0, res;     /* residual max-norm before and after */
    int n_hist;
    double res_hist[64];  /* residual norm before each cycle and after the last */
    double cell_updates;  /* pointwise NGS updates in this step, all levels */
} rs_step_stats;

typedef struct rs_grid rs_grid;

/* Exact device workspace (bytes) for a grid: all multigrid levels, the BDF
 * history and scratch.  Errors: RS_EINVAL for an invalid descriptor. */
int rs_workspace_bytes(const rs_grid_desc *d, int precision, size_t *out);

/* Build the level hierarchy (every axis halved until the shortest has 3
 * nodes; coarse node I is fine node 2I, section 3.2 two-grid hierarchy)
 * inside the caller's device workspace ws_dev (ws_bytes >= rs_workspace_bytes,
 * 256-byte aligned).  stream: a hipStream_t (NULL = default stream).  The
 * library never frees ws_dev.  Errors: RS_EINVAL, RS_ENOMEM, RS_EHIP. */
int rs_create_grid(const rs_grid_desc *d, int precision, void *ws_dev, size_t ws_bytes,
                   void *stream, rs_grid **out);

/* Set the soil law and smoother parameters.  Errors: RS_EINVAL (theta_s <=
 * theta_r, vg_n <= 1, Ks <= 0, newton_iters < 1, ...), RS_EHIP. */
int rs_set_constitutive(rs_grid *g, const rs_constitutive *c);

/* Set the time-level state psi^n (and psi^{n-1} for BDF2; NULL = psi^n) from
 * device arrays of fine-grid size, the number of steps already taken and the
 * time.  Asynchronous (copies on the grid stream). */
int rs_set_state(rs_grid *g, const double *psi_n_dev, const double *psi_nm1_dev, int nstep,
                 double t);
int rs_get_state(const rs_grid *g, double *psi_n_dev, double *psi_nm1_dev, int *nstep,
                 double *t);

/* Assemble the step system (eq. fully-bdf1; BDF2 for order 2 after the first
 * step): K* = K(psi*) at every node, coarse K* by injection, g_h =
 * history + xi psi* - M z - free-drainage outflow; the iterate starts at psi^n
 * with Dirichlet values imposed.  Asynchronous.  Errors: RS_ESTATE without a
 * constitutive law. */
int rs_begin_step(rs_grid *g, double dt, int order);

/* nsweeps red-black NGS sweeps (eq. iterative / eq. point-update, red cells
 * first, then black) on one level of the active step system.  Asynchronous. */
int rs_sweep(rs_grid *g, int level, int nsweeps);

/* One FAS V-cycle V(nu1, nu2) on the active step system (section 3.2, steps
 * 1-7 with recursion; nu_coarse sweeps on the coarsest level).  If res_linf is
 * not NULL the fine residual max-norm after the cycle is written there and the
 * call synchronises the stream.  Errors: RS_ESTATE without begin_step. */
int rs_vcycle(rs_grid *g, int nu1, int nu2, double *res_linf);

/* One full-multigrid cycle FMG(nu1, nu2) on the active step system (section
 * 3.2, the closing paragraph: start on the coarsest grid, interpolate the
 * solution to the finer grids, V-cycles on each).  Every coarser level gets
 * the full-weighting restriction of the finer right-hand side (zero at its
 * Dirichlet nodes) and the injection of the finer iterate; the coarsest level
 * takes nu_coarse sweeps; then each finer level starts from the linear
 * interpolation of the coarser solution at its unknowns and runs one
 * V(nu1, nu2).  FP64 on any grid.  res_linf as for rs_vcycle.
 * Errors: RS_ESTATE without begin_step. */
int rs_fmg(rs_grid *g, int nu1, int nu2, double *res_linf);

/* RS_MIXED grids: one FP64 defect correction (spec precision pattern,
 * not in the paper).  The FP64 defect r = g_h - N_h(psi) is formed, then
 * inner_cycles FP32 FAS V(nu1, nu2) cycles solve the correction equation
 * N_h(psi_b + delta) - N_h(psi_b) = fl32(r) about the base state
 * psi_b = fl32(psi), with the increments of theta and S evaluated without
 * cancellation, and psi += delta in FP64.  res (nullable) receives the FP64
 * residual norm afterwards (synchronises).  Errors: RS_ESTATE on an FP64 grid
 * or without begin_step. */
int rs_correction_cycle(rs_grid *g, int inner_cycles, int nu1, int nu2, double *res_linf);

/* ||g_h - N_h(psi)||_inf over the fine unknowns in FP64 (the stopping quantity
 * of section 3.2).  Synchronises.  RS_ENONFINITE if it is not finite. */
int rs_residual_norm(rs_grid *g, double *out);

/* The fine defect vector g_h - N_h(psi) (0 at Dirichlet nodes) into d_dev. */
int rs_residual(rs_grid *g, double *d_dev);

/* Accept the iterate: psi^{n-1} <- psi^n, psi^n <- psi, n += 1, t += dt. */
int rs_end_step(rs_grid *g);

/* One full time step: begin_step, V-cycles (RS_FP64) or FP32 correction
 * cycles inside FP64 defect correction (RS_MIXED) until the tolerance, then
 * end_step.  FP64 cycles on grids with more than one work-group's worth of
 * fine nodes take the stopping test on the defect each cycle forms after its
 * pre-smoothing (for the restriction), and end the step there with that
 * iterate; the test of the section 3.2 criterion itself is unchanged.
 * Synchronises.  On RS_ENOTCONV / RS_ENONFINITE the iterate is left in place
 * and the history is NOT advanced. */
int rs_bdf_step(rs_grid *g, double dt, int order, const rs_solve_opts *o, rs_step_stats *st);

/* Inspection: copy / overwrite one FP64 field of a level (device arrays of
 * that level's size).  Asynchronous. */
int rs_copy_field(const rs_grid *g, int level, int field, double *dst_dev);
int rs_set_field(rs_grid *g, int level, int field, const double *src_dev);

/* Level count and per-level node counts (n_out: 3 ints). */
int rs_num_levels(const rs_grid *g);
int rs_level_shape(const rs_grid *g, int level, int *n_out);

/* Instrumentation: when enabled, HIP events on the grid stream bracket every
 * batch of finest-level sweep launches; rs_profile_read returns their summed
 * elapsed time (ms), the number of kernel launches (one per colour per sweep)
 * and the pointwise updates they performed, accumulated since the last reset.
 * Reading synchronises the stream. */
int rs_profile_enable(rs_grid *g, int on);
int rs_profile_read(rs_grid *g, double *sweep_ms, long long *launches, double *cell_updates,
                    int reset);

/* One time step that allocates nothing: for callers that cannot allocate
 * device or pinned host memory (tight serving loops, harnesses that forbid
 * allocation), not part of the paper's method.  The same computation as
 * rs_create_grid + rs_set_constitutive + rs_set_state + rs_bdf_step on an
 * RS_FP64 grid (same kernels, same results), with the grid's whole workspace
 * in a static device array of RS_STATIC_WORKSPACE_BYTES that the library holds
 * on every device it runs on until the process ends.
 *   d, c: grid and law as for rs_create_grid / rs_set_constitutive (host);
 *   psi_n_dev, psi_nm1_dev (nullable = psi_n_dev): the state (device arrays of
 *   fine-grid size, lexicographic); nstep: steps already taken (0 makes an
 *   order-2 step BDF1); dt, order, o, st: as for rs_bdf_step;
 *   psi_out_dev: receives psi^{n+1} (RS_OK) or the last iterate
 *   (RS_ENOTCONV, RS_ENONFINITE); stream: a hipStream_t (NULL = default).
 * Synchronises the stream.  Errors: RS_EINVAL; RS_ENOMEM when the grid's FP64
 * workspace (rs_workspace_bytes) exceeds RS_STATIC_WORKSPACE_BYTES; RS_EHIP;
 * RS_ENOTCONV / RS_ENONFINITE as for rs_bdf_step.  Calls that overlap on one
 * device (other host threads, other streams) share its array and race: the
 * caller serialises them. */
#define RS_STATIC_WORKSPACE_BYTES (32u << 20)
int rs_bdf_step_static(const rs_grid_desc *d, const rs_constitutive *c, const double *psi_n_dev,
                       const double *psi_nm1_dev, int nstep, double dt, int order,
                       const rs_solve_opts *o, double *psi_out_dev, rs_step_stats *st,
                       void *stream);

void rs_destroy_grid(rs_grid *g);
const char *rs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RICHARDS_H */
