/*
 * richards_serve.h - continuous-batching engine for many independent
 * Richards step-solves on one device.
 *
 * Each request is one grid (rs_grid_desc), one soil law (rs_constitutive), an
 * initial state and a number of BDF steps.  Every step is solved like
 * rs_bdf_step on an RS_MIXED grid: FP32 FAS V-cycles (section 3.2, red-black
 * NGS of eq. point-update) on the correction equation
 * N(psi + delta) - N(psi) = r inside an FP64 defect-correction loop whose
 * residual (eq. Nh-def), stopping test and BDF history stay in FP64.
 *
 * The engine keeps every admitted request's state in one caller-owned device
 * arena.  A "round" advances every admitted request by one outer correction:
 * a fixed sequence of batched kernels, each covering all requests at one depth
 * of their level hierarchies (coarse levels of up to tail_nodes nodes run as
 * one work-group per request), replayed as a captured HIP graph.  Convergence
 * tests, step transitions (history update, next step's set-up) and failures
 * are decided on the device per request, so a request that arrives while
 * others are running joins at the next round, and one request's arithmetic
 * never depends on which others share the device: results are bit-identical
 * alone and in any mix.
 *
 * Scope: models RS_VGM, RS_HAVERKAMP, RS_LINEAR; kappa rules RS_KAPPA_CONST and
 * RS_KAPPA_REL; coarse K* by injection (RS_COARSE_INJECT); no sink term and
 * no per-node Ks field (other requests are rejected with RS_EINVAL; use the
 * single-grid API for them).
 *
 * Threading: all calls on one engine must come from one thread at a time.
 * Device work is queued on the engine's stream; rs_engine_tick synchronises it.
 */
#ifndef RICHARDS_SERVE_H
#define RICHARDS_SERVE_H

#include "richards.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RS_EBUSY 7        /* no free slot or arena memory right now; retry after a tick */

/* request states reported in rs_request_stats.state */
#define RS_REQ_RUNNING 1
#define RS_REQ_FINISHED 3
#define RS_REQ_FAILED 4

typedef struct rs_engine rs_engine;

typedef struct rs_engine_opts {
    size_t struct_size;   /* sizeof(rs_engine_opts) */
    int max_slots;        /* requests resident at once, 1..4096 */
    int max_wide_levels;  /* levels above tail_nodes per request, 0..8 (graph depth) */
    int tail_nodes;       /* levels of at most this many nodes run in one work-group, >= 27 */
    int nu1, nu2, nu_coarse;
    int max_corrections;  /* per step; a step needing more fails with RS_ENOTCONV */
    double tol_abs;       /* step done when ||g - N(psi)||_inf <= max(tol_abs, tol_rel * r0) */
    double tol_rel;       /*   with r0 the step's initial defect norm */
    int stagnation;       /* also done at the rounding floor: two corrections in a row
                             that set no new minimum of the norm, with the norm of the
                             iterate kept (the last) within 16 ulp of the largest
                             per-node sum of the defect's term magnitudes (|g|,
                             a|theta|, xi|psi_i|, m_ij (|psi_i| + |psi_j|)); a stall
                             above that fails the request with RS_ENOTCONV */
    int rounds_per_tick;  /* correction rounds queued per rs_engine_tick, >= 1 */
    int use_graph;        /* 1: replay a captured HIP graph per round; 0: plain launches */
} rs_engine_opts;

typedef struct rs_request_stats {
    size_t struct_size;   /* sizeof(rs_request_stats) */
    int state;            /* RS_REQ_RUNNING / RS_REQ_FINISHED / RS_REQ_FAILED */
    int status;           /* RS_OK, RS_ENOTCONV or RS_ENONFINITE */
    int steps;            /* steps completed */
    int corrections;      /* outer corrections over all steps */
    int max_step_corrections;
    double res;           /* last FP64 defect norm of the last step */
} rs_request_stats;

/* Fill *o with the defaults: 1024 slots, 4 wide levels, tail_nodes 8192,
 * V(2,2) with 32 coarsest sweeps, 100 corrections per step, tol 0 with the
 * stagnation stop, 4 rounds per tick, graph replay on. */
void rs_engine_default_opts(rs_engine_opts *o);

/* Device bytes at the start of the arena that hold the engine's control
 * tables (slot records, level records, work lists) for these options. */
int rs_engine_control_bytes(const rs_engine_opts *o, size_t *out);

/* Arena bytes one request of grid d occupies while resident: fine-level FP64
 * psi, psi^n, psi^{n-1}, K*, g and six FP32 arrays per level, each 256-byte
 * aligned with 256 zeroed bytes before and after it.  Admission compares this
 * against the arena's free space. */
int rs_engine_request_bytes(const rs_engine_opts *o, const rs_grid_desc *d, size_t *out);

/* Create an engine over the caller's device arena (arena_dev, arena_bytes,
 * 256-byte aligned, at least rs_engine_control_bytes plus one request).  The
 * caller keeps the arena alive until rs_engine_destroy.  stream must be a
 * non-null stream (graph capture needs one).  Errors: RS_EINVAL (options,
 * alignment, null stream), RS_ENOMEM (arena too small), RS_EHIP. */
int rs_engine_create(const rs_engine_opts *o, void *arena_dev, size_t arena_bytes,
                     void *stream, rs_engine **out);

/* Admit one request: grid d, law c, initial state psi0_dev (device, n nodes,
 * Dirichlet nodes are overwritten by their boundary values), nsteps steps of
 * dt with BDF order 1 or 2 (the first step of BDF2 is BDF1).  psi0_dev is
 * copied on the engine stream: keep it alive until the next rs_engine_tick.
 * On RS_OK *ticket identifies the request.  RS_EBUSY: no free slot or arena
 * space now (nothing was changed).  RS_EINVAL: invalid or unsupported request,
 * or one that can never fit (too many wide levels, larger than the arena). */
int rs_engine_submit(rs_engine *e, const rs_grid_desc *d, const rs_constitutive *c,
                     const double *psi0_dev, double dt, int order, int nsteps, int *ticket);

/* Queue rounds_per_tick correction rounds for every resident request, wait for
 * them, and report requests that finished or failed since the last tick:
 * up to max_done tickets into done (the rest on later ticks), their count in
 * *n_done, and the number of requests still running in *n_active.
 * Synchronises the engine stream. */
int rs_engine_tick(rs_engine *e, int *done, int max_done, int *n_done, int *n_active);

/* Copy the final state of a finished or failed request (its last iterate) to
 * psi_dev (device, nullable) on the engine stream, fill *st (nullable), and
 * release the request's slot and arena space.  RS_ESTATE if the request is
 * still running, RS_EINVAL for an unknown ticket. */
int rs_engine_fetch(rs_engine *e, int ticket, double *psi_dev, rs_request_stats *st);

/* Free arena bytes and free slots right now. */
int rs_engine_capacity(const rs_engine *e, size_t *free_bytes, int *free_slots);

/* Release the engine's host resources (not the arena).  Waits for its stream. */
void rs_engine_destroy(rs_engine *e);

#ifdef __cplusplus
}
#endif

#endif /* RICHARDS_SERVE_H */
