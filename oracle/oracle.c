/*
 * Plain FP64 CPU oracle for the NGS-FAS solver of the BDF-discretised
 * Richards equation (Gu & Wang).  TEST INFRASTRUCTURE ONLY: this library is
 * what the HIP path is checked against.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it; the product never
 * does.  It shares no source, header, table or helper with the HIP path.
 *
 * Everything is written as the paper states it, in the paper's order, with no
 * blocking or fusion:
 *   - constitutive laws: Table "tab:models" (Haverkamp, van Genuchten-Mualem
 *     with l = 1/2, Gardner), psi >= 0 treated as saturated; optionally a law
 *     per node from a table of soils (the layered and two-layer cases of
 *     section 4);
 *   - space: the conservative second-order finite-difference operator of
 *     eq. (discrete-strong) with arithmetic face averages of K, on a
 *     vertex-centred grid (2^k+1 nodes per axis);
 *   - time: BDF1 of eq. (fully-bdf1) with the stabilisation xi and the
 *     diffusion matrix lagged; BDF2 with the lagged state 2 psi^n - psi^{n-1};
 *   - smoother: the triangular splitting M = L + D_kappa + U_kappa of the
 *     Lemma, giving the pointwise equation eq. (point-update) solved by a fixed
 *     number of safeguarded Newton steps; lexicographic (first index fastest)
 *     or red-black ordering;
 *   - multigrid: the two-grid FAS algorithm of section 3.2 applied
 *     recursively (V-cycle), full-weighting restriction and linear
 *     interpolation, operators rediscretised on every level.
 * Readings where the paper is silent (boundary kinds other than Dirichlet,
 * BDF2, the kappa rules, the local-solve safeguard, the coarsest solve) are
 * documented at the functions that implement them.
 *
 * Parallelism: OpenMP over the cells of one colour in red-black sweeps and
 * over cells in pointwise passes (setup, residual); every cell is computed
 * independently, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_BC_DIRICHLET 1
#define ORC_BC_NOFLUX 2
#define ORC_BC_FREEDRAIN 3
#define ORC_BC_DIRICHLET_STATE 4

#define ORC_MODEL_VGM 1
#define ORC_MODEL_HAVERKAMP 2
#define ORC_MODEL_LINEAR 3
#define ORC_MODEL_GARDNER 4

#define ORC_MAXSOIL 16

#define ORC_SINK_NONE 0
#define ORC_SINK_FEDDES_EXP 1

#define ORC_KAPPA_CONST 1
#define ORC_KAPPA_REL 2
#define ORC_KAPPA_REMARK 3

/* Coarse-level K* (the paper defines the coarse operator only by analogy with
 * the fine one): the fine value at the coinciding node, or the full-weighting
 * average of the fine K* around it. */
#define ORC_COARSE_INJECT 0
#define ORC_COARSE_FW 1

#define ORC_ORDER_LEX 0
#define ORC_ORDER_RB 1

#define ORC_FIELD_PSI 0
#define ORC_FIELD_KSTAR 1
#define ORC_FIELD_G 2
#define ORC_FIELD_PSIBAR 3
#define ORC_FIELD_PSI_N 4
#define ORC_FIELD_PSI_NM1 5

#define ORC_MAXLEV 16

typedef struct {
    int dim;
    int n[3];
    double L[3];
    int face_bc[6];
    double face_value[6];
    int patch_face;
    int patch_lo[2];
    int patch_hi[2];
    double patch_value;
} orc_grid;

typedef struct {
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
    double newton_tol;  /* stop once a Newton step moves x by <= newton_tol |x| (0: never early) */
    double gd_alpha;    /* Gardner exponent (per law unit of psi) */
    int coarse_k;       /* ORC_COARSE_INJECT or ORC_COARSE_FW: coarse-level K* */
} orc_params;

typedef struct {
    int n[3];          /* nodes per axis (1 for unused axes) */
    int N;             /* total nodes */
    double h[3];
    int patch_lo[2], patch_hi[2];
    double *psi, *Kstar, *g, *psibar, *d;
    double lambdaU;    /* max row sum of U on this level (kappa rule REMARK) */
    unsigned char *sid; /* soil of each node (NULL: one law everywhere) */
} orc_level;

typedef struct {
    orc_grid grid;
    orc_params p;
    int ordering;
    int nu_coarse;
    int nlev;
    orc_level lev[ORC_MAXLEV];
    double *Ks_field;  /* per fine node, or NULL */
    double *psi_n, *psi_nm1;
    int nstep;
    double dt, a;      /* current step size and BDF leading coefficient */
    int order_eff;
    double beta_norm;  /* normalising integral of the root density */
    int nsoil;         /* soils of the per-node table (0: the law in p everywhere) */
    orc_params soil[ORC_MAXSOIL];
} orc_solver;

/* ------------------------------------------------------------------------ */
/* Constitutive laws (Table tab:models).                                     */
/* ------------------------------------------------------------------------ */

/* Water content theta(psi).  Haverkamp: theta_r + alpha (theta_s - theta_r) /
 * (alpha + |psi|^beta); vGM: theta_r + (theta_s - theta_r) (1 + (alpha |psi|)^n)^-m,
 * m = 1 - 1/n; Gardner: theta_r + (theta_s - theta_r) e^(alpha psi).  For
 * psi >= 0 the soil is saturated, theta = theta_s. */
double orc_theta(const orc_params *p, double psi)
{
    if (p->model == ORC_MODEL_LINEAR)
        return p->theta_r + p->lin_c * psi;
    if (psi >= 0.0)
        return p->theta_s;
    if (p->model == ORC_MODEL_GARDNER)
        return p->theta_r + (p->theta_s - p->theta_r) * exp(p->gd_alpha * p->psi_unit * psi);
    if (p->model == ORC_MODEL_HAVERKAMP) {
        double hu = fabs(p->psi_unit * psi);
        return p->theta_r + p->hk_alpha * (p->theta_s - p->theta_r) /
                                (p->hk_alpha + pow(hu, p->hk_beta));
    }
    {
        double m = 1.0 - 1.0 / p->vg_n;
        double Se = pow(1.0 + pow(p->vg_alpha * fabs(psi), p->vg_n), -m);
        return p->theta_r + (p->theta_s - p->theta_r) * Se;
    }
}

/* d theta / d psi (the specific moisture capacity of assumption A1). */
double orc_dtheta(const orc_params *p, double psi)
{
    if (p->model == ORC_MODEL_LINEAR)
        return p->lin_c;
    if (psi >= 0.0)
        return 0.0;
    if (p->model == ORC_MODEL_GARDNER) {
        double au = p->gd_alpha * p->psi_unit;
        return (p->theta_s - p->theta_r) * au * exp(au * psi);
    }
    if (p->model == ORC_MODEL_HAVERKAMP) {
        /* d/dpsi of alpha dT / (alpha + (u|psi|)^beta), u = psi_unit */
        double hu = fabs(p->psi_unit * psi);
        double q = pow(hu, p->hk_beta);
        double den = p->hk_alpha + q;
        return p->psi_unit * p->hk_alpha * (p->theta_s - p->theta_r) * p->hk_beta *
               pow(hu, p->hk_beta - 1.0) / (den * den);
    }
    {
        /* d/dpsi of (1 + (alpha|psi|)^n)^-m for psi < 0:
         * m n alpha (alpha|psi|)^(n-1) (1 + (alpha|psi|)^n)^(-m-1) */
        double n = p->vg_n, m = 1.0 - 1.0 / n;
        double ap = p->vg_alpha * fabs(psi);
        return (p->theta_s - p->theta_r) * m * n * p->vg_alpha * pow(ap, n - 1.0) *
               pow(1.0 + pow(ap, n), -m - 1.0);
    }
}

/* Relative conductivity K(psi)/Ks.  Haverkamp: A / (A + |psi|^gamma);
 * vGM (Mualem, l = 1/2): Se^(1/2) [1 - (1 - Se^(1/m))^m]^2; Gardner: e^(alpha psi). */
double orc_Krel(const orc_params *p, double psi)
{
    if (p->model == ORC_MODEL_LINEAR)
        return 1.0;
    if (psi >= 0.0)
        return 1.0;
    if (p->model == ORC_MODEL_GARDNER)
        return exp(p->gd_alpha * p->psi_unit * psi);
    if (p->model == ORC_MODEL_HAVERKAMP) {
        double hu = fabs(p->psi_unit * psi);
        return p->hk_A / (p->hk_A + pow(hu, p->hk_gamma));
    }
    {
        double m = 1.0 - 1.0 / p->vg_n;
        double Se = pow(1.0 + pow(p->vg_alpha * fabs(psi), p->vg_n), -m);
        double t = 1.0 - pow(1.0 - pow(Se, 1.0 / m), m);
        return sqrt(Se) * t * t;
    }
}

/* Feddes-type water-stress factor a(psi), piecewise linear with half-open
 * segments: 0 below h4, rising on [h4,h3), 1 on [h3,h2), falling on [h2,h1),
 * 0 from h1 up.  The derivative is the slope of the segment holding psi. */
double orc_feddes(const orc_params *p, double psi)
{
    if (psi < p->h4) return 0.0;
    if (psi < p->h3) return (psi - p->h4) / (p->h3 - p->h4);
    if (psi < p->h2) return 1.0;
    if (psi < p->h1) return (p->h1 - psi) / (p->h1 - p->h2);
    return 0.0;
}

double orc_dfeddes(const orc_params *p, double psi)
{
    if (psi < p->h4) return 0.0;
    if (psi < p->h3) return 1.0 / (p->h3 - p->h4);
    if (psi < p->h2) return 0.0;
    if (psi < p->h1) return -1.0 / (p->h1 - p->h2);
    return 0.0;
}

/* Vector evaluation helper for tests. */
void orc_eval_law(const orc_params *p, int n, const double *psi, double *th,
                  double *dth, double *Kr)
{
    for (int i = 0; i < n; i++) {
        if (th) th[i] = orc_theta(p, psi[i]);
        if (dth) dth[i] = orc_dtheta(p, psi[i]);
        if (Kr) Kr[i] = orc_Krel(p, psi[i]);
    }
}

void orc_eval_feddes(const orc_params *p, int n, const double *psi, double *a, double *da)
{
    for (int i = 0; i < n; i++) {
        if (a) a[i] = orc_feddes(p, psi[i]);
        if (da) da[i] = orc_dfeddes(p, psi[i]);
    }
}

/* ------------------------------------------------------------------------ */
/* Grid, node kinds, level hierarchy.                                        */
/* ------------------------------------------------------------------------ */

static void coords(const orc_level *lv, int idx, int ii[3])
{
    ii[0] = idx % lv->n[0];
    ii[1] = (idx / lv->n[0]) % lv->n[1];
    ii[2] = idx / (lv->n[0] * lv->n[1]);
}

static int index_of(const orc_level *lv, const int ii[3])
{
    return ii[0] + lv->n[0] * (ii[1] + lv->n[1] * ii[2]);
}

/* Is node ii on the optional Dirichlet patch (a face sub-rectangle)? */
static int in_patch(const orc_solver *S, const orc_level *lv, const int ii[3])
{
    int f = S->grid.patch_face;
    if (f < 0) return 0;
    int ax = f / 2;
    int at = (f % 2 == 0) ? 0 : lv->n[ax] - 1;
    if (ii[ax] != at) return 0;
    int t = 0;
    for (int l = 0; l < S->grid.dim; l++) {
        if (l == ax) continue;
        if (ii[l] < lv->patch_lo[t] || ii[l] > lv->patch_hi[t]) return 0;
        t++;
    }
    return 1;
}

static int dirichlet_face(int bc)
{
    return bc == ORC_BC_DIRICHLET || bc == ORC_BC_DIRICHLET_STATE;
}

/* A node is Dirichlet if it lies on a Dirichlet face or on the patch.  Its
 * value: the patch value on the patch, otherwise that of the last Dirichlet
 * face (in face order) holding it.  A face of kind DIRICHLET_STATE holds
 * non-uniform boundary data (the 2-D top boundary of section 4.2): its value
 * is the node's entry of the state psi^n, reported through *from_state. */
static int is_dirichlet_src(const orc_solver *S, const orc_level *lv, const int ii[3],
                            double *val, int *from_state)
{
    int dir = 0, st = 0;
    double v = 0.0;
    for (int l = 0; l < S->grid.dim; l++) {
        if (ii[l] == 0 && dirichlet_face(S->grid.face_bc[2 * l])) {
            dir = 1;
            v = S->grid.face_value[2 * l];
            st = S->grid.face_bc[2 * l] == ORC_BC_DIRICHLET_STATE;
        }
        if (ii[l] == lv->n[l] - 1 && dirichlet_face(S->grid.face_bc[2 * l + 1])) {
            dir = 1;
            v = S->grid.face_value[2 * l + 1];
            st = S->grid.face_bc[2 * l + 1] == ORC_BC_DIRICHLET_STATE;
        }
    }
    if (in_patch(S, lv, ii)) {
        dir = 1;
        v = S->grid.patch_value;
        st = 0;
    }
    if (val) *val = v;
    if (from_state) *from_state = st;
    return dir;
}

static int is_dirichlet(const orc_solver *S, const orc_level *lv, const int ii[3], double *val)
{
    return is_dirichlet_src(S, lv, ii, val, NULL);
}

/* Control-volume fraction along axis l for an unknown node: a node on the
 * boundary of axis l owns half a cell there (reading for no-flux and
 * free-drainage faces). */
static double wfrac(const orc_level *lv, const int ii[3], int l)
{
    return (ii[l] == 0 || ii[l] == lv->n[l] - 1) ? 0.5 : 1.0;
}

static double elev(const orc_solver *S, const orc_level *lv, const int ii[3])
{
    int v = S->grid.dim - 1;
    return ii[v] * lv->h[v];
}

/* Root density beta(z) = Tp exp(-(Lz - z)/root_len) / Z with Z the
 * trapezoidal integral over the fine column, so that beta integrates to Tp. */
static double root_beta(const orc_solver *S, double z)
{
    if (S->p.sink != ORC_SINK_FEDDES_EXP) return 0.0;
    int v = S->grid.dim - 1;
    return S->p.Tp * exp(-(S->grid.L[v] - z) / S->p.root_len) / S->beta_norm;
}

/* The soil law of node i of a level: its entry of the soil table (layered
 * media, section 4), else the one law of the problem. */
static const orc_params *law_at(const orc_solver *S, const orc_level *lv, int i)
{
    return lv->sid ? &S->soil[lv->sid[i]] : &S->p;
}

/* ------------------------------------------------------------------------ */
/* Operator M(psi*) (eq. discrete-strong and the matrix M of section 2).      */
/* ------------------------------------------------------------------------ */

/* Face coefficient m_ij between unknown node i and its neighbour j across a
 * face normal to axis l: the arithmetic face average of K* divided by w h^2. */
static double mcoef(const orc_level *lv, int i, int j, const int ii[3], int l)
{
    double k = 0.5 * (lv->Kstar[i] + lv->Kstar[j]);
    double w = wfrac(lv, ii, l);
    return k / (w * lv->h[l] * lv->h[l]);
}

/* Iterate over the existing neighbours of node idx: up to 2*dim of them. */
typedef struct { int j; int axis; int side; } orc_nb;

static int neighbours(const orc_solver *S, const orc_level *lv, const int ii[3], orc_nb nb[6])
{
    int k = 0;
    for (int l = 0; l < S->grid.dim; l++) {
        int jj[3] = {ii[0], ii[1], ii[2]};
        if (ii[l] > 0) {
            jj[l] = ii[l] - 1;
            nb[k].j = index_of(lv, jj); nb[k].axis = l; nb[k].side = -1; k++;
        }
        if (ii[l] < lv->n[l] - 1) {
            jj[l] = ii[l] + 1;
            nb[k].j = index_of(lv, jj); nb[k].axis = l; nb[k].side = +1; k++;
        }
    }
    return k;
}

/* (M z)_i: gravity, sum over the vertical faces of m_ij (z_i - z_j). */
static double Mz(const orc_solver *S, const orc_level *lv, int i, const int ii[3])
{
    orc_nb nb[6];
    int k = neighbours(S, lv, ii, nb);
    int v = S->grid.dim - 1;
    double s = 0.0;
    for (int q = 0; q < k; q++) {
        if (nb[q].axis != v) continue;
        double dz = -nb[q].side * lv->h[v];     /* z_i - z_j */
        s += mcoef(lv, i, nb[q].j, ii, v) * dz;
    }
    return s;
}

/* (M psi)_i over all neighbours (Dirichlet neighbours included through the
 * values stored in the array). */
static double Mpsi(const orc_solver *S, const orc_level *lv, const double *psi, int i, const int ii[3])
{
    orc_nb nb[6];
    int k = neighbours(S, lv, ii, nb);
    double s = 0.0;
    for (int q = 0; q < k; q++)
        s += mcoef(lv, i, nb[q].j, ii, nb[q].axis) * (psi[i] - psi[nb[q].j]);
    return s;
}

/* The nonlinear operator N(psi)_i = a theta(psi_i) + S(psi_i) + xi psi_i + (M psi)_i
 * (eq. Nh-def, with a = 1/tau for BDF1 and 3/(2 tau) for BDF2). */
static double Nop(const orc_solver *S, const orc_level *lv, const double *psi, int i, const int ii[3])
{
    double x = psi[i];
    const orc_params *law = law_at(S, lv, i);
    double s = S->a * orc_theta(law, x);
    if (S->p.sink == ORC_SINK_FEDDES_EXP)
        s += root_beta(S, elev(S, lv, ii)) * orc_feddes(&S->p, x);
    s += S->p.xi * x + Mpsi(S, lv, psi, i, ii);
    return s;
}

/* Apply N on level l to an arbitrary psi; Dirichlet entries are set to 0. */
void orc_apply_N(orc_solver *S, int l, const double *psi, double *out)
{
    orc_level *lv = &S->lev[l];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < lv->N; i++) {
        int ii[3];
        coords(lv, i, ii);
        if (is_dirichlet(S, lv, ii, NULL)) { out[i] = 0.0; continue; }
        out[i] = Nop(S, lv, psi, i, ii);
    }
}

/* ------------------------------------------------------------------------ */
/* Splitting and the pointwise update (Lemma lem:decompos, eq. point-update). */
/* ------------------------------------------------------------------------ */

/* Does neighbour j come after node i in the sweep ordering?  Lexicographic:
 * larger flattened index.  Red-black: colour parity of the global index sum;
 * all red nodes precede all black ones. */
static int later(const orc_solver *S, const orc_level *lv, int i, int j)
{
    if (S->ordering == ORC_ORDER_LEX) return j > i;
    int a[3], b[3];
    coords(lv, i, a);
    coords(lv, j, b);
    int ci = (a[0] + a[1] + a[2]) & 1, cj = (b[0] + b[1] + b[2]) & 1;
    if (ci != cj) return cj > ci;   /* red (0) before black (1) */
    return j > i;
}

/* Row sum of the strictly upper part U restricted to unknown columns. */
static double rowsum_U(const orc_solver *S, const orc_level *lv, int i, const int ii[3])
{
    orc_nb nb[6];
    int k = neighbours(S, lv, ii, nb);
    double s = 0.0;
    for (int q = 0; q < k; q++) {
        int jj[3];
        coords(lv, nb[q].j, jj);
        if (is_dirichlet(S, lv, jj, NULL)) continue;
        if (later(S, lv, i, nb[q].j)) s += mcoef(lv, i, nb[q].j, ii, nb[q].axis);
    }
    return s;
}

static double mdiag(const orc_solver *S, const orc_level *lv, int i, const int ii[3])
{
    orc_nb nb[6];
    int k = neighbours(S, lv, ii, nb);
    double s = 0.0;
    for (int q = 0; q < k; q++) s += mcoef(lv, i, nb[q].j, ii, nb[q].axis);
    return s;
}

/* Diagonal shift kappa_i (reading; the paper leaves it to the user):
 * CONST  kappa_i = kappa;
 * REL    kappa_i = kappa * m_ii;
 * REMARK kappa_i = lambda_bar(U) - (row sum of U)_i, the first choice of the
 *        Remark after the contraction theorem (equal row sums of U_kappa). */
static double kappa_i(const orc_solver *S, const orc_level *lv, int i, const int ii[3])
{
    switch (S->p.kappa_rule) {
    case ORC_KAPPA_CONST: return S->p.kappa;
    case ORC_KAPPA_REL: return S->p.kappa * mdiag(S, lv, i, ii);
    default: return lv->lambdaU - rowsum_U(S, lv, i, ii);
    }
}

static void compute_lambdaU(orc_solver *S, orc_level *lv)
{
    double mx = 0.0;
    for (int i = 0; i < lv->N; i++) {
        int ii[3];
        coords(lv, i, ii);
        if (is_dirichlet(S, lv, ii, NULL)) continue;
        double r = rowsum_U(S, lv, i, ii);
        if (r > mx) mx = r;
    }
    lv->lambdaU = mx;
}

/* Scalar solve of a theta(x) + beta a_F(x) + c x = f (eq. point-update with
 * the BDF coefficient a, the sink S = beta * a_F and c = xi + kappa_i + m_ii).
 * The paper leaves the number of (damped) Newton steps open, backtracking
 * optional; reading: at most `iters` Newton steps from x0, each kept
 * inside a bracket [lo, hi] that holds the root (initially
 * [(f - a theta_s - beta)/c, (f - a theta_r)/c], widened by 1e-12 of the sum
 * of the ends' magnitudes so that a root on an end -- a saturated cell, where
 * F is linear and its root is the lower end -- lies strictly inside;
 * tightened by the sign of F at every iterate); a step that does not land strictly inside the bracket,
 * or a non-positive F', is replaced by bisection, except a step that leaves
 * the iterate unchanged (below rounding resolution), which is kept so that a
 * converged cell stays put.  Landing on a bracket end is rejected because a
 * previous iterate sits there, which would allow a two-cycle.  The iteration
 * ends early after a Newton step (not a bisection) that moved x by at most
 * newton_tol |x_new|: near the root Newton converges quadratically, so the
 * steps left out would have moved x by about (F''/2F') times that step
 * squared, below rounding for newton_tol = 1e-10.  A step of zero always ends
 * it (a fixed iterate stays fixed).  *evals (nullable) receives the number of
 * evaluations of F taken. */
double orc_local_solve(const orc_params *p, double a, double beta, double c, double f,
                       double x0, int iters, int *evals)
{
    double lo, hi;
    if (p->model == ORC_MODEL_LINEAR) {
        lo = -HUGE_VAL;
        hi = HUGE_VAL;
    } else {
        lo = (f - a * p->theta_s - beta) / c;
        hi = (f - a * p->theta_r) / c;
        double pad = 1e-12 * (fabs(lo) + fabs(hi));
        lo -= pad;
        hi += pad;
    }
    double x = x0;
    int k = 0;
    while (k < iters) {
        k++;
        double F = a * orc_theta(p, x) + c * x - f;
        double dF = a * orc_dtheta(p, x) + c;
        if (p->sink == ORC_SINK_FEDDES_EXP) {
            F += beta * orc_feddes(p, x);
            dF += beta * orc_dfeddes(p, x);
        }
        if (F > 0.0) {
            if (x < hi) hi = x;
        } else if (F < 0.0) {
            if (x > lo) lo = x;
        } else {
            lo = x;
            hi = x;
        }
        double xn = x - F / dF;
        int bisect = !(dF > 0.0) || (xn != x && !(xn > lo && xn < hi));
        if (bisect) xn = 0.5 * (lo + hi);
        int small = !bisect && fabs(xn - x) <= p->newton_tol * fabs(xn);
        x = xn;
        if (small) break;
    }
    if (evals) *evals = k;
    return x;
}

/* Update node i in place from the current values of its neighbours:
 * f_i = g_i + sum_j m_ij psi_j + kappa_i psi_i,  c_i = xi + kappa_i + m_ii. */
static void point_update(orc_solver *S, orc_level *lv, int i, const int ii[3])
{
    orc_nb nb[6];
    int k = neighbours(S, lv, ii, nb);
    double mii = 0.0, f = lv->g[i];
    for (int q = 0; q < k; q++) {
        double m = mcoef(lv, i, nb[q].j, ii, nb[q].axis);
        mii += m;
        f += m * lv->psi[nb[q].j];
    }
    double kap = kappa_i(S, lv, i, ii);
    f += kap * lv->psi[i];
    double c = S->p.xi + kap + mii;
    double beta = root_beta(S, elev(S, lv, ii));
    lv->psi[i] = orc_local_solve(law_at(S, lv, i), S->a, beta, c, f, lv->psi[i],
                                 S->p.newton_iters, NULL);
}

/* One NGS sweep on level l in the solver's ordering. */
void orc_sweep(orc_solver *S, int l, int nsweeps)
{
    orc_level *lv = &S->lev[l];
    for (int s = 0; s < nsweeps; s++) {
        if (S->ordering == ORC_ORDER_LEX) {
            for (int i = 0; i < lv->N; i++) {
                int ii[3];
                coords(lv, i, ii);
                if (is_dirichlet(S, lv, ii, NULL)) continue;
                point_update(S, lv, i, ii);
            }
        } else {
            for (int colour = 0; colour < 2; colour++) {
#pragma omp parallel for schedule(static)
                for (int i = 0; i < lv->N; i++) {
                    int ii[3];
                    coords(lv, i, ii);
                    if (((ii[0] + ii[1] + ii[2]) & 1) != colour) continue;
                    if (is_dirichlet(S, lv, ii, NULL)) continue;
                    point_update(S, lv, i, ii);
                }
            }
        }
    }
}

/* Update only the listed nodes of one colour (red-black ordering) from the
 * current array contents, writing the results to out (array not modified).
 * Used to check single outputs of large sweeps one by one. */
void orc_update_points(orc_solver *S, int l, int npts, const int *idx, double *out)
{
    orc_level *lv = &S->lev[l];
#pragma omp parallel for schedule(static)
    for (int q = 0; q < npts; q++) {
        int i = idx[q], ii[3];
        coords(lv, i, ii);
        if (is_dirichlet(S, lv, ii, NULL)) { out[q] = lv->psi[i]; continue; }
        orc_nb nb[6];
        int k = neighbours(S, lv, ii, nb);
        double mii = 0.0, f = lv->g[i];
        for (int t = 0; t < k; t++) {
            double m = mcoef(lv, i, nb[t].j, ii, nb[t].axis);
            mii += m;
            f += m * lv->psi[nb[t].j];
        }
        double kap = kappa_i(S, lv, i, ii);
        f += kap * lv->psi[i];
        double c = S->p.xi + kap + mii;
        double beta = root_beta(S, elev(S, lv, ii));
        out[q] = orc_local_solve(law_at(S, lv, i), S->a, beta, c, f, lv->psi[i],
                                 S->p.newton_iters, NULL);
    }
}

/* Defect d = g - N(psi) on level l (0 at Dirichlet nodes); returns max |d|. */
double orc_residual(orc_solver *S, int l, double *dout)
{
    orc_level *lv = &S->lev[l];
    double *d = dout ? dout : lv->d;
    double mx = 0.0;
#pragma omp parallel for schedule(static) reduction(max:mx)
    for (int i = 0; i < lv->N; i++) {
        int ii[3];
        coords(lv, i, ii);
        if (is_dirichlet(S, lv, ii, NULL)) { d[i] = 0.0; continue; }
        d[i] = lv->g[i] - Nop(S, lv, lv->psi, i, ii);
        double ad = fabs(d[i]);
        if (ad > mx || ad != ad) mx = ad;
    }
    return mx;
}

/* Scale of the rounding floor of the defect on level l: the largest sum over
 * an unknown node of the magnitudes of the terms its defect adds up, |g_i|,
 * a |theta(psi_i)|, |S(psi_i)|, xi |psi_i| and m_ij (|psi_i| + |psi_j|) per
 * face.  Rounding psi_i by one ulp moves the defect by m_ii ulp(psi_i), and
 * evaluating it rounds each of these terms, so a converged iterate cannot
 * bring the max-norm of the defect much below eps times this scale (the
 * stopping test of section 3.2 then stalls). */
double orc_defect_scale(orc_solver *S, int l)
{
    orc_level *lv = &S->lev[l];
    double mx = 0.0;
#pragma omp parallel for schedule(static) reduction(max:mx)
    for (int i = 0; i < lv->N; i++) {
        int ii[3];
        coords(lv, i, ii);
        if (is_dirichlet(S, lv, ii, NULL)) continue;
        double x = lv->psi[i];
        const orc_params *law = law_at(S, lv, i);
        double t = fabs(lv->g[i]) + fabs(S->a * orc_theta(law, x)) + fabs(S->p.xi * x);
        if (S->p.sink == ORC_SINK_FEDDES_EXP)
            t += fabs(root_beta(S, elev(S, lv, ii)) * orc_feddes(&S->p, x));
        orc_nb nb[6];
        int k = neighbours(S, lv, ii, nb);
        for (int q = 0; q < k; q++)
            t += mcoef(lv, i, nb[q].j, ii, nb[q].axis) * (fabs(x) + fabs(lv->psi[nb[q].j]));
        if (t > mx) mx = t;
    }
    return mx;
}

/* ------------------------------------------------------------------------ */
/* Transfer operators: full weighting and linear interpolation.             */
/* ------------------------------------------------------------------------ */

/* Full-weighting restriction of a fine array to coarse node I: tensor product
 * of (1/4, 1/2, 1/4) around fine node 2I; at a boundary node the missing
 * fine neighbour is mirrored (weights 1/2, 1/2). */
static double fw_at(const orc_level *fl, const double *v, const int I[3], int dim)
{
    double s = 0.0;
    int c[3] = {2 * I[0], 2 * I[1], 2 * I[2]};
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int l = 0; l < dim; l++) { lo[l] = -1; hi[l] = 1; }
    for (int d2 = lo[2]; d2 <= hi[2]; d2++)
        for (int d1 = lo[1]; d1 <= hi[1]; d1++)
            for (int d0 = lo[0]; d0 <= hi[0]; d0++) {
                int dd[3] = {d0, d1, d2}, jj[3];
                double w = 1.0;
                for (int l = 0; l < 3; l++) {
                    jj[l] = c[l] + dd[l];
                    if (l >= dim) continue;
                    w *= (dd[l] == 0) ? 0.5 : 0.25;
                    if (jj[l] < 0) jj[l] = -jj[l];                       /* mirror */
                    if (jj[l] > fl->n[l] - 1) jj[l] = 2 * (fl->n[l] - 1) - jj[l];
                }
                s += w * v[index_of(fl, jj)];
            }
    return s;
}

/* Step 3-4 of the two-grid FAS algorithm: restrict psi and the defect, then
 * g_H = N_H(psibar_H) + d_H and psi_H = psibar_H.  Coarse Dirichlet nodes
 * take the fine value by injection. */
void orc_restrict(orc_solver *S, int l)
{
    orc_level *fl = &S->lev[l], *cl = &S->lev[l + 1];
    int dim = S->grid.dim;
    double *dH = (double *)malloc(sizeof(double) * cl->N);
#pragma omp parallel for schedule(static)
    for (int I = 0; I < cl->N; I++) {
        int II[3];
        coords(cl, I, II);
        if (is_dirichlet(S, cl, II, NULL)) {
            int jj[3] = {2 * II[0], 2 * II[1], 2 * II[2]};
            cl->psibar[I] = fl->psi[index_of(fl, jj)];
            dH[I] = 0.0;
        } else {
            cl->psibar[I] = fw_at(fl, fl->psi, II, dim);
            dH[I] = fw_at(fl, fl->d, II, dim);
        }
    }
#pragma omp parallel for schedule(static)
    for (int I = 0; I < cl->N; I++) {
        int II[3];
        coords(cl, I, II);
        if (is_dirichlet(S, cl, II, NULL)) { cl->g[I] = 0.0; continue; }
        cl->g[I] = Nop(S, cl, cl->psibar, I, II) + dH[I];
    }
    memcpy(cl->psi, cl->psibar, sizeof(double) * cl->N);
    free(dH);
}

/* Step 6: e_H = psi_H - psibar_H, psi_h += I_h^H e_H (tensor linear
 * interpolation) at fine unknown nodes. */
void orc_prolong(orc_solver *S, int l)
{
    orc_level *fl = &S->lev[l], *cl = &S->lev[l + 1];
    int dim = S->grid.dim;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < fl->N; i++) {
        int ii[3];
        coords(fl, i, ii);
        if (is_dirichlet(S, fl, ii, NULL)) continue;
        int ia[3][2], na[3];
        double wa[3][2];
        for (int a = 0; a < 3; a++) {
            if (a >= dim || (ii[a] % 2) == 0) {
                na[a] = 1; ia[a][0] = ii[a] / 2; wa[a][0] = 1.0;
            } else {
                na[a] = 2;
                ia[a][0] = (ii[a] - 1) / 2; wa[a][0] = 0.5;
                ia[a][1] = (ii[a] + 1) / 2; wa[a][1] = 0.5;
            }
        }
        double e = 0.0;
        for (int c2 = 0; c2 < na[2]; c2++)
            for (int c1 = 0; c1 < na[1]; c1++)
                for (int c0 = 0; c0 < na[0]; c0++) {
                    int JJ[3] = {ia[0][c0], ia[1][c1], ia[2][c2]};
                    int J = index_of(cl, JJ);
                    e += wa[0][c0] * wa[1][c1] * wa[2][c2] * (cl->psi[J] - cl->psibar[J]);
                }
        fl->psi[i] += e;
    }
}

/* FAS V-cycle (section 3.2, the two-grid algorithm with the coarse solve
 * replaced by recursion).  On the coarsest level (3 nodes on the shortest
 * axis) a fixed number of sweeps stands in for the coarse solve. */
static void vcycle_level(orc_solver *S, int l, int nu1, int nu2)
{
    if (l == S->nlev - 1) {
        orc_sweep(S, l, S->nu_coarse);
        return;
    }
    orc_sweep(S, l, nu1);
    orc_residual(S, l, NULL);
    orc_restrict(S, l);
    vcycle_level(S, l + 1, nu1, nu2);
    orc_prolong(S, l);
    orc_sweep(S, l, nu2);
}

void orc_vcycle(orc_solver *S, int nu1, int nu2)
{
    vcycle_level(S, 0, nu1, nu2);
}

/* Full multigrid (section 3.2, the closing paragraph on V-cycles and FMG: start
 * on the coarsest grid, interpolate the solution to the finer grids and run
 * V-cycles on each; the standard scheme, read as follows).  Going down, every
 * coarser level gets the full-weighting restriction of the finer right-hand
 * side (zero at its Dirichlet nodes) and the injection of the finer iterate;
 * the coarsest level is smoothed nu_coarse times; going up, every level starts
 * from the linear interpolation of the coarser solution at its unknown nodes
 * (Dirichlet nodes keep their values) and runs one FAS V-cycle V(nu1, nu2)
 * with its own right-hand side. */
void orc_fmg(orc_solver *S, int nu1, int nu2)
{
    int dim = S->grid.dim;
    for (int l = 0; l + 1 < S->nlev; l++) {
        orc_level *fl = &S->lev[l], *cl = &S->lev[l + 1];
#pragma omp parallel for schedule(static)
        for (int I = 0; I < cl->N; I++) {
            int II[3];
            coords(cl, I, II);
            int jj[3] = {2 * II[0], 2 * II[1], 2 * II[2]};
            cl->psi[I] = fl->psi[index_of(fl, jj)];
            cl->g[I] = is_dirichlet(S, cl, II, NULL) ? 0.0 : fw_at(fl, fl->g, II, dim);
        }
    }
    orc_sweep(S, S->nlev - 1, S->nu_coarse);
    for (int l = S->nlev - 2; l >= 0; l--) {
        orc_level *fl = &S->lev[l], *cl = &S->lev[l + 1];
#pragma omp parallel for schedule(static)
        for (int i = 0; i < fl->N; i++) {
            int ii[3];
            coords(fl, i, ii);
            if (is_dirichlet(S, fl, ii, NULL)) continue;
            int ia[3][2], na[3];
            double wa[3][2];
            for (int a = 0; a < 3; a++) {
                if (a >= dim || (ii[a] % 2) == 0) {
                    na[a] = 1; ia[a][0] = ii[a] / 2; wa[a][0] = 1.0;
                } else {
                    na[a] = 2;
                    ia[a][0] = (ii[a] - 1) / 2; wa[a][0] = 0.5;
                    ia[a][1] = (ii[a] + 1) / 2; wa[a][1] = 0.5;
                }
            }
            double v = 0.0;
            for (int c2 = 0; c2 < na[2]; c2++)
                for (int c1 = 0; c1 < na[1]; c1++)
                    for (int c0 = 0; c0 < na[0]; c0++) {
                        int JJ[3] = {ia[0][c0], ia[1][c1], ia[2][c2]};
                        v += wa[0][c0] * wa[1][c1] * wa[2][c2] * cl->psi[index_of(cl, JJ)];
                    }
            fl->psi[i] = v;
        }
        vcycle_level(S, l, nu1, nu2);
    }
}

/* ------------------------------------------------------------------------ */
/* Time stepping (eq. fully-bdf1; BDF2 reading).                             */
/* ------------------------------------------------------------------------ */

/* Prepare the system N(psi) = g of one step.  BDF1 (eq. fully-bdf1):
 * a = 1/tau, history theta(psi^n)/tau, lagged state psi* = psi^n.  BDF2
 * (reading): a = 3/(2 tau), history (4 theta(psi^n) - theta(psi^{n-1}))/(2 tau);
 * the lagged state is psi* = psi^n as in BDF1 (the paper lags the diffusion
 * operator at the previous state), or, when lag_extrap is set, the
 * extrapolation 2 psi^n - psi^{n-1}; the first step is BDF1.  K* = K(psi*) at every
 * node (Dirichlet nodes take their boundary value as lagged state), and
 * g = history + xi psi* - (M z) - free-drainage outflow (eq. Nh-def).  Coarse
 * levels take K* by injection, or as the full-weighting average of the finer
 * level's K* (coarse_k = ORC_COARSE_FW).  The iterate starts from psi^n. */
void orc_begin_step(orc_solver *S, double dt, int order)
{
    orc_level *f0 = &S->lev[0];
    S->dt = dt;
    S->order_eff = (order == 2 && S->nstep > 0) ? 2 : 1;
    S->a = (S->order_eff == 1) ? 1.0 / dt : 1.5 / dt;
    double *psistar = (double *)malloc(sizeof(double) * f0->N);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < f0->N; i++) {
        int ii[3];
        double bv;
        coords(f0, i, ii);
        int from_state;
        if (is_dirichlet_src(S, f0, ii, &bv, &from_state)) {
            if (from_state) bv = S->psi_n[i];
            psistar[i] = bv;
            f0->psi[i] = bv;
        } else {
            psistar[i] = (S->order_eff == 2 && S->p.lag_extrap) ? 2.0 * S->psi_n[i] - S->psi_nm1[i] : S->psi_n[i];
            f0->psi[i] = S->psi_n[i];
        }
        const orc_params *law = law_at(S, f0, i);
        double ks = S->Ks_field ? S->Ks_field[i] : law->Ks;
        f0->Kstar[i] = ks * orc_Krel(law, psistar[i]);
    }
    int v = S->grid.dim - 1;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < f0->N; i++) {
        int ii[3];
        coords(f0, i, ii);
        if (is_dirichlet(S, f0, ii, NULL)) { f0->g[i] = 0.0; continue; }
        const orc_params *law = law_at(S, f0, i);
        double H;
        if (S->order_eff == 1)
            H = orc_theta(law, S->psi_n[i]) / dt;
        else
            H = (4.0 * orc_theta(law, S->psi_n[i]) - orc_theta(law, S->psi_nm1[i])) / (2.0 * dt);
        double gi = H + S->p.xi * psistar[i] - Mz(S, f0, i, ii);
        if (ii[v] == 0 && S->grid.face_bc[2 * v] == ORC_BC_FREEDRAIN)
            gi -= f0->Kstar[i] / (wfrac(f0, ii, v) * f0->h[v]);
        f0->g[i] = gi;
    }
    free(psistar);
    for (int l = 1; l < S->nlev; l++) {
        orc_level *cl = &S->lev[l], *fl = &S->lev[l - 1];
        for (int I = 0; I < cl->N; I++) {
            int II[3];
            coords(cl, I, II);
            int jj[3] = {2 * II[0], 2 * II[1], 2 * II[2]};
            cl->Kstar[I] = (S->p.coarse_k == ORC_COARSE_FW) ? fw_at(fl, fl->Kstar, II, S->grid.dim)
                                                             : fl->Kstar[index_of(fl, jj)];
        }
    }
    for (int l = 0; l < S->nlev; l++) {
        if (S->p.kappa_rule == ORC_KAPPA_REMARK) compute_lambdaU(S, &S->lev[l]);
    }
}

/* Accept the iterate as psi^{n+1}. */
void orc_end_step(orc_solver *S)
{
    orc_level *f0 = &S->lev[0];
    memcpy(S->psi_nm1, S->psi_n, sizeof(double) * f0->N);
    memcpy(S->psi_n, f0->psi, sizeof(double) * f0->N);
    S->nstep++;
}

/* V-cycles until the fine residual max-norm is <= tol or max_cycles is hit.
 * res_hist receives the norm before each cycle and after the last (length
 * max_cycles+1).  Returns the number of cycles done. */
int orc_solve_step(orc_solver *S, int nu1, int nu2, int max_cycles, double tol, double *res_hist)
{
    int c = 0;
    double r = orc_residual(S, 0, NULL);
    if (res_hist) res_hist[0] = r;
    while (c < max_cycles && r > tol) {
        orc_vcycle(S, nu1, nu2);
        c++;
        r = orc_residual(S, 0, NULL);
        if (res_hist) res_hist[c] = r;
    }
    return c;
}

/* ------------------------------------------------------------------------ */
/* Construction and field access.                                            */
/* ------------------------------------------------------------------------ */

orc_solver *orc_create(const orc_grid *g, const orc_params *p, const double *Ks_field,
                       int ordering, int nu_coarse)
{
    orc_solver *S = (orc_solver *)calloc(1, sizeof(orc_solver));
    S->grid = *g;
    S->p = *p;
    S->ordering = ordering;
    S->nu_coarse = nu_coarse;
    int n[3] = {1, 1, 1};
    for (int l = 0; l < g->dim; l++) n[l] = g->n[l];
    int nmin = n[0];
    for (int l = 1; l < g->dim; l++) if (n[l] < nmin) nmin = n[l];
    int nlev = 1;
    while (nmin > 3) { nmin = (nmin - 1) / 2 + 1; nlev++; }
    S->nlev = nlev;
    for (int k = 0; k < nlev; k++) {
        orc_level *lv = &S->lev[k];
        int N = 1;
        for (int l = 0; l < 3; l++) {
            if (l < g->dim) {
                lv->n[l] = ((n[l] - 1) >> k) + 1;
                lv->h[l] = g->L[l] / (lv->n[l] - 1);
            } else {
                lv->n[l] = 1;
                lv->h[l] = 1.0;
            }
            N *= lv->n[l];
        }
        lv->N = N;
        for (int t = 0; t < 2; t++) {
            int s = 1 << k;
            lv->patch_lo[t] = (g->patch_lo[t] + s - 1) / s;   /* ceil */
            lv->patch_hi[t] = g->patch_hi[t] / s;             /* floor */
        }
        lv->psi = (double *)calloc(N, sizeof(double));
        lv->Kstar = (double *)calloc(N, sizeof(double));
        lv->g = (double *)calloc(N, sizeof(double));
        lv->psibar = (double *)calloc(N, sizeof(double));
        lv->d = (double *)calloc(N, sizeof(double));
    }
    int N0 = S->lev[0].N;
    S->psi_n = (double *)calloc(N0, sizeof(double));
    S->psi_nm1 = (double *)calloc(N0, sizeof(double));
    if (Ks_field) {
        S->Ks_field = (double *)malloc(sizeof(double) * N0);
        memcpy(S->Ks_field, Ks_field, sizeof(double) * N0);
    }
    /* trapezoidal integral of exp(-(Lz - z)/root_len) over the fine column */
    {
        int v = g->dim - 1;
        orc_level *f0 = &S->lev[0];
        double Z = 0.0;
        for (int k = 0; k < f0->n[v]; k++) {
            double w = (k == 0 || k == f0->n[v] - 1) ? 0.5 : 1.0;
            Z += w * f0->h[v] * exp(-(g->L[v] - k * f0->h[v]) / p->root_len);
        }
        S->beta_norm = Z;
    }
    S->a = 1.0;
    return S;
}

/* Per-node soils (the layered and two-layer media of section 4): table
 * entries supply the soil law (model, theta_s, theta_r, Ks and the model's
 * parameters); everything else (sink, xi, kappa, Newton settings) stays that
 * of the problem.  ids holds one table index per fine node.  Reading: a
 * coarse node takes the soil of the fine node it coincides with (injection,
 * as for K*).  Returns 0, or -1 for a bad table or index, or when a per-node
 * Ks field is set (a soil's Ks comes from its entry). */
int orc_set_soils(orc_solver *S, int n, const orc_params *table, const unsigned char *ids)
{
    if (n < 1 || n > ORC_MAXSOIL || S->Ks_field) return -1;
    orc_level *f0 = &S->lev[0];
    for (int i = 0; i < f0->N; i++)
        if (ids[i] >= n) return -1;
    S->nsoil = n;
    for (int s = 0; s < n; s++) {
        orc_params q = S->p;
        q.model = table[s].model;
        q.theta_s = table[s].theta_s;
        q.theta_r = table[s].theta_r;
        q.Ks = table[s].Ks;
        q.vg_alpha = table[s].vg_alpha;
        q.vg_n = table[s].vg_n;
        q.hk_alpha = table[s].hk_alpha;
        q.hk_beta = table[s].hk_beta;
        q.hk_A = table[s].hk_A;
        q.hk_gamma = table[s].hk_gamma;
        q.psi_unit = table[s].psi_unit;
        q.lin_c = table[s].lin_c;
        q.gd_alpha = table[s].gd_alpha;
        S->soil[s] = q;
    }
    for (int k = 0; k < S->nlev; k++) {
        orc_level *lv = &S->lev[k];
        if (!lv->sid) lv->sid = (unsigned char *)malloc((size_t)lv->N);
        if (k == 0) {
            memcpy(lv->sid, ids, (size_t)lv->N);
            continue;
        }
        orc_level *fl = &S->lev[k - 1];
        for (int I = 0; I < lv->N; I++) {
            int II[3];
            coords(lv, I, II);
            int jj[3] = {2 * II[0], 2 * II[1], 2 * II[2]};
            lv->sid[I] = fl->sid[index_of(fl, jj)];
        }
    }
    return 0;
}

void orc_destroy(orc_solver *S)
{
    if (!S) return;
    for (int k = 0; k < S->nlev; k++) {
        free(S->lev[k].psi); free(S->lev[k].Kstar); free(S->lev[k].g);
        free(S->lev[k].psibar); free(S->lev[k].d); free(S->lev[k].sid);
    }
    free(S->psi_n); free(S->psi_nm1); free(S->Ks_field);
    free(S);
}

int orc_nlevels(const orc_solver *S) { return S->nlev; }

void orc_level_shape(const orc_solver *S, int l, int *n)
{
    for (int a = 0; a < 3; a++) n[a] = S->lev[l].n[a];
}

double orc_get_a(const orc_solver *S) { return S->a; }
void orc_set_a(orc_solver *S, double a) { S->a = a; }
double orc_get_lambdaU(const orc_solver *S, int l) { return S->lev[l].lambdaU; }

/* psi^n (and psi^{n-1} for BDF2 restarts) and the step counter. */
void orc_set_state(orc_solver *S, const double *psi_n, const double *psi_nm1, int nstep)
{
    int N0 = S->lev[0].N;
    memcpy(S->psi_n, psi_n, sizeof(double) * N0);
    memcpy(S->psi_nm1, psi_nm1 ? psi_nm1 : psi_n, sizeof(double) * N0);
    S->nstep = nstep;
}

static double *field_ptr(orc_solver *S, int l, int which)
{
    orc_level *lv = &S->lev[l];
    switch (which) {
    case ORC_FIELD_PSI: return lv->psi;
    case ORC_FIELD_KSTAR: return lv->Kstar;
    case ORC_FIELD_G: return lv->g;
    case ORC_FIELD_PSIBAR: return lv->psibar;
    case ORC_FIELD_PSI_N: return S->psi_n;
    case ORC_FIELD_PSI_NM1: return S->psi_nm1;
    default: return NULL;
    }
}

int orc_get_field(orc_solver *S, int l, int which, double *out)
{
    double *p = field_ptr(S, l, which);
    if (!p) return -1;
    int N = (which >= ORC_FIELD_PSI_N) ? S->lev[0].N : S->lev[l].N;
    memcpy(out, p, sizeof(double) * N);
    return 0;
}

int orc_set_field(orc_solver *S, int l, int which, const double *in)
{
    double *p = field_ptr(S, l, which);
    if (!p) return -1;
    int N = (which >= ORC_FIELD_PSI_N) ? S->lev[0].N : S->lev[l].N;
    memcpy(p, in, sizeof(double) * N);
    if (which == ORC_FIELD_KSTAR && S->p.kappa_rule == ORC_KAPPA_REMARK)
        compute_lambdaU(S, &S->lev[l]);
    return 0;
}

/* Node kinds of level l: 1 Dirichlet, 0 unknown. */
void orc_node_kinds(orc_solver *S, int l, int8_t *out)
{
    orc_level *lv = &S->lev[l];
    for (int i = 0; i < lv->N; i++) {
        int ii[3];
        coords(lv, i, ii);
        out[i] = (int8_t)is_dirichlet(S, lv, ii, NULL);
    }
}

/* Assemble the dense matrix M (unknown rows and columns only, in flattened
 * order) of level l, together with kappa_i, for the structural checks of the
 * Proposition, the Lemma and the contraction theorem.  mat is nu x nu
 * row-major, nu = number of unknowns; unk receives their flattened indices. */
int orc_dense_M(orc_solver *S, int l, double *mat, double *kap, int *unk)
{
    orc_level *lv = &S->lev[l];
    int *pos = (int *)malloc(sizeof(int) * lv->N);
    int nu = 0;
    for (int i = 0; i < lv->N; i++) {
        int ii[3];
        coords(lv, i, ii);
        pos[i] = is_dirichlet(S, lv, ii, NULL) ? -1 : nu++;
    }
    if (mat) memset(mat, 0, sizeof(double) * (size_t)nu * nu);
    for (int i = 0; i < lv->N; i++) {
        if (pos[i] < 0) continue;
        int ii[3];
        coords(lv, i, ii);
        if (unk) unk[pos[i]] = i;
        if (kap) kap[pos[i]] = kappa_i(S, lv, i, ii);
        if (!mat) continue;
        orc_nb nb[6];
        int k = neighbours(S, lv, ii, nb);
        for (int q = 0; q < k; q++) {
            double m = mcoef(lv, i, nb[q].j, ii, nb[q].axis);
            mat[(size_t)pos[i] * nu + pos[i]] += m;
            if (pos[nb[q].j] >= 0) mat[(size_t)pos[i] * nu + pos[nb[q].j]] -= m;
        }
    }
    free(pos);
    return nu;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
