"""Pins of the oracle's FAS V-cycle (section 3.2, the two-grid FAS algorithm
applied recursively): the converged result against a dense global Newton
solve, the iterates against linear correction-scheme multigrid for a linear
law, and symmetry / dimension-reduction properties."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.linalg import solve_triangular

from paper_2606_04292_amd import workloads as W
from tests.test_oracle_operator import textbook_laplacian

RNG = np.random.default_rng(7)


def law_vg(**kw):
    base = dict(model=W.MODEL_VGM, theta_s=0.43, theta_r=0.05, Ks=1e-5, vg_alpha=3.6, vg_n=1.56)
    base.update(kw)
    return W.LawSpec(**base)


def workload(g, law, psi0, ks=None, order=1, dt=120.0, nu1=2, nu2=2):
    return W.Workload("t", g, law, np.ascontiguousarray(psi0, dtype=np.float64), dt=dt, steps=1,
                      order=order, Ks_field=ks, nu1=nu1, nu2=nu2)


def dense_newton(orc, S, law, iters=60):
    """Global Newton on N(psi) = g over the unknowns, Jacobian
    diag(a theta' + S' + xi) + M, using the oracle's N and M."""
    kinds = S.kinds().astype(bool).ravel()
    M, _, unk = S.dense_M()
    g = S.get(orc.FIELD_G).ravel()
    psi = S.psi().ravel().copy()
    _, dth, _, _, dfa = orc.law_fns(law)
    shape = S.shapes[0]
    for _ in range(iters):
        F = (S.apply_N(psi.reshape(shape)).ravel() - g)[unk]
        if np.abs(F).max() < 1e-17:
            break
        dg = np.array([S.a * dth(x) + law.xi for x in psi[unk]])
        J = M + np.diag(dg)
        psi[unk] -= np.linalg.solve(J, F)
    return psi.reshape(shape), kinds


CASES = [
    ("1d", W.GridSpec(dim=1, n=[33], L=[1.0], face_bc=[W.BC_FREEDRAIN, W.BC_DIRICHLET],
                      face_value=[0.0, -0.2])),
    ("2d", W.GridSpec(dim=2, n=[9, 9], L=[1.0, 1.0],
                      face_bc=[W.BC_NOFLUX, W.BC_NOFLUX, W.BC_DIRICHLET, W.BC_NOFLUX],
                      face_value=[0, 0, -1.5, 0], patch_face=3, patch_lo=(3, 0), patch_hi=(5, 0),
                      patch_value=-0.05)),
    ("3d", W.GridSpec(dim=3, n=[5, 5, 5], L=[1.0, 1.0, 1.0],
                      face_bc=[W.BC_NOFLUX] * 4 + [W.BC_FREEDRAIN, W.BC_DIRICHLET],
                      face_value=[0.0] * 5 + [-0.1])),
]


@pytest.mark.parametrize("name,g", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("ordering", ["lex", "rb"])
def test_converged_fas_equals_dense_newton(orc, name, g, ordering):
    """The step system N_h(psi) = g_h (eq. Nh-system) has a unique solution;
    the FAS V-cycle iterated to the rounding floor must reach the same root as
    an independent dense Newton solve."""
    o = orc.ORDER_LEX if ordering == "lex" else orc.ORDER_RB
    ks = np.exp(RNG.normal(np.log(1e-5), 0.8, size=g.shape))
    psin = RNG.uniform(-1.5, -0.3, size=g.shape)
    law = law_vg(xi=1e-6)
    S = orc.Solver(workload(g, law, psin, ks), o)
    S.begin_step()
    ref, kinds = dense_newton(orc, S, law)
    hist = orc.solve_to_floor(S, 80, 0.0)
    assert hist[-1] < 1e-15 * S.a
    got = S.psi()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


# --- linear correction-scheme multigrid, written independently ------------

def fw_1d(nf, lo_dir, hi_dir):
    nc = (nf - 1) // 2 + 1
    R = np.zeros((nc, nf))
    for I in range(nc):
        i = 2 * I
        R[I, i] += 0.5
        for j in (i - 1, i + 1):
            jj = -j if j < 0 else (2 * (nf - 1) - j if j > nf - 1 else j)
            R[I, jj] += 0.25
    return R


def interp_1d(nf):
    nc = (nf - 1) // 2 + 1
    P = np.zeros((nf, nc))
    for i in range(nf):
        if i % 2 == 0:
            P[i, i // 2] = 1.0
        else:
            P[i, (i - 1) // 2] = 0.5
            P[i, (i + 1) // 2] = 0.5
    return P


def kron_all(mats):
    out = None
    for m in reversed(mats):          # axis 0 fastest
        out = m if out is None else np.kron(out, m)
    return out


def unknown_mask(g):
    mask = np.ones(g.shape, dtype=bool)
    for l in range(g.dim):
        ax = g.dim - 1 - l
        for side, f in ((0, 2 * l), (-1, 2 * l + 1)):
            if g.face_bc[f] == W.BC_DIRICHLET:
                idx = [slice(None)] * g.dim
                idx[ax] = side
                mask[tuple(idx)] = False
    return mask.ravel()


def coarsen(g):
    return W.GridSpec(dim=g.dim, n=[(m - 1) // 2 + 1 for m in g.n], L=g.L,
                      face_bc=g.face_bc, face_value=g.face_value)


def rb_perm(g, unk_idx):
    shape = g.shape
    col = np.array([sum(np.unravel_index(i, shape)) % 2 for i in unk_idx])
    return np.concatenate([np.where(col == 0)[0], np.where(col == 1)[0]])


def kappa_rel(A, kappa):
    return kappa * np.diag(A)


def cs_vcycle(levels, l, x, b, nu1, nu2, nuc):
    A, P, R, perm, kap, diag = levels[l]

    def smooth(x, k):
        Ap = A[np.ix_(perm, perm)] + np.diag(diag[perm])
        kp = kap[perm]
        low = np.tril(Ap) + np.diag(kp)
        up = np.triu(Ap, 1)
        for _ in range(k):
            xp = x[perm]
            xn = solve_triangular(low, b[perm] + kp * xp - up @ xp, lower=True)
            x = np.empty_like(xn)
            x[perm] = xn
        return x

    if l == len(levels) - 1:
        return smooth(x, nuc)
    x = smooth(x, nu1)
    r = b - (A + np.diag(diag)) @ x
    rH = R @ r
    eH = cs_vcycle(levels, l + 1, np.zeros(len(rH)), rH, nu1, nu2, nuc)
    x = x + P @ eH
    return smooth(x, nu2)


@pytest.mark.parametrize("dim,n", [(1, 33), (2, 17), (3, 9)])
def test_linear_law_fas_iterates_equal_correction_scheme_mg(orc, dim, n):
    """For a linear law, FAS (coarse rhs N_H(R psi) + R d, correction
    psi_H - R psi) and correction-scheme multigrid on A e = r produce the same
    iterates.  The CS cycle here uses its own full-weighting / interpolation
    matrices, textbook Laplacians on every level and shifted red-black GS."""
    bcs = [W.BC_NOFLUX] * (2 * dim)
    bcs[2 * (dim - 1)] = W.BC_DIRICHLET
    bcs[0] = W.BC_DIRICHLET
    g = W.GridSpec(dim=dim, n=[n] * dim, L=[1.0] * dim, face_bc=bcs, face_value=[0.0] * (2 * dim))
    law = W.LawSpec(model=W.MODEL_LINEAR, theta_s=0.4, theta_r=0.1, Ks=1e-3, lin_c=0.02,
                    xi=1e-5, kappa_rule=W.KAPPA_REL, kappa=0.1, newton_iters=2)
    psin = RNG.uniform(-1, 1, size=g.shape)
    S = orc.Solver(workload(g, law, psin), orc.ORDER_RB)
    S.begin_step()
    a = S.a
    unk_mask = unknown_mask(g)
    levels = []
    gl = g
    for l in range(S.nlev):
        A = textbook_laplacian(gl) * law.Ks
        um = unknown_mask(gl)
        unk_idx = np.where(um)[0]
        diag = np.full(A.shape[0], a * law.lin_c + law.xi)
        P = R = None
        if l < S.nlev - 1:
            gc = coarsen(gl)
            umc = unknown_mask(gc)
            Rf = kron_all([fw_1d(gl.n[k], 0, 0) for k in range(dim)])
            Pf = kron_all([interp_1d(gl.n[k]) for k in range(dim)])
            R = Rf[np.ix_(umc, um)]
            P = Pf[np.ix_(um, umc)]
            gnext = gc
        levels.append((A, P, R, rb_perm(gl, unk_idx), kappa_rel(A, law.kappa), diag))
        if l < S.nlev - 1:
            gl = gnext
    M0, _, unk0 = S.dense_M()
    assert np.allclose(M0, levels[0][0], rtol=1e-13, atol=1e-13 * np.abs(M0).max())
    x = S.psi().ravel()[unk_mask]
    b = S.get(orc.FIELD_G).ravel()[unk_mask] - a * law.theta_r
    for cyc in range(3):
        x = cs_vcycle(levels, 0, x, b, 2, 2, 32)
        S.vcycle(2, 2)
        got = S.psi().ravel()[unk_mask]
        np.testing.assert_allclose(got, x, rtol=0, atol=1e-11 * max(1.0, np.abs(x).max()))


def test_laterally_uniform_3d_equals_1d_column(orc):
    """With no-flux side faces and laterally uniform data the 3-D solution is
    the 1-D column solution (the side half-volumes cancel)."""
    n = 17
    law = law_vg(xi=0.0)
    z = np.linspace(0.0, 1.0, n)
    psi_col = -1.0 + 0.5 * z
    g1 = W.GridSpec(dim=1, n=[n], L=[1.0], face_bc=[W.BC_DIRICHLET, W.BC_DIRICHLET],
                    face_value=[-1.0, -0.1])
    g3 = W.GridSpec(dim=3, n=[n, n, n], L=[1.0, 1.0, 1.0],
                    face_bc=[W.BC_NOFLUX] * 4 + [W.BC_DIRICHLET, W.BC_DIRICHLET],
                    face_value=[0.0] * 4 + [-1.0, -0.1])
    S1 = orc.Solver(workload(g1, law, psi_col, order=2), orc.ORDER_RB)
    S3 = orc.Solver(workload(g3, law, np.broadcast_to(psi_col[:, None, None], g3.shape), order=2),
                    orc.ORDER_RB)
    for _ in range(3):
        for S in (S1, S3):
            S.begin_step()
            orc.solve_to_floor(S, 80, 0.0)
            S.end_step()
    p1 = S1.get(orc.FIELD_PSI_N)
    p3 = S3.get(orc.FIELD_PSI_N)
    assert np.abs(p3 - p1[:, None, None]).max() <= 1e-12 * np.abs(p1).max()


def test_mirror_symmetric_data_give_mirror_symmetric_iterates(orc):
    g = W.GridSpec(dim=2, n=[33, 33], L=[1.0, 1.0],
                   face_bc=[W.BC_NOFLUX, W.BC_NOFLUX, W.BC_FREEDRAIN, W.BC_NOFLUX],
                   face_value=[0.0] * 4, patch_face=3, patch_lo=(12, 0), patch_hi=(20, 0),
                   patch_value=0.0)
    ks = np.exp(RNG.normal(np.log(1e-5), 1.0, size=g.shape))
    ks = 0.5 * (ks + ks[:, ::-1])
    psin = RNG.uniform(-1.5, -0.5, size=g.shape)
    psin = 0.5 * (psin + psin[:, ::-1])
    S = orc.Solver(workload(g, law_vg(), psin, ks), orc.ORDER_RB)
    S.begin_step()
    for _ in range(3):
        S.vcycle()
        p = S.psi()
        assert np.abs(p - p[:, ::-1]).max() <= 1e-13 * np.abs(p).max()


def inject_1d(nf):
    nc = (nf - 1) // 2 + 1
    Q = np.zeros((nc, nf))
    for I in range(nc):
        Q[I, 2 * I] = 1.0
    return Q


@pytest.mark.parametrize("dim,n", [(1, 33), (2, 17), (3, 9)])
def test_linear_law_fmg_equals_textbook_fmg(orc, dim, n):
    """Full multigrid, linear law: the oracle's FMG(2,2) equals a textbook
    linear FMG written here from explicit matrices: right-hand sides restricted
    down the hierarchy by full weighting (zero at Dirichlet nodes), the
    injected fine state smoothed on the coarsest level, then on every finer
    level linear interpolation of the coarse solution followed by one
    correction-scheme V(2,2) cycle."""
    bcs = [W.BC_NOFLUX] * (2 * dim)
    bcs[2 * (dim - 1)] = W.BC_DIRICHLET
    bcs[0] = W.BC_DIRICHLET
    g = W.GridSpec(dim=dim, n=[n] * dim, L=[1.0] * dim, face_bc=bcs, face_value=[0.0] * (2 * dim))
    law = W.LawSpec(model=W.MODEL_LINEAR, theta_s=0.4, theta_r=0.1, Ks=1e-3, lin_c=0.02,
                    xi=1e-5, kappa_rule=W.KAPPA_REL, kappa=0.1, newton_iters=2)
    psin = RNG.uniform(-1, 1, size=g.shape)
    S = orc.Solver(workload(g, law, psin), orc.ORDER_RB)
    S.begin_step()
    a = S.a
    levels, grids = [], []
    gl = g
    for l in range(S.nlev):
        grids.append(gl)
        A = textbook_laplacian(gl) * law.Ks
        um = unknown_mask(gl)
        diag = np.full(A.shape[0], a * law.lin_c + law.xi)
        P = R = None
        if l < S.nlev - 1:
            gc = coarsen(gl)
            umc = unknown_mask(gc)
            R = kron_all([fw_1d(gl.n[k], 0, 0) for k in range(dim)])[np.ix_(umc, um)]
            P = kron_all([interp_1d(gl.n[k]) for k in range(dim)])[np.ix_(um, umc)]
        levels.append((A, P, R, rb_perm(gl, np.where(um)[0]), kappa_rel(A, law.kappa), diag))
        if l < S.nlev - 1:
            gl = gc
    # right-hand sides: full-grid g restricted with zeros kept at Dirichlet nodes
    G = [S.get(orc.FIELD_G).ravel()]
    X = [S.psi().ravel()]
    for l in range(S.nlev - 1):
        gf, gc = grids[l], grids[l + 1]
        Rf = kron_all([fw_1d(gf.n[k], 0, 0) for k in range(dim)])
        Qf = kron_all([inject_1d(gf.n[k]) for k in range(dim)])
        gn = Rf @ G[-1]
        gn[~unknown_mask(gc)] = 0.0
        G.append(gn)
        X.append(Qf @ X[-1])
    B = [G[l][unknown_mask(grids[l])] - a * law.theta_r for l in range(S.nlev)]
    L = S.nlev - 1
    x = cs_vcycle(levels, L, X[L][unknown_mask(grids[L])], B[L], 2, 2, 32)
    for l in range(L - 1, -1, -1):
        x = levels[l][1] @ x
        x = cs_vcycle(levels, l, x, B[l], 2, 2, 32)
    S.fmg(2, 2)
    got = S.psi().ravel()[unknown_mask(g)]
    np.testing.assert_allclose(got, x, rtol=0, atol=1e-11 * max(1.0, np.abs(x).max()))


@pytest.mark.parametrize("name,g", CASES)
def test_fmg_then_vcycles_reach_the_dense_newton_solution(orc, name, g):
    """FMG only changes the start of the iteration: FMG(2,2) reduces the
    residual, and V-cycles after it reach the same step solution as the dense
    Newton solve."""
    law = law_vg()
    rng = np.random.default_rng(3)
    psin = rng.uniform(-2.0, -0.2, size=g.shape)
    S = orc.Solver(workload(g, law, psin), orc.ORDER_RB)
    S.begin_step()
    ref, _ = dense_newton(orc, S, law)
    r0 = S.residual()
    S.fmg(2, 2)
    r1 = S.residual()
    assert r1 < 0.1 * r0
    orc.solve_to_floor(S, 200, 0.0)
    got = S.psi()
    assert np.abs(got - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
