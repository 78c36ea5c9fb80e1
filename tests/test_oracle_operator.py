"""Pins of the oracle's discrete operator (section 2: eq. discrete-strong, the
matrix M, eq. Nh-def) against the textbook Laplacian, exact steady states, the
conservation identity and the structural statements of section 3 (the
Proposition and the Lemma)."""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2606_04292_amd import workloads as W

RNG = np.random.default_rng(1234)


def grid(dim, n, bcs, vals=None, L=None):
    return W.GridSpec(dim=dim, n=[n] * dim, L=L or [1.0] * dim, face_bc=list(bcs),
                      face_value=list(vals or [0.0] * (2 * dim)))


def law_vg(**kw):
    base = dict(model=W.MODEL_VGM, theta_s=0.43, theta_r=0.05, Ks=1e-5, vg_alpha=3.6, vg_n=1.56)
    base.update(kw)
    return W.LawSpec(**base)


def workload(g, law, psi0, ks=None, order=1, dt=30.0):
    return W.Workload("t", g, law, np.ascontiguousarray(psi0, dtype=np.float64), dt=dt, steps=1,
                      order=order, Ks_field=ks)


def textbook_1d(n, h, lo_bc, hi_bc):
    """(-1, 2, -1)/h^2 on the unknown nodes of one axis: Dirichlet ends are
    removed; a no-flux end uses the mirrored ghost node (row 2, -2)."""
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    if lo_bc == W.BC_NOFLUX:
        A[0, 1] = -2.0
    if hi_bc == W.BC_NOFLUX:
        A[n - 1, n - 2] = -2.0
    keep = [i for i in range(n)
            if not ((i == 0 and lo_bc == W.BC_DIRICHLET) or (i == n - 1 and hi_bc == W.BC_DIRICHLET))]
    A = A.tocsr()[keep][:, keep] / h ** 2
    return A


def textbook_laplacian(g):
    mats = [textbook_1d(g.n[l], g.L[l] / (g.n[l] - 1), g.face_bc[2 * l], g.face_bc[2 * l + 1])
            for l in range(g.dim)]
    eyes = [sp.identity(m.shape[0]) for m in mats]
    total = None
    for l in range(g.dim):
        # flattening has axis 0 fastest: kron(..., axis1, axis0)
        term = None
        for a in reversed(range(g.dim)):
            f = mats[a] if a == l else eyes[a]
            term = f if term is None else sp.kron(term, f)
        total = term if total is None else total + term
    return total.toarray()


CASES = [
    (1, 9, [W.BC_DIRICHLET, W.BC_DIRICHLET]),
    (1, 9, [W.BC_NOFLUX, W.BC_DIRICHLET]),
    (2, 9, [W.BC_NOFLUX, W.BC_NOFLUX, W.BC_DIRICHLET, W.BC_DIRICHLET]),
    (2, 5, [W.BC_DIRICHLET, W.BC_NOFLUX, W.BC_NOFLUX, W.BC_DIRICHLET]),
    (3, 5, [W.BC_NOFLUX, W.BC_NOFLUX, W.BC_NOFLUX, W.BC_NOFLUX, W.BC_DIRICHLET, W.BC_NOFLUX]),
    (3, 5, [W.BC_DIRICHLET] * 6),
]


@pytest.mark.parametrize("dim,n,bcs", CASES)
def test_constant_K_gives_textbook_laplacian(orc, dim, n, bcs):
    """With K constant (the test-only LINEAR law) M is Ks times the textbook
    (2d+1)-point Laplacian with mirrored ghosts at no-flux faces."""
    g = grid(dim, n, bcs)
    law = W.LawSpec(model=W.MODEL_LINEAR, theta_s=0.4, theta_r=0.1, Ks=2.5e-3, lin_c=0.01)
    S = orc.Solver(workload(g, law, np.zeros(g.shape)), orc.ORDER_LEX)
    S.begin_step()
    M, _, _ = S.dense_M()
    A = textbook_laplacian(g) * law.Ks
    assert M.shape == A.shape
    np.testing.assert_allclose(M, A, rtol=1e-13, atol=1e-13 * np.abs(A).max())


@pytest.mark.parametrize("dim,n,bcs", CASES)
def test_proposition_rows_and_conservative_symmetry(orc, dim, n, bcs):
    """Proposition of section 3 (reading: sum_{j!=i} m_ij <= m_ii, with
    equality on rows without Dirichlet neighbours); m_ii > 0, m_ij >= 0; and
    V M is symmetric (control-volume weights), i.e. fluxes are conservative."""
    g = grid(dim, n, bcs)
    ks = np.exp(RNG.normal(np.log(1e-5), 1.0, size=g.shape))
    psi0 = RNG.uniform(-2.0, -0.1, size=g.shape)
    S = orc.Solver(workload(g, law_vg(), psi0, ks), orc.ORDER_RB)
    S.begin_step()
    M, kap, unk = S.dense_M()
    kinds = S.kinds().ravel()
    off = M - np.diag(np.diag(M))
    assert np.all(np.diag(M) > 0) and np.all(off <= 0)
    rows = M.sum(axis=1)
    assert np.all(rows >= -1e-12 * np.diag(M))
    # rows without a Dirichlet neighbour sum to zero
    shape = S.shapes[0]
    for r, i in enumerate(unk):
        ii = np.unravel_index(i, shape)
        has_dir = False
        for ax in range(dim):
            for s in (-1, 1):
                jj = list(ii)
                jj[ax] += s
                if 0 <= jj[ax] < shape[ax] and kinds[np.ravel_multi_index(jj, shape)]:
                    has_dir = True
        if not has_dir:
            assert abs(rows[r]) <= 1e-12 * M[r, r]
        else:
            assert rows[r] > 0
    # control volumes V_i = prod_l w_l h_l
    V = np.ones(len(unk))
    for r, i in enumerate(unk):
        ii = np.unravel_index(i, shape)
        for ax in range(dim):
            w = 0.5 if ii[ax] in (0, shape[ax] - 1) else 1.0
            V[r] *= w / (shape[ax] - 1)
    VM = V[:, None] * M
    np.testing.assert_allclose(VM, VM.T, rtol=1e-13, atol=1e-13 * np.abs(VM).max())
    assert np.all(kap > 0)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("order", [1, 2])
def test_hydrostatic_state_is_exact_steady_state(orc, dim, order):
    """psi = c - z with a consistent Dirichlet bottom and no-flux elsewhere has
    zero total-head gradient, so N(psi^n) = g for any K field, xi and order."""
    n = 9
    bcs = [W.BC_NOFLUX] * (2 * dim)
    vals = [0.0] * (2 * dim)
    bcs[2 * (dim - 1)] = W.BC_DIRICHLET
    c = -0.3
    vals[2 * (dim - 1)] = c
    g = grid(dim, n, bcs, vals)
    z = W.elevation(g)
    ks = np.exp(RNG.normal(np.log(1e-5), 1.0, size=g.shape))
    law = law_vg(xi=3e-4)
    S = orc.Solver(workload(g, law, c - z, ks, order=order), orc.ORDER_RB)
    S.set_state(c - z, c - z, nstep=1)
    S.begin_step()
    r = S.residual()
    scale = S.a * law.theta_s
    assert r <= 1e-13 * scale


def test_unit_gradient_free_drainage_is_steady(orc):
    """Uniform psi with uniform K: the flux is K (unit gradient, downward) on
    every face; a top Dirichlet face at the same psi feeds it and the
    free-drainage bottom lets it out, so the state is steady."""
    c = -0.7
    g = grid(2, 17, [W.BC_NOFLUX, W.BC_NOFLUX, W.BC_FREEDRAIN, W.BC_DIRICHLET], [0, 0, 0, c])
    law = law_vg()
    S = orc.Solver(workload(g, law, np.full(g.shape, c)), orc.ORDER_RB)
    S.begin_step()
    _, d = S.residual(want_vector=True)
    assert np.abs(d).max() <= 1e-13 * S.a * law.theta_s
    # and without the drainage term the bottom row would be out of balance
    g2 = dataclasses.replace(g, face_bc=[W.BC_NOFLUX, W.BC_NOFLUX, W.BC_NOFLUX, W.BC_DIRICHLET])
    S2 = orc.Solver(workload(g2, law, np.full(g.shape, c)), orc.ORDER_RB)
    S2.begin_step()
    assert S2.residual() > 1e-3 * law.Ks


def _sink_numpy(law, g, psi):
    """Feddes-exponential sink written out from its definition (input side)."""
    if law.sink != W.SINK_FEDDES_EXP:
        return np.zeros_like(psi)
    nz = g.n[-1]
    hz = g.L[-1] / (nz - 1)
    zk = np.arange(nz) * hz
    wk = np.ones(nz)
    wk[0] = wk[-1] = 0.5
    Z = np.sum(wk * hz * np.exp(-(g.L[-1] - zk) / law.root_len))
    z = W.elevation(g)
    beta = law.Tp * np.exp(-(g.L[-1] - z) / law.root_len) / Z
    a = np.where(psi < law.h4, 0.0,
        np.where(psi < law.h3, (psi - law.h4) / (law.h3 - law.h4),
        np.where(psi < law.h2, 1.0,
        np.where(psi < law.h1, (law.h1 - psi) / (law.h1 - law.h2), 0.0))))
    return beta * a


@pytest.mark.parametrize("dim", [2, 3])
def test_mass_balance_identity_for_arbitrary_iterate(orc, dim):
    """Conservation (section 2: conservative flux form): for ANY iterate psi,
    sum_i V_i (N(psi) - g)_i equals the storage/sink/xi terms plus the fluxes
    through Dirichlet faces and the free-drainage outflow, because interior
    face fluxes cancel pairwise.  Terms are summed here from raw arrays."""
    n = 9
    bcs = [W.BC_NOFLUX] * (2 * dim)
    bcs[2 * (dim - 1)] = W.BC_FREEDRAIN
    bcs[2 * (dim - 1) + 1] = W.BC_NOFLUX
    g = W.GridSpec(dim=dim, n=[n] * dim, L=[1.0] * (dim - 1) + [0.5], face_bc=bcs,
                   face_value=[0.0] * (2 * dim), patch_face=2 * dim - 1,
                   patch_lo=(2, 3), patch_hi=(5, 6), patch_value=-0.05)
    law = law_vg(xi=2e-5, sink=W.SINK_FEDDES_EXP, Tp=5e-3 / 86400, root_len=0.2)
    ks = np.exp(RNG.normal(np.log(1e-5), 1.0, size=g.shape))
    psin = RNG.uniform(-2.0, -0.2, size=g.shape)
    psinm1 = psin + RNG.uniform(-0.1, 0.1, size=g.shape)
    S = orc.Solver(workload(g, law, psin, ks, order=2, dt=60.0), orc.ORDER_RB)
    S.set_state(psin, psinm1, nstep=1)
    S.begin_step()
    kinds = S.kinds().astype(bool)
    psi = S.psi().copy()
    psi[~kinds] = RNG.uniform(-3.0, -0.05, size=(~kinds).sum())
    S.set(orc.FIELD_PSI, psi)
    _, r = S.residual(want_vector=True)
    K = S.get(orc.FIELD_KSTAR)
    th = np.vectorize(orc.law_fns(law)[0])
    a = S.a
    H = (4 * th(psin) - th(psinm1)) / (2 * 60.0)
    shape = S.shapes[0]
    hs = [g.L[l] / (g.n[l] - 1) for l in range(dim)]
    z = W.elevation(g)
    phi = psi + z
    unk = ~kinds
    # control volumes and face areas (axis l is numpy axis dim-1-l)
    wl = []
    for l in range(dim):
        w = np.ones(g.n[l])
        w[0] = w[-1] = 0.5
        sh = [1] * dim
        sh[dim - 1 - l] = g.n[l]
        wl.append(w.reshape(sh))
    V = np.ones(shape)
    for l in range(dim):
        V = V * wl[l] * hs[l]
    storage = a * th(psi) - H + _sink_numpy(law, g, psi) + law.xi * (psi - psin)
    lhs = np.sum((V * storage)[unk])
    flux = 0.0
    for l in range(dim):
        ax = dim - 1 - l
        area = np.ones(shape)
        for m in range(dim):
            if m != l:
                area = area * wl[m] * hs[m]
        for s in (-1, 1):
            nb_phi = np.roll(phi, -s, axis=ax)
            nb_K = np.roll(K, -s, axis=ax)
            nb_kind = np.roll(kinds, -s, axis=ax)
            valid = np.ones(shape, dtype=bool)
            idx = [slice(None)] * dim
            idx[ax] = -1 if s == 1 else 0
            valid[tuple(idx)] = False
            sel = unk & valid & nb_kind
            kf = 0.5 * (K + nb_K)
            flux += np.sum((area * kf * (phi - nb_phi) / hs[l])[sel])
    bottom = [slice(None)] * dim
    bottom[0] = 0
    area_z = np.ones(shape)
    for m in range(dim - 1):
        area_z = area_z * wl[m] * hs[m]
    fd = np.sum((area_z * K)[tuple(bottom)][unk[tuple(bottom)]])
    total = lhs + flux + fd + np.sum((V * r)[unk])
    scale = np.sum(np.abs(V * storage)[unk]) + abs(flux) + fd
    assert abs(total) <= 1e-12 * scale


@pytest.mark.parametrize("rule", [W.KAPPA_CONST, W.KAPPA_REL, W.KAPPA_REMARK])
def test_lemma_bounds(orc, rule):
    """Lemma (splitting with diagonal shift): ||alpha I - beta U_k|| equals
    alpha + beta max-rowsum(U_k) and ||(alpha Lambda_mu + beta (L + D_k))^-1||
    is bounded by 1/(alpha min(mu) + beta min-rowsum(U_k))."""
    g = grid(2, 5, [W.BC_NOFLUX, W.BC_DIRICHLET, W.BC_NOFLUX, W.BC_DIRICHLET])
    ks = np.exp(RNG.normal(np.log(1e-5), 1.0, size=g.shape))
    psi0 = RNG.uniform(-2.0, -0.1, size=g.shape)
    S = orc.Solver(workload(g, law_vg(kappa_rule=rule, kappa=0.3 if rule != W.KAPPA_CONST else 5.0),
                            psi0, ks), orc.ORDER_LEX)
    S.begin_step()
    M, kap, _ = S.dense_M()
    L = np.tril(M, -1)
    U = np.triu(M, 1)
    D = np.diag(np.diag(M))
    Uk = U - np.diag(kap)
    Dk = D + np.diag(kap)
    rows_Uk = np.abs(Uk).sum(axis=1)
    inf = lambda A: np.abs(A).sum(axis=1).max()
    for _ in range(5):
        al, be = RNG.uniform(0.1, 10.0, size=2)
        mu = RNG.uniform(0.5, 3.0, size=M.shape[0])
        assert inf(al * np.eye(M.shape[0]) - be * Uk) == pytest.approx(al + be * rows_Uk.max(), rel=1e-13)
        Ainv = np.linalg.inv(al * np.diag(mu) + be * (L + Dk))
        assert inf(Ainv) <= 1.0 / (al * mu.min() + be * rows_Uk.min()) * (1 + 1e-12)
    if rule == W.KAPPA_REMARK:
        # the first choice of the Remark equalises the row sums of U_kappa
        assert rows_Uk.max() == pytest.approx(rows_Uk.min(), rel=1e-12)
        assert rows_Uk.max() == pytest.approx(S.lambdaU(), rel=1e-12)
