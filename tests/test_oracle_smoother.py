"""Pins of the oracle's pointwise solve and NGS sweeps (section 3.1:
eq. iterative, eq. point-update, the contraction theorem and its Remark)."""
import dataclasses

import numpy as np
import pytest
from scipy.linalg import solve_triangular

from paper_2606_04292_amd import workloads as W

RNG = np.random.default_rng(99)


def law_vg(**kw):
    base = dict(model=W.MODEL_VGM, theta_s=0.43, theta_r=0.05, Ks=1e-5, vg_alpha=3.6, vg_n=1.56)
    base.update(kw)
    return W.LawSpec(**base)


def workload(g, law, psi0, ks=None, order=1, dt=60.0):
    return W.Workload("t", g, law, np.ascontiguousarray(psi0, dtype=np.float64), dt=dt, steps=1,
                      order=order, Ks_field=ks)


def bisect(F, lo, hi, steps=200):
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        if F(mid) > 0:
            hi = mid
        else:
            lo = mid
    return 0.5 * (lo + hi)


LAWS = [law_vg(), W.config3(5).law, W.config1(5).law,
        W.config4(5, 5).law]


@pytest.mark.parametrize("k", range(len(LAWS)))
def test_local_newton_converges_to_bisection_root(orc, k):
    """eq. point-update: the left side is strictly increasing, so the root is
    unique; the safeguarded Newton iteration reaches the 200-step bisection
    root (the bracket of the reading is also checked to hold it)."""
    law = LAWS[k]
    th, dth, _, fa, dfa = orc.law_fns(law)
    for _ in range(25):
        a = 10 ** RNG.uniform(-4, -1)
        c = 10 ** RNG.uniform(-9, 0)
        beta = 1e-6 * RNG.uniform(0, 1) if law.sink else 0.0
        target = -10 ** RNG.uniform(-2, 0.5)
        f = a * th(target) + c * target + beta * fa(target)
        F = lambda x: a * th(x) + c * x + beta * fa(x) - f
        lo = (f - a * law.theta_s - beta) / c
        hi = (f - a * law.theta_r) / c
        assert F(lo) <= 0 <= F(hi)
        root = bisect(F, lo, hi)
        x0 = RNG.uniform(-3.0, 0.5)
        x = orc.local_solve(law, a, beta, c, f, x0, 60)
        assert abs(x - root) <= 1e-12 * max(1.0, abs(root))
        # three steps land inside the bracket and do not increase |F| beyond F(x0)'s bracket
        x3 = orc.local_solve(law, a, beta, c, f, x0, 3)
        assert lo <= x3 <= hi


@pytest.mark.parametrize("k", range(len(LAWS)))
def test_local_solve_keeps_a_converged_cell(orc, k):
    """A cell already at its root stays there (a step below rounding resolution
    must not trigger the bisection safeguard)."""
    law = LAWS[k]
    th, _, _, fa, _ = orc.law_fns(law)
    for _ in range(50):
        a = 10 ** RNG.uniform(-4, -1)
        c = 10 ** RNG.uniform(-9, -3)
        target = -10 ** RNG.uniform(-2, 0.7)
        f = a * th(target) + c * target
        x = orc.local_solve(law, a, 0.0, c, f, target, 60)
        x3 = orc.local_solve(law, a, 0.0, c, f, x, 3)
        assert abs(x3 - x) <= 4 * np.spacing(abs(x))


@pytest.mark.parametrize("k", range(len(LAWS)))
def test_early_newton_stop_changes_the_solve_only_at_rounding(orc, k):
    """The early stop after a Newton step of at most newton_tol |x| (the
    reading of the open Newton step count): from starts at every distance from the
    root, the result equals that of all the steps to within rounding (the
    steps left out are quadratically small), converged starts take one
    evaluation, and far starts still reach the bisection root."""
    law = dataclasses.replace(LAWS[k], newton_tol=1e-10)
    exact = dataclasses.replace(law, newton_tol=0.0)
    th, dth, _, fa, dfa = orc.law_fns(law)
    stopped = 0
    for _ in range(200):
        a = 10 ** RNG.uniform(-4, -1)
        c = 10 ** RNG.uniform(-9, -2)
        beta = 1e-6 * RNG.uniform(0, 1) if law.sink else 0.0
        target = -10 ** RNG.uniform(-2, 0.5)
        f = a * th(target) + c * target + beta * fa(target)
        x0 = target * (1.0 + 10 ** RNG.uniform(-14, -1) * RNG.choice([-1.0, 1.0]))
        for iters in (3, 6):
            x, n = orc.local_solve(law, a, beta, c, f, x0, iters, evals=True)
            xe, ne = orc.local_solve(exact, a, beta, c, f, x0, iters, evals=True)
            # rounding floor of the root: F's rounding error over F'
            noise = 8 * np.finfo(float).eps * (a * th(xe) + c * abs(xe) + abs(f)) / (
                a * dth(xe) + c + beta * dfa(xe))
            assert abs(x - xe) <= 1e-14 * abs(xe) + noise
            assert n <= ne <= iters
            stopped += n < ne
        x, n = orc.local_solve(law, a, beta, c, f, target, 3, evals=True)
        xr, nr = orc.local_solve(law, a, beta, c, f, x, 3, evals=True)
        floor = 8 * np.finfo(float).eps * (a * th(x) + c * abs(x) + abs(f)) / (
            a * dth(x) + c + beta * dfa(x))
        assert nr == 1 and abs(xr - x) <= 4 * np.spacing(abs(x)) + floor
        far, nf = orc.local_solve(law, a, beta, c, f, -2.5, 60, evals=True)
        assert nf < 60 and abs(far - target) <= 1e-12 * max(1.0, abs(target))
    assert stopped > 100


def linear_setup(orc, dim, n, ordering, rule=W.KAPPA_REL):
    bcs = [W.BC_NOFLUX] * (2 * dim)
    bcs[2 * (dim - 1)] = W.BC_DIRICHLET
    bcs[1] = W.BC_DIRICHLET
    g = W.GridSpec(dim=dim, n=[n] * dim, L=[1.0] * dim, face_bc=bcs, face_value=[0.0] * (2 * dim))
    law = W.LawSpec(model=W.MODEL_LINEAR, theta_s=0.4, theta_r=0.1, Ks=1e-3, lin_c=0.02,
                    xi=1e-4, kappa_rule=rule, kappa=0.2, newton_iters=2)
    psin = RNG.uniform(-1.0, 1.0, size=g.shape)
    S = orc.Solver(workload(g, law, psin), ordering)
    S.begin_step()
    kinds = S.kinds().astype(bool)
    psi = np.where(kinds, 0.0, RNG.uniform(-1.0, 1.0, size=g.shape))
    S.set(orc.FIELD_PSI, psi)
    return S, law, kinds, psi


@pytest.mark.parametrize("dim,n", [(1, 17), (2, 9), (3, 5)])
@pytest.mark.parametrize("ordering", ["lex", "rb"])
def test_linear_law_sweep_equals_textbook_splitting(orc, dim, n, ordering):
    """With theta affine the pointwise equation is linear, Newton is exact in
    one step, and one NGS sweep is the splitting iteration of eq. iterative:
    (a c I + xi I + L + D_kappa) x_new = g - a theta_r + (Lambda_kappa - U) x_old,
    solved here by forward substitution in the sweep's ordering."""
    o = orc.ORDER_LEX if ordering == "lex" else orc.ORDER_RB
    S, law, kinds, psi = linear_setup(orc, dim, n, o)
    M, kap, unk = S.dense_M()
    g = S.get(orc.FIELD_G).ravel()[unk]
    x_old = psi.ravel()[unk]
    if o == orc.ORDER_RB:
        shape = S.shapes[0]
        col = np.array([sum(np.unravel_index(i, shape)) % 2 for i in unk])
        perm = np.concatenate([np.where(col == 0)[0], np.where(col == 1)[0]])
    else:
        perm = np.arange(len(unk))
    Mp = M[np.ix_(perm, perm)]
    kp = kap[perm]
    a = S.a
    A = np.tril(Mp) + np.diag(a * law.lin_c + law.xi + kp)
    rhs = g[perm] - a * law.theta_r + kp * x_old[perm] - np.triu(Mp, 1) @ x_old[perm]
    x_new_p = solve_triangular(A, rhs, lower=True)
    x_new = np.empty_like(x_new_p)
    x_new[perm] = x_new_p
    S.sweep(1)
    got = S.psi().ravel()[unk]
    np.testing.assert_allclose(got, x_new, rtol=1e-12, atol=1e-12 * np.abs(x_new).max())


def nonlinear_case(orc, n=17, rule=W.KAPPA_REMARK, iters=40, xi=0.0):
    g = W.GridSpec(dim=2, n=[n, n], L=[1.0, 1.0],
                   face_bc=[W.BC_NOFLUX, W.BC_NOFLUX, W.BC_DIRICHLET, W.BC_DIRICHLET],
                   face_value=[0, 0, -1.0, -0.2])
    law = law_vg(kappa_rule=rule, newton_iters=iters, xi=xi)
    ks = np.exp(RNG.normal(np.log(1e-5), 0.7, size=g.shape))
    psin = np.full(g.shape, -1.0)
    return workload(g, law, psin, ks, dt=600.0)


def test_contraction_bound_of_the_theorem(orc):
    """Theorem (L-infinity contraction) with the Remark's kappa (equal row sums
    of U_kappa, so xi >= 0 suffices): each sweep reduces ||psi - psi*||_inf at
    least by lambda(U_k) / (theta_0/tau + xi + lambda(U_k)), theta_0 the least
    theta' over the values the iterates and the solution take."""
    w = nonlinear_case(orc)
    S = orc.Solver(w, orc.ORDER_LEX)
    S.begin_step()
    for _ in range(40):
        S.vcycle(3, 3)
    assert S.residual() < 1e-16
    exact = S.psi().copy()
    S.begin_step()                         # restart from psi^n
    lam = S.lambdaU()
    it = [S.psi().copy()]
    for _ in range(6):
        S.sweep(1)
        it.append(S.psi().copy())
    lo = min(x.min() for x in it + [exact])
    hi = max(x.max() for x in it + [exact])
    _, dth, _, _, _ = orc.law_fns(w.law)
    theta0 = min(dth(x) for x in np.linspace(lo, min(hi, -1e-12), 2000))
    bound = lam / (S.a * theta0 + w.law.xi + lam)
    assert bound < 1.0
    errs = [np.abs(x - exact).max() for x in it]
    for e0, e1 in zip(errs, errs[1:]):
        assert e1 <= bound * e0 * (1 + 1e-9) + 1e-14


def test_order_preservation(orc):
    """The splitting has m_ij >= 0, kappa >= 0 and an increasing pointwise
    equation, so one sweep maps ordered iterates to ordered iterates."""
    w = nonlinear_case(orc, rule=W.KAPPA_REL)
    S = orc.Solver(w, orc.ORDER_RB)
    S.begin_step()
    kinds = S.kinds().astype(bool)
    base = S.psi().copy()
    lo = np.where(kinds, base, base + RNG.uniform(-0.5, 0.0, size=base.shape))
    hi = np.where(kinds, base, lo + RNG.uniform(0.0, 0.5, size=base.shape))
    S.set(orc.FIELD_PSI, lo)
    S.sweep(1)
    a = S.psi().copy()
    S.set(orc.FIELD_PSI, hi)
    S.sweep(1)
    b = S.psi().copy()
    assert np.all(a <= b + 1e-15)


@pytest.mark.parametrize("ordering", ["lex", "rb"])
def test_solution_is_a_fixed_point_of_the_sweep(orc, ordering):
    o = orc.ORDER_LEX if ordering == "lex" else orc.ORDER_RB
    w = nonlinear_case(orc, rule=W.KAPPA_REL, iters=3)
    S = orc.Solver(w, o)
    S.begin_step()
    for _ in range(40):
        S.vcycle()
    assert S.residual() < 1e-16
    x = S.psi().copy()
    S.sweep(2)
    assert np.abs(S.psi() - x).max() <= 1e-13


@pytest.mark.parametrize("k", range(len(LAWS)))
def test_saturated_cell_root_on_the_bracket_end(orc, k):
    """For psi >= 0 theta = theta_s and F is linear, with its root exactly at the
    lower end of the initial bracket; the safeguarded Newton must return that
    root (one exact Newton step), not a bisection point."""
    law = LAWS[k]
    for _ in range(50):
        a = 10 ** RNG.uniform(-4, -1)
        c = 10 ** RNG.uniform(-6, 0)
        root = RNG.uniform(0.0, 2.0)
        f = a * law.theta_s + c * root
        x0 = RNG.uniform(-1.0, 3.0) if k != 3 else RNG.uniform(0.0, 3.0)
        x = orc.local_solve(law, a, 0.0, c, f, abs(x0) + 1e-3, 3)
        exact = (f - a * law.theta_s) / c
        cond = np.finfo(float).eps * (abs(f) + a * law.theta_s + c * abs(x0)) / c
        assert abs(x - exact) <= 16 * cond + 1e-15
