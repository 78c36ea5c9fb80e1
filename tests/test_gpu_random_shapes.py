"""Seeded random grids against the oracle: anisotropic shapes of 3 to 33 nodes
per axis in one to three dimensions, random face conditions (Dirichlet with a
fixed value or with the state's values, no-flux, free drainage at the
bottom), Dirichlet rectangles on the top face, five laws (one with root
uptake); non-smooth start states on grids of at most 33 nodes per axis and
smooth random ones on the larger grids that run the multi-launch kernels.
Two FP64 V-cycles match the oracle's red-black cycles to the sweep bar, and a
mixed-precision step iterated to the rounding floor matches the oracle's step
solution to the converged bar.  Axes of 3 nodes (one interior node) and rows
whose last node ends a paired load of the grid transfers occur among them."""
import dataclasses

import numpy as np
import pytest

import oracle
import paper_2606_04292_amd as rsl
from paper_2606_04292_amd import workloads as W
from tests.test_gpu_parity import FLOOR_CYCLES, TOL_CONV, TOL_SWEEP, rel, np_, say

pytestmark = pytest.mark.gpu

NCASES = 15


def random_case(k, big=False):
    rng = np.random.default_rng(W.seed_sequence(7 if not big else 8, k))
    dim = int(rng.integers(1, 4))
    if big:
        # fine levels above the one-work-group tail: the multi-launch kernels
        sizes = {1: [4097, 8193], 2: [65, 129, 257], 3: [17, 33]}[dim]
        n = [int(rng.choice(sizes)) for _ in range(dim)]
        if dim == 3:
            n[int(rng.integers(0, 3))] = 65
    else:
        sizes = [3, 5, 9, 17, 33] if dim < 3 else [3, 5, 9, 17]
        n = [int(rng.choice(sizes)) for _ in range(dim)]
        if dim == 3 and k % 4 == 1:
            n[int(rng.integers(0, 3))] = 33
    L = [float(rng.uniform(0.5, 2.0)) for _ in range(dim)]
    bc, val = [], []
    for f in range(2 * dim):
        choices = [W.BC_NOFLUX, W.BC_DIRICHLET, W.BC_DIRICHLET_STATE]
        if f == 2 * (dim - 1):   # bottom face of the vertical (last) axis
            choices.append(W.BC_FREEDRAIN)
        bc.append(int(rng.choice(choices)))
        val.append(float(rng.uniform(-1.0, -0.1)))
    patch = {}
    if dim >= 2 and rng.random() < 0.6:
        # a Dirichlet rectangle on the top face (tangential index ranges)
        lo, hi = [], []
        for l in range(dim - 1):
            a, b = sorted(int(v) for v in rng.integers(0, n[l], size=2))
            lo.append(a)
            hi.append(b)
        lo += [0] * (2 - len(lo))
        hi += [0] * (2 - len(hi))
        patch = dict(patch_face=2 * (dim - 1) + 1, patch_lo=tuple(lo), patch_hi=tuple(hi),
                     patch_value=float(rng.uniform(-0.3, 0.0)))
    g = W.GridSpec(dim=dim, n=n, L=L, face_bc=bc, face_value=val, **patch)
    laws = [W.config1(5).law, W.config3(5).law,
            W.LawSpec(model=W.MODEL_LINEAR, theta_s=0.4, theta_r=0.1, Ks=1e-4, lin_c=0.01),
            W.config2(5).law, W.config4(5, 5).law]
    law = laws[k % len(laws)]
    law = dataclasses.replace(law, xi=max(law.xi, 1e-5))
    psi0 = -0.2 - 0.6 * rng.random(g.shape)
    if big:
        # a smooth random state: on long grids a state drawn per node makes the
        # lagged K* jump by decades between neighbours, where coarse operators
        # built from injected K* no longer represent the fine one and the FAS
        # cycle diverges (the oracle as well); a running mean over about 1/16
        # of each axis removes those jumps
        for ax in range(dim):
            wdt = max(3, g.shape[ax] // 16) | 1
            ker = np.ones(wdt) / wdt
            psi0 = np.apply_along_axis(
                lambda v: np.convolve(np.pad(v, wdt // 2, mode="edge"), ker, mode="valid"), ax, psi0)
    return W.Workload(("randbig%d_%s" if big else "random%d_%s") % (k, "x".join(map(str, n))), g, law, psi0,
                      dt=float(rng.choice([30.0, 120.0])), steps=1, order=int(rng.integers(1, 3)))


CASES = [random_case(k) for k in range(NCASES)] + [random_case(k, big=True) for k in range(6)]


def test_the_draw_covers_the_edge_shapes():
    shapes = [c.grid.n for c in CASES]
    assert {1, 2, 3} <= {len(s) for s in shapes}
    assert any(3 in s for s in shapes)
    assert any(c.grid.face_bc[2 * (c.grid.dim - 1)] == W.BC_FREEDRAIN for c in CASES)
    assert any(W.BC_DIRICHLET_STATE in c.grid.face_bc for c in CASES)
    assert any(c.grid.patch_face >= 0 and c.grid.dim == 3 for c in CASES)
    assert any(c.grid.nodes > 2049 for c in CASES)
    assert {c.grid.dim for c in CASES if c.law.sink != W.SINK_NONE} == {1, 2, 3}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("k", range(len(CASES)))
def test_random_grid_vcycles_and_mixed_step(torch_cuda, k):
    w = CASES[k]
    say("random grid", k, w.grid.n, "bc", w.grid.face_bc, "model", w.law.model)
    S = oracle.Solver(w, oracle.ORDER_RB)
    G = rsl.Grid(w)
    S.begin_step()
    G.begin_step()
    for c in range(2):
        S.vcycle()
        G.vcycle()
        e = rel(np_(G.psi()), S.psi())
        say("  V-cycle", c + 1, "rel", e)
        assert e <= TOL_SWEEP
    G.close()

    M = rsl.Grid(w, precision=rsl.RS_MIXED)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=FLOOR_CYCLES, tol_abs=0.0,
                          stagnation=1, mp_inner_cycles=1)
    oracle.solve_to_floor(S, FLOOR_CYCLES, 0.0)
    S.end_step()
    code, st = M.bdf_step(opts=opts)
    assert code == rsl.RS_OK, rsl.lib().rs_last_error()
    e = rel(np_(M.get_state()[0]), S.get(oracle.FIELD_PSI_N))
    say("  mixed step: corrections", st.cycles, "res %.2e" % st.res, "rel", e)
    assert e <= TOL_CONV
    M.close()
