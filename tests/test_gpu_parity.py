"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (normwise max-relative, ||a - b||_inf / ||b||_inf):
  * step set-up (K*, g), one red-black sweep, one V-cycle: 1e-12;
  * converged solutions after several time steps: 1e-10.
Both sides evaluate the same formulas in FP64 with different libm
implementations and summation orders, so per-element differences are a few
ulps amplified by the local conditioning of the pointwise solve.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import paper_2606_04292_amd as rsl
from paper_2606_04292_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_SWEEP = 1e-12
TOL_CONV = 1e-10
# Cycle budget for iterating to the rounding floor.  The REMARK shift gives
# black rows kappa = max row sum of U over the whole grid, which on a drying
# Haverkamp block (K* over many decades) contracts at 0.93-0.99 per cycle:
# thousands of cycles on 17^3.
FLOOR_CYCLES = 8000


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def np_(t):
    return t.detach().cpu().numpy()


def cases():
    out = {
        "c1_col257": W.config1(),
        "c2_slice65": W.shrink(W.config2(), 65),
        "c3_block33": W.shrink(W.config3(), 33),
        "c4_root33x17": W.shrink(W.config4(), 33),
    }
    w = W.shrink(W.config3(), 17)
    out["c3_remark17"] = dataclasses.replace(
        w, law=dataclasses.replace(w.law, kappa_rule=W.KAPPA_REMARK, xi=1e-6))
    w = W.shrink(W.config2(), 33)
    out["c2_const_xi33"] = dataclasses.replace(
        w, law=dataclasses.replace(w.law, kappa_rule=W.KAPPA_CONST, kappa=1e-4, xi=1e-5))
    # root uptake in a 1-D column: the vertical axis is the row axis, so every
    # node carries its own root density
    for n in (65, 4097):
        g1 = W.GridSpec(dim=1, n=[n], L=[0.5], face_bc=[W.BC_NOFLUX, W.BC_NOFLUX], face_value=[0.0, 0.0])
        out["c4_col_sink%d" % n] = W.Workload("root_column%d" % n, g1, W.config4(5, 5).law,
                                              np.full(g1.shape, -1.0), dt=300.0, steps=3, order=2)
    # a column longer than the one-work-group tail (2049 nodes): its fine
    # levels run the multi-launch 1-D kernels
    out["c1_col4097"] = W.config1(4097)
    # coarse K* by full weighting: a smooth 3-D block, and a column whose start
    # state is drawn per node (K* jumps by decades between neighbours; the
    # injected cycle diverges there, the averaged one converges)
    w = W.shrink(W.config3(), 33)
    out["c3_block33_fw"] = dataclasses.replace(w, name="block33_fw",
                                               law=dataclasses.replace(w.law, coarse_k=W.COARSE_FW))
    g1 = W.GridSpec(dim=1, n=[1025], L=[0.5], face_bc=[W.BC_NOFLUX, W.BC_DIRICHLET], face_value=[0.0, -0.5])
    rough = -0.2 - 0.6 * np.random.default_rng(W.seed_sequence(9, 0)).random(g1.shape)
    out["rough_col1025_fw"] = W.Workload("rough_column1025_fw", g1,
                                         dataclasses.replace(W.config1(5).law, xi=1e-5,
                                                             coarse_k=W.COARSE_FW),
                                         rough, dt=120.0, steps=3, order=2)
    # layered media and the Gardner law (section 4)
    out["lay_celia129"] = W.celia_composite(129)
    out["lay_2layer33"] = W.two_layer_vg(33)
    out["gd_col129"] = dataclasses.replace(W.celia_column(129), name="gardner_col129",
                                           law=W.celia_soils()[0])
    # non-uniform boundary data through the state: the 2-D Gardner infiltration,
    # and a vGM slice whose top head varies along the face
    out["gd_2d33"] = W.gardner_2d(33)
    w = W.shrink(W.config2(), 33)
    bc = list(w.grid.face_bc)
    bc[3] = W.BC_DIRICHLET_STATE
    psi0 = w.psi0.copy()
    psi0[-1, :] = -0.5 + 0.4 * np.sin(np.pi * np.linspace(0.0, 1.0, 33))
    out["st_vg33"] = dataclasses.replace(w, name="state_top_vg33", psi0=psi0,
                                         grid=dataclasses.replace(w.grid, face_bc=bc))
    return out


CASES = cases()
NAMES = sorted(CASES)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def advance(w, steps):
    """State after `steps` converged oracle steps (same start for both sides)."""
    S = oracle.Solver(w, oracle.ORDER_RB)
    for _ in range(steps):
        S.begin_step()
        oracle.solve_to_floor(S, FLOOR_CYCLES, 0.0)
        S.end_step()
    return S.get(oracle.FIELD_PSI_N), S.get(oracle.FIELD_PSI_NM1)


@pytest.mark.parametrize("name", NAMES)
def test_setup_parity(torch_cuda, name):
    torch = torch_cuda
    w = CASES[name]
    say("setup parity", name, w.grid.n)
    pn, pm = advance(w, 1)
    G = rsl.Grid(w)
    G.set_state(torch.as_tensor(pn), torch.as_tensor(pm), nstep=1)
    G.begin_step()
    S = oracle.Solver(w, oracle.ORDER_RB)
    S.set_state(pn, pm, 1)
    S.begin_step()
    for lev in range(S.nlev):
        Kg = np_(G.field(rsl.FIELD_KSTAR, lev))
        Ko = S.get(oracle.FIELD_KSTAR, lev)
        assert np.all(np.abs(Kg - Ko) <= 1e-12 * np.abs(Ko)), (lev, rel(Kg, Ko))
    assert rel(np_(G.field(rsl.FIELD_G)), S.get(oracle.FIELD_G)) <= TOL_SWEEP
    assert rel(np_(G.psi()), S.psi()) == 0.0
    G.close()


@pytest.mark.parametrize("name", NAMES)
def test_single_sweep_parity_from_identical_inputs(torch_cuda, name):
    """One red-black sweep on identical psi, K*, g (the oracle's) on every level."""
    torch = torch_cuda
    w = CASES[name]
    say("sweep parity", name)
    pn, pm = advance(w, 1)
    S = oracle.Solver(w, oracle.ORDER_RB)
    S.set_state(pn, pm, 1)
    S.begin_step()
    G = rsl.Grid(w)
    G.set_state(torch.as_tensor(pn), torch.as_tensor(pm), nstep=1)
    G.begin_step()
    rng = np.random.default_rng(5)
    for lev in range(S.nlev):
        kinds = S.kinds(lev).astype(bool)
        psi = S.psi(lev)
        psi = np.where(kinds, psi, psi + rng.uniform(-0.05, 0.05, size=psi.shape))
        S.set(oracle.FIELD_PSI, psi, lev)
        G.set_field(rsl.FIELD_PSI, torch.as_tensor(psi), lev)
        G.set_field(rsl.FIELD_KSTAR, torch.as_tensor(S.get(oracle.FIELD_KSTAR, lev)), lev)
        G.set_field(rsl.FIELD_G, torch.as_tensor(S.get(oracle.FIELD_G, lev)), lev)
        S.sweep(1, lev)
        G.sweep(1, lev)
        e = rel(np_(G.psi(lev)), S.psi(lev))
        say("  level", lev, "shape", S.shapes[lev], "rel", e)
        assert e <= TOL_SWEEP, (lev, e)
    G.close()


@pytest.mark.parametrize("name", NAMES)
def test_vcycle_parity(torch_cuda, name):
    torch = torch_cuda
    w = CASES[name]
    say("vcycle parity", name)
    pn, pm = advance(w, 1)
    S = oracle.Solver(w, oracle.ORDER_RB)
    S.set_state(pn, pm, 1)
    S.begin_step()
    G = rsl.Grid(w)
    G.set_state(torch.as_tensor(pn), torch.as_tensor(pm), nstep=1)
    G.begin_step()
    for c in range(2):
        S.vcycle()
        G.vcycle()
        e = rel(np_(G.psi()), S.psi())
        say("  cycle", c, "rel", e)
        assert e <= TOL_SWEEP, (c, e)
    rg = G.residual_norm()
    ro, do = S.residual(want_vector=True)
    assert abs(rg - ro) <= 1e-9 * max(ro, 1e-30) + 1e-13 * S.a
    # the defect vector itself, node by node (the fine-level defect kernel,
    # also where the cycle's coarse levels run in one work-group); each entry
    # is a difference of terms as large as g and a psi, rounded differently
    # on the two sides
    dg = np_(G.residual())
    scale = np.abs(S.get(oracle.FIELD_G)).max() + S.a * np.abs(S.psi()).max()
    assert np.abs(dg - do).max() <= 1e-9 * max(ro, 1e-30) + 1e-11 * scale


@pytest.mark.parametrize("name", NAMES)
def test_converged_steps_parity(torch_cuda, name):
    """Three full BDF steps, each iterated to the rounding floor on both sides."""
    w = CASES[name]
    say("converged parity", name)
    S = oracle.Solver(w, oracle.ORDER_RB)
    G = rsl.Grid(w)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=FLOOR_CYCLES, tol_abs=0.0, stagnation=1)
    for step in range(3):
        S.begin_step()
        oracle.solve_to_floor(S, FLOOR_CYCLES, 0.0)
        S.end_step()
        code, st = G.bdf_step(opts=opts)
        assert code == rsl.RS_OK, rsl.lib().rs_last_error()
        pg = np_(G.get_state()[0])
        po = S.get(oracle.FIELD_PSI_N)
        e = rel(pg, po)
        say("  step", step, "cycles", st.cycles, "res %.2e" % st.res, "rel", e)
        assert e <= TOL_CONV
    G.close()


@pytest.mark.parametrize("name", NAMES)
def test_fmg_cycle_parity(torch_cuda, name):
    """One FMG(nu1, nu2) cycle from the same step set-up, then one V-cycle:
    GPU against the oracle's FMG (normwise 1e-12)."""
    w = CASES[name]
    say("fmg parity", name)
    S = oracle.Solver(w, oracle.ORDER_RB)
    G = rsl.Grid(w)
    S.begin_step()
    G.begin_step()
    S.fmg()
    G.fmg()
    e = rel(np_(G.psi()), S.psi())
    say("  after FMG rel", e)
    assert e <= TOL_SWEEP
    S.vcycle()
    G.vcycle()
    e = rel(np_(G.psi()), S.psi())
    say("  after V-cycle rel", e)
    assert e <= TOL_SWEEP
    G.close()


@pytest.mark.parametrize("name", ["c1_col257", "c2_slice65", "c3_block33", "lay_2layer33"])
def test_converged_steps_with_fmg_start(torch_cuda, name):
    """Steps that start with one FMG cycle reach the oracle's step solutions."""
    w = CASES[name]
    say("fmg converged", name)
    S = oracle.Solver(w, oracle.ORDER_RB)
    G = rsl.Grid(w)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=FLOOR_CYCLES, tol_abs=0.0,
                          stagnation=1, fmg=1)
    for step in range(3):
        S.begin_step()
        oracle.solve_to_floor(S, FLOOR_CYCLES, 0.0)
        S.end_step()
        code, st = G.bdf_step(opts=opts)
        assert code == rsl.RS_OK, rsl.lib().rs_last_error()
        e = rel(np_(G.get_state()[0]), S.get(oracle.FIELD_PSI_N))
        say("  step", step, "cycles", st.cycles, "rel", e)
        assert e <= TOL_CONV
    G.close()


@pytest.mark.parametrize("cfg", ["block257", "rootbox257x129", "twolayer257"])
def test_full_size_sampled_sweep_and_setup(torch_cuda, cfg):
    """The 257^3 Haverkamp block (the benchmark's launch shape) and the
    257x257x129 root-uptake box at full size: set-up (K*, g) and one red-black
    sweep checked on sampled nodes that the oracle computes one by one from
    the GPU's own inputs (red from the pre-sweep state, black from the GPU's
    red values)."""
    torch = torch_cuda
    w = {"block257": W.config3, "rootbox257x129": W.config4, "twolayer257": W.two_layer_vg}[cfg]()
    say("full-size sampled", cfg, w.grid.n)
    G = rsl.Grid(w)
    G.begin_step()
    G.vcycle()      # move away from the initial state
    psi0 = np_(G.psi())
    G.sweep(1)
    psi1 = np_(G.psi())
    K = np_(G.field(rsl.FIELD_KSTAR))
    g = np_(G.field(rsl.FIELD_G))
    S = oracle.Solver(w, oracle.ORDER_RB)
    S.begin_step()
    Ko = S.get(oracle.FIELD_KSTAR)
    go = S.get(oracle.FIELD_G)
    assert np.all(np.abs(K - Ko) <= 1e-12 * np.abs(Ko))
    assert rel(g, go) <= TOL_SWEEP
    S.set(oracle.FIELD_KSTAR, K)
    S.set(oracle.FIELD_G, g)
    rng = np.random.default_rng(11)
    n0, n1, n2 = (list(w.grid.n) + [1, 1])[:3]
    idx = rng.integers(0, n0 * n1 * n2, size=6000)
    i0 = idx % n0
    i1 = (idx // n0) % n1
    i2 = idx // (n0 * n1)
    colour = (i0 + i1 + i2) % 2
    red = idx[colour == 0].astype(np.int32)
    black = idx[colour == 1].astype(np.int32)
    S.set(oracle.FIELD_PSI, psi0)
    red_o = S.update_points(red)
    mix = psi0.copy().ravel()
    cz = (np.indices(psi0.shape).sum(axis=0) % 2 == 0).ravel()
    mix[cz] = psi1.ravel()[cz]
    S.set(oracle.FIELD_PSI, mix.reshape(psi0.shape))
    black_o = S.update_points(black)
    scale = np.abs(psi1).max()
    e_red = np.abs(psi1.ravel()[red] - red_o).max() / scale
    e_black = np.abs(psi1.ravel()[black] - black_o).max() / scale
    say("  sampled red rel", e_red, "black rel", e_black)
    assert e_red <= TOL_SWEEP and e_black <= TOL_SWEEP
    G.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_slice_converged_steps(torch_cuda, precision):
    """The 513^2 slice with its lognormal Ks field at full size: two BDF steps
    iterated to the rounding floor on both sides (FP64, and FP32 correction
    cycles inside FP64 defect correction) against the FP64 oracle."""
    w = W.config2()
    say("full-size slice", precision, w.grid.n)
    S = oracle.Solver(w, oracle.ORDER_RB)
    G = rsl.Grid(w, precision=rsl.RS_FP64 if precision == "fp64" else rsl.RS_MIXED)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=FLOOR_CYCLES, tol_abs=0.0,
                          stagnation=1)
    for step in range(2):
        S.begin_step()
        oracle.solve_to_floor(S, FLOOR_CYCLES, 0.0)
        S.end_step()
        code, st = G.bdf_step(opts=opts)
        assert code == rsl.RS_OK, rsl.lib().rs_last_error()
        e = rel(np_(G.get_state()[0]), S.get(oracle.FIELD_PSI_N))
        say("  step", step, "cycles", st.cycles, "res %.2e" % st.res, "rel", e)
        assert e <= TOL_CONV
    G.close()


def test_edge_grids(torch_cuda):
    """Degenerate and ragged grids: one unknown (3 nodes), 1-D with free
    drainage, a 2-D grid whose rows are not a multiple of the tile width, the
    test-only linear law, and the smallest 3-D grid."""
    torch = torch_cuda
    grids = [
        W.GridSpec(dim=1, n=[3], L=[1.0], face_bc=[1, 1], face_value=[-1.0, -0.2]),
        W.GridSpec(dim=1, n=[129], L=[1.0], face_bc=[3, 1], face_value=[0.0, -0.3]),
        W.GridSpec(dim=2, n=[129, 17], L=[2.0, 1.0], face_bc=[2, 2, 1, 2], face_value=[0, 0, -1, 0],
                   patch_face=3, patch_lo=(60, 0), patch_hi=(70, 0), patch_value=0.0),
        W.GridSpec(dim=3, n=[3, 3, 3], L=[1, 1, 1], face_bc=[2, 2, 2, 2, 1, 2],
                   face_value=[0, 0, 0, 0, -0.5, 0]),
        W.GridSpec(dim=3, n=[9, 17, 5], L=[1, 2, 0.5], face_bc=[1, 2, 2, 1, 3, 2],
                   face_value=[-0.4, 0, 0, -0.8, 0, 0]),
    ]
    laws = [W.config1(5).law, W.config2(5).law, W.config3(5).law,
            W.LawSpec(model=W.MODEL_LINEAR, theta_s=0.4, theta_r=0.1, Ks=1e-4, lin_c=0.01),
            W.config4(5, 5).law]
    for k, g in enumerate(grids):
        law = laws[k % len(laws)]
        w = W.Workload("edge%d" % k, g, law, np.full(g.shape, -0.7), dt=60.0, steps=2, order=2)
        say("edge grid", k, g.n)
        S = oracle.Solver(w, oracle.ORDER_RB)
        G = rsl.Grid(w)
        S.begin_step()
        G.begin_step()
        for _ in range(2):
            S.vcycle()
            G.vcycle()
        assert rel(np_(G.psi()), S.psi()) <= TOL_SWEEP
        G.close()


def test_error_paths(torch_cuda):
    torch = torch_cuda
    w = W.shrink(W.config3(), 17)
    G = rsl.Grid(w)
    with pytest.raises(rsl.RsError) as ei:
        G.vcycle()
    assert ei.value.code == rsl.RS_ESTATE
    # not converged: tol 0, one cycle -> RS_ENOTCONV and the history is kept
    before = np_(G.get_state()[0])
    code, st = G.bdf_step(opts=rsl.solve_opts(max_cycles=1, tol_abs=0.0))
    assert code == rsl.RS_ENOTCONV and st.cycles == 1
    a, _, nstep, _ = G.get_state()
    assert nstep == 0 and np.array_equal(np_(a), before)
    # non-finite state -> RS_ENONFINITE from the residual norm
    bad = torch.as_tensor(w.psi0.copy())
    bad.view(-1)[1000] = float("nan")
    G.set_state(bad)
    G.begin_step()
    with pytest.raises(rsl.RsError) as ei:
        G.residual_norm()
    assert ei.value.code == rsl.RS_ENONFINITE
    G.close()


def test_repeatable_and_restartable(torch_cuda):
    """Red-black sweeps are race-free: two runs are bitwise equal; and
    4 steps = 2 steps + state round trip through a new grid + 2 steps."""
    torch = torch_cuda
    w = W.shrink(W.config2(), 65)
    opts = rsl.solve_opts(max_cycles=30, tol_abs=1e-13)
    runs = []
    for _ in range(2):
        G = rsl.Grid(w)
        for _ in range(4):
            code, _ = G.bdf_step(opts=opts)
            assert code == rsl.RS_OK
        runs.append(np_(G.get_state()[0]))
        G.close()
    assert np.array_equal(runs[0], runs[1])
    G = rsl.Grid(w)
    for _ in range(2):
        assert G.bdf_step(opts=opts)[0] == rsl.RS_OK
    a, b, n, t = G.get_state()
    H = rsl.Grid(w)
    H.set_state(a, b, n, t)
    for _ in range(2):
        assert H.bdf_step(opts=opts)[0] == rsl.RS_OK
    assert np.array_equal(np_(H.get_state()[0]), runs[0])


def test_fused_sweep_is_independent_of_the_tiling(torch_cuda):
    """The fused red-black sweep gives bitwise the same result for different
    lane grids and chunk depths (each node is written once, by its owner, from
    the same inputs), agrees with the two-pass sweep to rounding, and matches
    the oracle on a level that uses it."""
    import os
    torch = torch_cuda
    w = W.shrink(W.config3(), 65)
    pn, pm = advance(w, 1)
    outs = []
    old = os.environ.get("RS_FUSED_TILE")
    os.environ["RS_SWEEP"] = "fused"
    try:
        for tile in ("16,16,32", "8,4,3", "10,7,64", "3,3,1", "32,16,5"):
            os.environ["RS_FUSED_TILE"] = tile
            G = rsl.Grid(w)
            G.set_state(torch.as_tensor(pn), torch.as_tensor(pm), nstep=1)
            G.begin_step()
            G.sweep(2)
            outs.append(np_(G.psi()))
            G.close()
    finally:
        os.environ.pop("RS_SWEEP", None)
        if old is None:
            os.environ.pop("RS_FUSED_TILE", None)
        else:
            os.environ["RS_FUSED_TILE"] = old
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    # the two-pass sweep makes the same per-node arithmetic on the same values;
    # the compiler may fuse multiply-adds differently in the two kernels, so
    # they agree to rounding (a few units in the last place)
    G = rsl.Grid(w)
    G.set_state(torch.as_tensor(pn), torch.as_tensor(pm), nstep=1)
    G.begin_step()
    G.sweep(2)
    two = np_(G.psi())
    G.close()
    assert np.abs(two - outs[0]).max() <= 8 * np.finfo(np.float64).eps * np.abs(two).max()
    S = oracle.Solver(w, oracle.ORDER_RB)
    S.set_state(pn, pm, 1)
    S.begin_step()
    S.sweep(2)
    assert rel(outs[0], S.psi()) <= TOL_SWEEP


def test_a_diverging_cycle_is_not_reported_as_converged(torch_cuda):
    """With the stagnation stop on, a step whose cycle diverges (injected K* on
    a column whose start is drawn per node) ends as RS_ENOTCONV, leaving the
    history; with averaged coarse K* the same step reaches the rounding floor
    and returns RS_OK."""
    w = CASES["rough_col1025_fw"]
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=400, tol_abs=0.0, stagnation=1)
    G = rsl.Grid(dataclasses.replace(w, law=dataclasses.replace(w.law, coarse_k=W.COARSE_INJECT)))
    code, st = G.bdf_step(opts=opts)
    say("injected K*: code", code, "cycles", st.cycles, "res0 %.2e res %.2e" % (st.res0, st.res))
    assert code == rsl.RS_ENOTCONV
    assert G.get_state()[2] == 0          # history not advanced
    G.close()
    G = rsl.Grid(w)
    code, st = G.bdf_step(opts=opts)
    say("averaged K*: code", code, "cycles", st.cycles, "res0 %.2e res %.2e" % (st.res0, st.res))
    assert code == rsl.RS_OK and st.res < 1e-10 * st.res0
    G.close()


def test_layered_media_errors(torch_cuda):
    """Layered media and the Gardner law run on FP64 grids; a soil index beyond
    the table is refused; the serving engine refuses both."""
    w = W.two_layer_vg(17)
    with pytest.raises(rsl.RsError) as ei:
        rsl.Grid(w, precision=rsl.RS_MIXED)
    assert ei.value.code == rsl.RS_EINVAL
    g = W.celia_soils()[0]
    with pytest.raises(rsl.RsError) as ei:
        rsl.Grid(dataclasses.replace(W.celia_column(65), law=g), precision=rsl.RS_MIXED)
    assert ei.value.code == rsl.RS_EINVAL
    bad = w.soil_id.copy()
    bad[3, 4] = 2
    with pytest.raises(rsl.RsError) as ei:
        rsl.Grid(dataclasses.replace(w, soil_id=bad))
    assert ei.value.code == rsl.RS_EINVAL
    with pytest.raises(rsl.RsError) as ei:
        rsl.Grid(dataclasses.replace(w, Ks_field=np.full(w.grid.shape, 1.0)))
    assert ei.value.code == rsl.RS_EINVAL
    from paper_2606_04292_amd import serve
    opts = serve.engine_opts(max_slots=4)
    E = serve.Engine(serve.control_bytes(opts) + (64 << 20), opts)
    for bad_w in (w, dataclasses.replace(W.celia_column(65), law=g), CASES["st_vg33"]):
        with pytest.raises(rsl.RsError) as ei:
            E.submit(bad_w)
        assert ei.value.code == rsl.RS_EINVAL
    E.close()
