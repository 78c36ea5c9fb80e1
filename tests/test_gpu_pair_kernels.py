"""The kernels that take two nodes per lane, on every level.

The colour sweep (k_sweep_pair) and the grid transfers by coarse pairs
(k_restrict_pair, k_prolong_pair) run by default on large levels only.

By default the library takes the pair sweep on levels of at least 2^22 nodes
only (the 257^3 block's finest level, the root box); RS_SWEEP=pair sends every
buffer-path level to it, so the parity cases of test_gpu_parity.py exercise
it on 1-D, 2-D and 3-D levels with ragged half-rows (odd and even n0),
Dirichlet nodes on either lane of a pair, sinks and layered media.  Each
sweep is checked against the oracle's red-black sweep from identical inputs
(1e-12, as for the one-node sweep), and against the one-node sweep
(RS_SWEEP=single), which makes the same per-node arithmetic: the compiler may
contract multiply-adds differently in the two kernels, so they agree to a few
units in the last place.  The Remark's kappa rule always takes the one-node
sweep.  RS_SWEEP32=pair does the same for the FP32 correction sweep
(k_sweep32_pair).  RS_TRANSFER=pair sends every level with parity-split rows to the pair
transfers: V-cycles (FP64 restriction and prolongation), FMG (the
interpolation that assigns) and mixed-precision steps (FP32 transfers) are
compared with the oracle as in the other parity tests.
"""
import numpy as np
import pytest

import oracle
import paper_2606_04292_amd as rsl
from tests.test_gpu_parity import CASES, FLOOR_CYCLES, NAMES, TOL_SWEEP, advance, np_, rel, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def _sweep_all_levels(torch, w, pn, pm, mode, monkeypatch):
    monkeypatch.setenv("RS_SWEEP", mode)
    S = oracle.Solver(w, oracle.ORDER_RB)
    S.set_state(pn, pm, 1)
    S.begin_step()
    G = rsl.Grid(w)
    G.set_state(torch.as_tensor(pn), torch.as_tensor(pm), nstep=1)
    G.begin_step()
    rng = np.random.default_rng(11)
    out = []
    for lev in range(S.nlev):
        kinds = S.kinds(lev).astype(bool)
        psi = S.psi(lev)
        psi = np.where(kinds, psi, psi + rng.uniform(-0.05, 0.05, size=psi.shape))
        S.set(oracle.FIELD_PSI, psi, lev)
        G.set_field(rsl.FIELD_PSI, torch.as_tensor(psi), lev)
        G.set_field(rsl.FIELD_KSTAR, torch.as_tensor(S.get(oracle.FIELD_KSTAR, lev)), lev)
        G.set_field(rsl.FIELD_G, torch.as_tensor(S.get(oracle.FIELD_G, lev)), lev)
        S.sweep(2, lev)
        G.sweep(2, lev)
        got = np_(G.psi(lev))
        out.append(got)
        e = rel(got, S.psi(lev))
        say("  %s level" % mode, lev, "shape", S.shapes[lev], "rel", e)
        assert e <= TOL_SWEEP, (mode, lev, e)
    G.close()
    return out


@pytest.mark.parametrize("name", NAMES)
def test_pair_sweep_matches_oracle_and_one_node_sweep(torch_cuda, name, monkeypatch):
    w = CASES[name]
    say("pair sweep", name, w.grid.n)
    pn, pm = advance(w, 1)
    pair = _sweep_all_levels(torch_cuda, w, pn, pm, "pair", monkeypatch)
    single = _sweep_all_levels(torch_cuda, w, pn, pm, "single", monkeypatch)
    for lev, (a, b) in enumerate(zip(pair, single)):
        assert np.abs(a - b).max() <= 8 * np.finfo(np.float64).eps * np.abs(b).max(), lev


def test_pair_sweep_vcycle_and_step(torch_cuda, monkeypatch):
    """A converged step of the shrunken drainage block with the pair sweep on
    every level equals the oracle's step (1e-10)."""
    torch = torch_cuda
    from paper_2606_04292_amd import workloads as W
    monkeypatch.setenv("RS_SWEEP", "pair")
    w = W.shrink(W.config3(), 33)
    pn, pm = advance(w, 2)
    G = rsl.Grid(w)
    G.set_state(torch.as_tensor(pn), torch.as_tensor(pm), nstep=2)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=200, tol_abs=0.0, stagnation=1)
    code, st = G.bdf_step(opts=opts)
    assert code == rsl.RS_OK, rsl.lib().rs_last_error()
    S = oracle.Solver(w, oracle.ORDER_RB)
    S.set_state(pn, pm, 2)
    S.begin_step()
    oracle.solve_to_floor(S, 400, 0.0)
    S.end_step()
    e = rel(np_(G.get_state()[0]), S.get(oracle.FIELD_PSI_N))
    say("pair sweep step: cycles", st.cycles, "rel", e)
    assert e <= 1e-10, e
    G.close()


@pytest.mark.parametrize("name", NAMES)
def test_pair_transfers_vcycle_and_fmg_parity(torch_cuda, name, monkeypatch):
    """Two V-cycles, then one FMG cycle from the same start, with the pair
    sweep and pair transfers on every level, against the oracle (1e-12)."""
    torch = torch_cuda
    monkeypatch.setenv("RS_SWEEP", "pair")
    monkeypatch.setenv("RS_TRANSFER", "pair")
    w = CASES[name]
    say("pair transfers", name, w.grid.n)
    pn, pm = advance(w, 1)
    for mode in ("vcycle", "fmg"):
        S = oracle.Solver(w, oracle.ORDER_RB)
        S.set_state(pn, pm, 1)
        S.begin_step()
        G = rsl.Grid(w)
        G.set_state(torch.as_tensor(pn), torch.as_tensor(pm), nstep=1)
        G.begin_step()
        for c in range(2 if mode == "vcycle" else 1):
            if mode == "vcycle":
                S.vcycle()
                G.vcycle()
            else:
                S.fmg()
                G.fmg()
            e = rel(np_(G.psi()), S.psi())
            say("  %s %d rel" % (mode, c), e)
            assert e <= TOL_SWEEP, (mode, c, e)
        G.close()


MP_PAIR = ["c1_col4097", "c2_slice65", "c3_block33", "c4_root33x17", "st_vg33"]


@pytest.mark.parametrize("name", [n for n in MP_PAIR if n in CASES])
def test_pair_transfers_mixed_steps(torch_cuda, name, monkeypatch):
    """Mixed-precision steps (FP32 correction cycles with the pair sweeps and
    pair transfers on every level) to the rounding floor against the FP64
    oracle (1e-10)."""
    monkeypatch.setenv("RS_SWEEP", "pair")
    monkeypatch.setenv("RS_SWEEP32", "pair")
    monkeypatch.setenv("RS_TRANSFER", "pair")
    w = CASES[name]
    say("pair transfers, mixed", name)
    S = oracle.Solver(w, oracle.ORDER_RB)
    G = rsl.Grid(w, precision=rsl.RS_MIXED)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=FLOOR_CYCLES, tol_abs=0.0,
                          stagnation=1, mp_inner_cycles=1)
    for step in range(2):
        S.begin_step()
        oracle.solve_to_floor(S, FLOOR_CYCLES, 0.0)
        S.end_step()
        code, st = G.bdf_step(opts=opts)
        assert code == rsl.RS_OK, rsl.lib().rs_last_error()
        e = rel(np_(G.get_state()[0]), S.get(oracle.FIELD_PSI_N))
        say("  step", step, "corrections", st.cycles, "rel", e)
        assert e <= 1e-10, (step, e)
    G.close()


def _slab(n, law_from, seed, smooth=False):
    """A 3-D slab whose rows have 256 s + 1 nodes (the z-marching sweep's
    shape): spacing 1/256 along every axis, Dirichlet bottom, no-flux elsewhere,
    a start state drawn per node (or a smooth one: the injected coarse K* needs
    it for the cycle to converge)."""
    from paper_2606_04292_amd import workloads as W
    h = 1.0 / 256
    g = W.GridSpec(dim=3, n=list(n), L=[(m - 1) * h for m in n],
                   face_bc=[W.BC_NOFLUX] * 4 + [W.BC_DIRICHLET, W.BC_NOFLUX],
                   face_value=[0.0] * 4 + [-1.0, 0.0])
    if smooth:
        x = np.linspace(0.0, 1.0, n[0])
        psi0 = np.broadcast_to(-1.0 + 0.4 * np.sin(np.pi * x), g.shape).copy()
    else:
        psi0 = -0.5 - 2.0 * np.random.default_rng(seed).random(g.shape)
    base = law_from()
    return W.Workload("slab_%dx%dx%d" % tuple(n), g, base.law, psi0, dt=base.dt, steps=3,
                      order=2)


SLABS = {
    "hk_257x17x9": ((257, 17, 9), "config3", 1),
    "vg_sink_257x17x9": ((257, 17, 9), "config4", 2),
    "hk_513x9x9": ((513, 9, 9), "config3", 3),
}


@pytest.mark.parametrize("zc", ["16", "4"])
@pytest.mark.parametrize("name", sorted(SLABS))
def test_zm_sweep_matches_oracle_and_other_sweeps(torch_cuda, name, zc, monkeypatch):
    """The z-marching LDS sweep (RS_SWEEP=zm) on slabs with a partial row
    stripe, partial plane chunks (RS_ZM_ZC), one or two 128-position segments
    and the node past the last segment: two sweeps on the finest level against
    the oracle (1e-12) and against the pair and one-node sweeps (8 ulp)."""
    from paper_2606_04292_amd import workloads as W
    torch = torch_cuda
    n, cfg, seed = SLABS[name]
    w = _slab(n, getattr(W, cfg), seed)
    monkeypatch.setenv("RS_ZM_ZC", zc)
    pn = w.psi0.copy()
    S = oracle.Solver(w, oracle.ORDER_RB)
    S.set_state(pn, pn, 1)
    S.begin_step()
    S.sweep(2, 0)
    ref = S.psi(0)
    got = {}
    for mode in ("zm", "pair", "single"):
        monkeypatch.setenv("RS_SWEEP", mode)
        G = rsl.Grid(w)
        G.set_state(torch.as_tensor(pn), torch.as_tensor(pn), nstep=1)
        G.begin_step()
        G.sweep(2, 0)
        got[mode] = np_(G.psi(0))
        G.close()
        e = rel(got[mode], ref)
        say("  %s %s zc %s rel %.2e" % (name, mode, zc, e))
        assert e <= TOL_SWEEP, (mode, e)
    tol = 8 * np.finfo(np.float64).eps * np.abs(ref).max()
    assert np.abs(got["zm"] - got["pair"]).max() <= tol
    assert np.abs(got["zm"] - got["single"]).max() <= tol


def test_zm_sweep_converged_steps(torch_cuda, monkeypatch):
    """Two converged BDF steps of a slab with the z-marching sweep on its
    finest level against the oracle (1e-10)."""
    from paper_2606_04292_amd import workloads as W
    monkeypatch.setenv("RS_SWEEP", "zm")
    monkeypatch.setenv("RS_ZM_ZC", "4")
    w = _slab((257, 17, 9), W.config3, 4, smooth=True)
    S = oracle.Solver(w, oracle.ORDER_RB)
    G = rsl.Grid(w)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=FLOOR_CYCLES, tol_abs=0.0,
                          stagnation=1)
    for step in range(2):
        S.begin_step()
        oracle.solve_to_floor(S, FLOOR_CYCLES, 0.0)
        S.end_step()
        code, st = G.bdf_step(opts=opts)
        assert code == rsl.RS_OK, rsl.lib().rs_last_error()
        e = rel(np_(G.get_state()[0]), S.get(oracle.FIELD_PSI_N))
        say("  zm step", step, "cycles", st.cycles, "rel", e)
        assert e <= 1e-10, (step, e)
    G.close()


FUSE_CASES = ["c1_col4097", "c2_slice65", "c3_block33", "c4_root33x17", "lay_2layer33", "st_vg33"]


@pytest.mark.parametrize("name", [n for n in FUSE_CASES if n in CASES])
def test_presmoothing_with_fused_defect_is_bitwise_the_plain_one(torch_cuda, name, monkeypatch):
    """Steps whose pre-smoothing forms the defect on the way (the last colour
    pass with k_sweep_pair_defect, the other colour with k_defect_colour)
    give bitwise the states, cycle counts and residual histories of the plain
    sweeps followed by k_residual_pair (RS_DEFECT_FUSE=0); the pair sweep is
    forced on every level so that the small cases take the fused path."""
    torch = torch_cuda
    monkeypatch.setenv("RS_SWEEP", "pair")
    w = CASES[name]
    say("fused defect", name)
    runs = {}
    for fuse in ("1", "0"):
        monkeypatch.setenv("RS_DEFECT_FUSE", fuse)
        G = rsl.Grid(w)
        opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=FLOOR_CYCLES, tol_abs=0.0,
                              stagnation=1)
        out = []
        for step in range(3):
            code, st = G.bdf_step(opts=opts)
            assert code == rsl.RS_OK, (fuse, step, rsl.lib().rs_last_error())
            out.append((st.cycles, [st.res_hist[i] for i in range(st.n_hist)],
                        np_(G.get_state()[0])))
        G.close()
        runs[fuse] = out
    for (c1, h1, p1), (c0, h0, p0) in zip(runs["1"], runs["0"]):
        assert c1 == c0 and h1 == h0
        assert np.array_equal(p1, p0)
