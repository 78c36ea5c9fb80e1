"""Mixed precision (FP32 correction cycles inside FP64 defect correction)
against the FP64 oracle.  The FP32 cycles only ever see the correction
equation, so the converged result is the FP64 step solution: the tolerance is
the converged-parity bar, 1e-10 (normwise max-relative)."""
import sys

import numpy as np
import pytest

import oracle
import paper_2606_04292_amd as rsl
from paper_2606_04292_amd import workloads as W
from tests.test_gpu_parity import CASES, NAMES, FLOOR_CYCLES, rel, np_, say, advance

# the mixed path serves one vGM / Haverkamp / linear law per grid
MP_NAMES = [n for n in NAMES if CASES[n].soils is None and CASES[n].law.model != W.MODEL_GARDNER]

pytestmark = pytest.mark.gpu

TOL_CONV = 1e-10


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("name", MP_NAMES)
def test_mixed_converged_steps_match_fp64_oracle(torch_cuda, name):
    w = CASES[name]
    say("mixed converged", name)
    S = oracle.Solver(w, oracle.ORDER_RB)
    G = rsl.Grid(w, precision=rsl.RS_MIXED)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=FLOOR_CYCLES, tol_abs=0.0, stagnation=1,
                          mp_inner_cycles=1)
    for step in range(3):
        S.begin_step()
        oracle.solve_to_floor(S, FLOOR_CYCLES, 0.0)
        S.end_step()
        code, st = G.bdf_step(opts=opts)
        assert code == rsl.RS_OK, rsl.lib().rs_last_error()
        e = rel(np_(G.get_state()[0]), S.get(oracle.FIELD_PSI_N))
        say("  step", step, "corrections", st.cycles, "res %.2e" % st.res, "rel", e)
        assert e <= TOL_CONV
    G.close()


def test_zero_defect_is_a_fixed_point_and_outer_iteration_contracts(torch_cuda):
    """delta = 0 solves the correction equation when r = 0: once the FP64
    residual is at its floor a further correction leaves psi unchanged; before
    that, each correction reduces the FP64 residual well below 1e-10 of its
    start."""
    torch = torch_cuda
    w = W.shrink(W.config3(), 33)
    pn, pm = advance(w, 1)
    G = rsl.Grid(w, precision=rsl.RS_MIXED)
    G.set_state(torch.as_tensor(pn), torch.as_tensor(pm), nstep=1)
    G.begin_step()
    r0 = G.residual_norm()
    hist = [r0]
    for _ in range(25):
        hist.append(G.correction_cycle(1, want_norm=True))
    say("outer residuals", ["%.1e" % h for h in hist])
    assert min(hist) <= 1e-10 * r0
    before = np_(G.psi())
    G.correction_cycle(1)
    after = np_(G.psi())
    assert np.abs(after - before).max() <= 1e-13 * np.abs(before).max()
    G.close()


def test_mixed_requires_a_mixed_grid(torch_cuda):
    w = W.shrink(W.config1(), 33)
    G = rsl.Grid(w)
    G.begin_step()
    with pytest.raises(rsl.RsError) as ei:
        G.correction_cycle(1)
    assert ei.value.code == rsl.RS_ESTATE
    G.close()
