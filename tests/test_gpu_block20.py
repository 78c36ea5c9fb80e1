"""The 3-D drainage block through its whole time loop on the GPU.

The block (Haverkamp law in cm, hydrostatic saturated start, bottom head
-1 m, BDF2 with tau = 120 s and xi = 1e-4) drains through 20 steps; from the
second step the cells next to the bottom are over-drained by the lagged
conductivity and a drying front with K* jumping by six decades between
neighbouring nodes moves up the block, where the V-cycle contracts most
slowly.  Every step is iterated to the rounding floor on both sides (the
library's stop: two cycles without a new minimum, accepted within 16 ulp of
the defect's term scale) and the GPU state is compared with the oracle's after
every step (normwise 1e-10), in FP64 and in mixed precision.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2606_04292_amd as rsl
from paper_2606_04292_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_CONV = 1e-10
BUDGET = 150


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def oracle_states():
    """The oracle's state after each of the 20 steps, per grid size."""
    out = {}
    for n in (33, 65):
        w = W.shrink(W.config3(), n)
        S = oracle.Solver(w, oracle.ORDER_RB)
        states, cycles = [], []
        for _ in range(w.steps):
            S.begin_step()
            hist = oracle.solve_to_floor(S, BUDGET, 0.0)
            S.end_step()
            states.append(S.get(oracle.FIELD_PSI_N))
            cycles.append(len(hist) - 1)
        say("oracle block %d^3 cycles per step:" % n, cycles)
        out[n] = states
    return out


@pytest.mark.parametrize("precision", [rsl.RS_FP64, rsl.RS_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("n", [33, 65])
def test_block_twenty_steps_match_oracle(oracle_states, n, precision):
    import torch
    assert torch.cuda.is_available()
    w = W.shrink(W.config3(), n)
    say("block %d^3, 20 steps, precision %d" % (n, precision))
    G = rsl.Grid(w, precision=precision)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=BUDGET, tol_abs=0.0,
                          stagnation=1)
    worst = 0.0
    for step in range(w.steps):
        code, st = G.bdf_step(opts=opts)
        assert code == rsl.RS_OK, (step + 1, st.cycles, st.res, rsl.lib().rs_last_error())
        got = G.get_state()[0].cpu().numpy()
        e = rel(got, oracle_states[n][step])
        worst = max(worst, e)
        say("  step", step + 1, "cycles", st.cycles, "res %.2e" % st.res, "rel %.2e" % e)
        assert e <= TOL_CONV, (step + 1, e)
    say("  worst rel", worst)
    G.close()
