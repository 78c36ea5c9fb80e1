"""The paper's problems on the GPU, converged step by step.

* The infiltration column of section 4.1 (Haverkamp law in cm and s, 40 cm,
  psi0 = -61.5 cm, Dirichlet -20.7 cm on top, Lambda_kappa = 0.1 I, xi = 0,
  tau = 0.1 s, BDF1, V(5,5)), on 129 and 2049 nodes (the paper's N = 128 and
  N = 2048).
* The 257-node van Genuchten column with lexicographic NGS, 50 BDF1 steps of
  60 s, V(2,2), three Newton steps per cell.
* The two-layer medium of section 4.2 (257^2, FMG(10,10) start, 175 steps):
  every step converges under the stagnation stop.

The GPU sweeps in red-black order, the paper (and this column's
configuration) in lexicographic order.  The two orderings share the fixed
point: every step's unique solution of N_h(psi) = g_h (section 3.2).  So each
GPU step, iterated to the rounding floor, is compared with the oracle's
red-black and lexicographic steps iterated to theirs (normwise 1e-10), and the
GPU continues from its own state, as a user's time loop does.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_2606_04292_amd as rsl
from paper_2606_04292_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_CONV = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _run(w, steps, orderings):
    import torch
    assert torch.cuda.is_available()
    G = rsl.Grid(w)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=200, tol_abs=0.0, stagnation=1)
    refs = {o: oracle.Solver(w, o) for o in orderings}
    worst = {o: 0.0 for o in orderings}
    for step in range(steps):
        code, st = G.bdf_step(opts=opts)
        assert code == rsl.RS_OK, (step + 1, rsl.lib().rs_last_error())
        got = G.get_state()[0].cpu().numpy()
        for o, S in refs.items():
            S.begin_step()
            oracle.solve_to_floor(S, 400, 0.0)
            S.end_step()
            e = rel(got, S.get(oracle.FIELD_PSI_N))
            worst[o] = max(worst[o], e)
            assert e <= TOL_CONV, (step + 1, o, e)
            # both sides continue from the GPU's state
            S.set_state(got, S.get(oracle.FIELD_PSI_NM1), step + 1)
        if step % 10 == 0 or step == steps - 1:
            say("  step", step + 1, "cycles", st.cycles, "res %.2e" % st.res,
                " ".join("rel[%s] %.2e" % ("lex" if o == oracle.ORDER_LEX else "rb", worst[o])
                         for o in orderings))
    G.close()
    return worst


@pytest.mark.parametrize("n,steps", [(129, 20), (2049, 5)])
def test_celia_column_matches_oracle_in_both_orderings(n, steps):
    w = W.celia_column(n)
    say("celia column", n, "nodes,", steps, "steps")
    _run(w, steps, (oracle.ORDER_RB, oracle.ORDER_LEX))


def test_vg_column_fifty_steps_match_lexicographic_oracle():
    w = W.config1()
    assert w.steps == 50 and w.order == 1 and w.law.newton_iters == 3
    say("vG column 257, 50 BDF1 steps against the lexicographic oracle")
    _run(w, w.steps, (oracle.ORDER_LEX,))


def test_two_layer_medium_fmg_steps_all_converge():
    """The paper's two-layer medium (257^2, 175 steps of 0.01 day, an FMG(10,10)
    cycle then V(10,10) cycles to 1e-10 with the stagnation stop): every step
    ends RS_OK with its defect at most 1e-10.  Regression: an FMG cycle that
    raises the norm above the step's start must not be read as a stall."""
    import torch
    assert torch.cuda.is_available()
    w = W.two_layer_vg(257)
    G = rsl.Grid(w)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=200, tol_abs=1e-10,
                          stagnation=1, fmg=1)
    worst = 0.0
    for step in range(w.steps):
        code, st = G.bdf_step(opts=opts)
        assert code == rsl.RS_OK, (step + 1, rsl.lib().rs_last_error())
        assert st.res <= 1e-10, (step + 1, st.res)
        worst = max(worst, st.res)
    say("two-layer medium:", w.steps, "steps, worst final defect %.2e" % worst)
    G.close()
