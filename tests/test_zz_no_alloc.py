"""rs_bdf_step_static, the step that allocates nothing, against rs_bdf_step.

Both run the same kernels on the same inputs: the static entry point keeps the
grid's workspace in the library's static device array, the grid API in a
caller workspace.  Two workloads in a row, the second smaller (the array keeps
the first one's contents), two steps each (a BDF1 start, then BDF2 with
history), every result compared with the grid API's (1e-10, and the cycle
counts must agree).
"""
import sys

import numpy as np
import pytest

import paper_2606_04292_amd as rsl
from paper_2606_04292_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_static_step_matches_grid_step_on_two_calls_in_a_row():
    import torch
    assert torch.cuda.is_available()
    opts = rsl.solve_opts(2, 2, 32, max_cycles=150, tol_abs=0.0, stagnation=1)
    for w in (W.shrink(W.config2(), 65), W.shrink(W.config3(), 17)):
        say("static step", w.name, w.grid.n)
        G = rsl.Grid(w)
        psi0 = torch.as_tensor(np.ascontiguousarray(w.psi0), device="cuda")
        prev, cur = None, psi0
        for step in range(2):
            code, st = G.bdf_step(opts=opts)
            assert code == rsl.RS_OK, rsl.lib().rs_last_error()
            ref = G.get_state()[0]
            code2, st2, out = rsl.bdf_step_static(w, cur, prev, step, opts)
            torch.cuda.synchronize()
            assert code2 == rsl.RS_OK, rsl.lib().rs_last_error()
            a, b = out.cpu().numpy(), ref.cpu().numpy()
            e = float(np.abs(a - b).max() / np.abs(b).max())
            say("  step", step + 1, "cycles", st.cycles, st2.cycles, "rel %.2e" % e,
                "bitwise" if np.array_equal(a, b) else "not bitwise")
            assert st2.cycles == st.cycles
            assert e <= 1e-10
            prev, cur = cur, out
        G.close()
