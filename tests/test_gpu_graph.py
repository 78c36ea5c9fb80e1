"""Graph replay of the coarse part of the V-cycle against plain launches.

A grid replays one captured HIP graph for the part of every V-cycle below
the finest level (and of every FP32 correction cycle), capturing it again
when the step coefficients change (the first BDF2 step after a BDF1 one).
The same kernels run in the same order either way, so a grid created with
RS_GRAPH=0 (plain launches) must give bitwise the same states, step after
step, with the program's own synchronisations between the replays.
"""
import os
import sys

import numpy as np
import pytest

import paper_2606_04292_amd as rsl
from paper_2606_04292_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _grid(w, precision, graph):
    old = os.environ.get("RS_GRAPH")
    os.environ["RS_GRAPH"] = "1" if graph else "0"
    try:
        return rsl.Grid(w, precision=precision)
    finally:
        if old is None:
            del os.environ["RS_GRAPH"]
        else:
            os.environ["RS_GRAPH"] = old


@pytest.mark.parametrize("name,w", [("block33", W.shrink(W.config3(), 33)),
                                    ("slice65", W.shrink(W.config2(), 65)),
                                    ("root33", W.shrink(W.config4(), 33))])
@pytest.mark.parametrize("precision", [rsl.RS_FP64, rsl.RS_MIXED], ids=["fp64", "mixed"])
def test_graph_replay_equals_plain_launches(name, w, precision):
    import torch
    assert torch.cuda.is_available()
    say("graph vs plain", name, precision)
    A = _grid(w, precision, True)
    B = _grid(w, precision, False)
    opts = rsl.solve_opts(w.nu1, w.nu2, w.nu_coarse, max_cycles=150, tol_abs=0.0, stagnation=1)
    for step in range(4):
        ca, sa = A.bdf_step(opts=opts)
        cb, sb = B.bdf_step(opts=opts)
        assert ca == cb == rsl.RS_OK
        torch.cuda.synchronize()
        pa, pb = A.get_state()[0].cpu().numpy(), B.get_state()[0].cpu().numpy()
        say("  step", step + 1, "cycles", sa.cycles, sb.cycles,
            "max diff %.3e" % float(np.abs(pa - pb).max()))
        assert sa.cycles == sb.cycles
        assert sa.cell_updates == sb.cell_updates
        assert np.array_equal(pa, pb)
    # an explicit V-cycle after the steps replays the same graph
    A.begin_step()
    B.begin_step()
    ra = A.vcycle(want_norm=True)
    rb = B.vcycle(want_norm=True)
    assert ra == rb
    A.close()
    B.close()
