"""Host-side logic of the serving engine (no GPU): default options, control
and per-request footprints, and argument errors that are rejected before any
device call."""
import ctypes as C

import pytest

import paper_2606_04292_amd as rsl
from paper_2606_04292_amd import serve
from paper_2606_04292_amd import workloads as W


def align(v):
    return (v + 255) // 256 * 256


def test_default_options():
    o = serve.engine_opts()
    assert o.struct_size == C.sizeof(serve.EngineOpts)
    assert (o.max_slots, o.max_wide_levels, o.tail_nodes) == (1024, 4, 8192)
    assert (o.nu1, o.nu2, o.nu_coarse, o.max_corrections) == (2, 2, 32, 100)
    assert o.stagnation == 1 and o.rounds_per_tick == 4 and o.use_graph == 1


def test_request_footprint_is_fine_fp64_plus_fp32_levels():
    o = serve.engine_opts()
    for g in (W.config1(257).grid, W.shrink(W.config2(), 129).grid):
        nb = serve.request_bytes(o, g)
        shapes = [g.n]
        n = list(g.n)
        while min(n) > 3:
            n = [(m - 1) // 2 + 1 for m in n]
            shapes.append(n)
        N = [int(__import__("numpy").prod(s)) for s in shapes]
        # each array is placed with 256 zeroed bytes before and after it
        want = 5 * (align(8 * N[0]) + 512) + sum(6 * (align(4 * m) + 512) for m in N)
        assert nb == want


def test_control_region_grows_with_slots():
    a = serve.control_bytes(serve.engine_opts(max_slots=16))
    b = serve.control_bytes(serve.engine_opts(max_slots=1024))
    assert 0 < a < b and a % 256 == 0 and b % 256 == 0


@pytest.mark.parametrize("bad", [dict(max_slots=0), dict(max_slots=5000),
                                 dict(max_wide_levels=9), dict(tail_nodes=8),
                                 dict(nu_coarse=0), dict(max_corrections=0),
                                 dict(tol_abs=-1.0), dict(rounds_per_tick=0)])
def test_invalid_options_are_rejected(bad):
    o = serve.engine_opts(**bad)
    out = C.c_size_t()
    assert serve._lib().rs_engine_control_bytes(C.byref(o), C.byref(out)) == rsl.RS_EINVAL


def test_requests_the_engine_cannot_hold_are_rejected():
    o = serve.engine_opts(max_wide_levels=1)
    out = C.c_size_t()
    # 513^2: three levels above 8192 nodes, more than the one wide level allowed
    d = rsl.grid_desc(W.shrink(W.config2(), 513).grid)
    assert serve._lib().rs_engine_request_bytes(C.byref(o), C.byref(d), C.byref(out)) == rsl.RS_EINVAL
    assert b"above tail_nodes" in rsl.lib().rs_last_error()
    # a 2049 x 3 x ... grid whose coarsest level exceeds tail_nodes
    g = W.GridSpec(dim=2, n=[2049, 3], L=[1.0, 1.0], face_bc=[2, 2, 1, 2],
                   face_value=[0.0, 0.0, -1.0, 0.0])
    o2 = serve.engine_opts(tail_nodes=1024)
    d2 = rsl.grid_desc(g)
    assert serve._lib().rs_engine_request_bytes(C.byref(o2), C.byref(d2), C.byref(out)) == rsl.RS_EINVAL


def test_create_checks_arguments_before_the_device():
    o = serve.engine_opts(max_slots=4)
    h = C.c_void_p()
    L = serve._lib()
    assert L.rs_engine_create(C.byref(o), C.c_void_p(256), 1 << 20, None, C.byref(h)) == rsl.RS_EINVAL
    assert L.rs_engine_create(C.byref(o), C.c_void_p(258), 1 << 20, C.c_void_p(1),
                              C.byref(h)) == rsl.RS_EINVAL
    assert L.rs_engine_create(C.byref(o), C.c_void_p(256), 512, C.c_void_p(1),
                              C.byref(h)) == rsl.RS_ENOMEM
