"""The C-ABI library loads and exports every entry point declared in
include/richards.h; host-only logic (workspace planning, descriptor
validation) works without a GPU."""
import ctypes as C
import glob
import os
import re

import pytest

import paper_2606_04292_amd as rsl
from paper_2606_04292_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names.update(re.findall(r"\b(rs_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_method_calls():
    names = declared_functions()
    for must in ("rs_create_grid", "rs_set_constitutive", "rs_bdf_step", "rs_vcycle",
                 "rs_residual_norm"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(rsl.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(rsl.EXPORTS) == declared_functions()


def _desc(g):
    return rsl.grid_desc(g)


def test_workspace_bytes_counts_every_level():
    g = W.config3().grid
    nb = rsl.workspace_bytes(g)
    N0 = 257 ** 3
    # five FP64 arrays on every level + history + Ks field >= 8 fine arrays
    assert nb >= 8 * 8 * N0
    assert nb < 8 * 8 * N0 * 1.3
    assert nb % 256 == 0


@pytest.mark.parametrize("bad", [
    dict(n=[256]), dict(n=[2]), dict(dim=4), dict(face_bc=[0, 1]), dict(face_bc=[1, 3]),
    dict(L=[-1.0]),
])
def test_invalid_descriptors_are_rejected(bad):
    g = W.config1(33).grid
    for k, v in bad.items():
        if k != "dim":
            setattr(g, k, v)
    d = _desc(g)
    if "dim" in bad:
        d.dim = bad["dim"]
    out = C.c_size_t()
    code = rsl.lib().rs_workspace_bytes(C.byref(d), rsl.RS_FP64, C.byref(out))
    assert code == rsl.RS_EINVAL
    assert rsl.lib().rs_last_error()


def test_create_rejects_small_workspace_before_touching_the_device():
    g = W.config1(33).grid
    h = C.c_void_p()
    code = rsl.lib().rs_create_grid(C.byref(_desc(g)), rsl.RS_FP64, C.c_void_p(256), 512,
                                    None, C.byref(h))
    assert code == rsl.RS_ENOMEM
    code = rsl.lib().rs_create_grid(C.byref(_desc(g)), rsl.RS_FP64, C.c_void_p(258), 1 << 30,
                                    None, C.byref(h))
    assert code == rsl.RS_EINVAL


def test_struct_sizes_match_the_header():
    g = W.config1(33).grid
    d = _desc(g)
    d.struct_size = 8
    out = C.c_size_t()
    assert rsl.lib().rs_workspace_bytes(C.byref(d), rsl.RS_FP64, C.byref(out)) == rsl.RS_EINVAL


def test_static_step_refuses_a_grid_beyond_its_array_before_touching_the_device():
    """rs_bdf_step_static checks the grid's FP64 workspace against its static
    array (RS_STATIC_WORKSPACE_BYTES) before any device call."""
    w = W.shrink(W.config3(), 129)
    assert rsl.workspace_bytes(w.grid) > rsl.RS_STATIC_WORKSPACE_BYTES
    c, keep = rsl.constitutive(w.law)
    st = rsl.StepStats()
    st.struct_size = C.sizeof(rsl.StepStats)
    o = rsl.solve_opts()
    code = rsl.lib().rs_bdf_step_static(C.byref(_desc(w.grid)), C.byref(c), C.c_void_p(256), None,
                                        0, w.dt, w.order, C.byref(o), C.c_void_p(256),
                                        C.byref(st), None)
    assert code == rsl.RS_ENOMEM
    assert b"static scratch" in rsl.lib().rs_last_error()
    code = rsl.lib().rs_bdf_step_static(C.byref(_desc(w.grid)), C.byref(c), None, None, 0, w.dt,
                                        w.order, C.byref(o), C.c_void_p(256), C.byref(st), None)
    assert code == rsl.RS_EINVAL
    del keep


def test_static_workspace_size_matches_the_header():
    import re
    with open(os.path.join(ROOT, "include", "richards.h")) as f:
        m = re.search(r"#define RS_STATIC_WORKSPACE_BYTES \((\d+)u << (\d+)\)", f.read())
    assert m and int(m.group(1)) << int(m.group(2)) == rsl.RS_STATIC_WORKSPACE_BYTES
