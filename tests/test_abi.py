"""The C-ABI library loads on a machine without a GPU and exports every
function that include/rbfsl.h declares (no compute calls here)."""
import ctypes
import os
import re

import paper_1804_01609_amd as rb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rbfsl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbfsl_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    assert set(names) == set(rb.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(rb.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_params_struct_layout_matches_header():
    # 8 int32 + 8 doubles + 2 doubles, naturally aligned
    assert ctypes.sizeof(rb.Params) == 8 * 4 + 10 * 8
    assert rb.Params.vel.offset == 32


def test_invalid_arguments_are_rejected_without_a_device():
    L = rb.lib()
    assert L.rbfsl_max_system() >= 184
    assert L.rbfsl_strerror(rb.RBFSL_E_SINGULAR) == b"singular stencil system"
    out = ctypes.c_void_p()
    p = rb.make_params(31, 3, 2)
    # null nodes, N < n, k > L: all rejected on the host before any HIP call
    assert L.rbfsl_create(None, 10, 0, ctypes.byref(p), None, ctypes.byref(out)) == rb.RBFSL_E_INVAL
    import numpy as np
    X = np.zeros((10, 3))
    assert L.rbfsl_create(X.ctypes.data_as(ctypes.c_void_p), 10, 0, ctypes.byref(p), None,
                          ctypes.byref(out)) == rb.RBFSL_E_INVAL
    p2 = rb.make_params(31, 2, 3)
    X = np.zeros((100, 3))
    assert L.rbfsl_create(X.ctypes.data_as(ctypes.c_void_p), 100, 0, ctypes.byref(p2), None,
                          ctypes.byref(out)) == rb.RBFSL_E_INVAL
    assert not out.value


def test_pu_arguments_are_rejected_without_a_device():
    import numpy as np
    L = rb.lib()
    out = ctypes.c_void_p()
    X = np.zeros((100, 3))
    C = np.zeros((10, 3))
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    good = rb.make_params(31, 3, 2, rb.STENCIL_PU)
    # RBF-PU needs its own stencil mode; plain create refuses it
    assert L.rbfsl_create(vp(X), 100, 0, ctypes.byref(good), None, ctypes.byref(out)) == rb.RBFSL_E_INVAL
    p0 = rb.make_params(31, 3, 2, 0)
    assert L.rbfsl_create_pu(vp(X), 100, 0, vp(C), 10, 0.5, ctypes.byref(p0), None,
                             ctypes.byref(out)) == rb.RBFSL_E_INVAL
    for R in (0.0, -1.0, 3.0, float("nan")):
        assert L.rbfsl_create_pu(vp(X), 100, 0, vp(C), 10, R, ctypes.byref(good), None,
                                 ctypes.byref(out)) == rb.RBFSL_E_INVAL
    assert L.rbfsl_create_pu(vp(X), 100, 0, None, 10, 0.5, ctypes.byref(good), None,
                             ctypes.byref(out)) == rb.RBFSL_E_INVAL
    assert L.rbfsl_create_pu(vp(X), 100, 0, vp(C), 0, 0.5, ctypes.byref(good), None,
                             ctypes.byref(out)) == rb.RBFSL_E_INVAL
    assert L.rbfsl_pu_info(None, None, None, None, None) == rb.RBFSL_E_INVAL
    assert not out.value
    assert rb.pu_radius(84, 23042) == 2.0 * np.sqrt(84 / 23042) and rb.pu_count(2.5, 84, 23042) == 686


def _c_layout(exprs):
    """sizeof/offsetof values of header types, from a tiny C program built with gcc."""
    import subprocess
    import tempfile
    src = '#include <stddef.h>\n#include <stdio.h>\n#include "rbfsl.h"\nint main(void){\n'
    for e in exprs:
        src += f'  printf("%zu\\n", (size_t)({e}));\n'
    src += "  return 0;\n}\n"
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split()
    return [int(v) for v in out]


def test_struct_layouts_match_the_c_compiler():
    exprs = ["sizeof(rbfsl_params)", "offsetof(rbfsl_params, vel)", "offsetof(rbfsl_params, dt)",
             "sizeof(rbfsl_pool_config)", "sizeof(rbfsl_pool_stats)", "offsetof(rbfsl_pool_stats, blocks)",
             "sizeof(rbfsl_tune_result)", "sizeof(rbfsl_request)", "offsetof(rbfsl_request, params)",
             "offsetof(rbfsl_request, q_out)", "sizeof(rbfsl_request_result)",
             "offsetof(rbfsl_request_result, steps)"]
    want = [ctypes.sizeof(rb.Params), rb.Params.vel.offset, rb.Params.dt.offset,
            ctypes.sizeof(rb.PoolConfig), ctypes.sizeof(rb.PoolStats), rb.PoolStats.blocks.offset,
            ctypes.sizeof(rb.TuneResult), ctypes.sizeof(rb.Request), rb.Request.params.offset,
            rb.Request.q_out.offset, ctypes.sizeof(rb.RequestResult), rb.RequestResult.steps.offset]
    assert _c_layout(exprs) == want


def test_pool_host_checks_without_a_device():
    L = rb.lib()
    out = ctypes.c_void_p()
    assert L.rbfsl_pool_create(None, ctypes.byref(out)) == rb.RBFSL_E_INVAL
    bad = rb.PoolConfig(0, 1, 0)
    assert L.rbfsl_pool_create(ctypes.byref(bad), ctypes.byref(out)) == rb.RBFSL_E_INVAL
    assert not out.value
    assert L.rbfsl_strerror(rb.RBFSL_E_BUDGET) == b"no free run slot or HBM budget"
    p = rb.make_params(84, 5, 3, n_tracers=2)
    small = rb.pool_run_bytes(10000, p, 100)
    large = rb.pool_run_bytes(40000, p, 100)
    # nodes, sorted nodes, q ping-pong, staging: at least 104 bytes per node with two tracers
    assert 104 * 10000 <= small < large
    assert rb.pool_run_bytes(0, p, 100) == -1
    vs = rb.pool_variants()
    assert max(v["mcap"] for v in vs) >= 184
    assert {v["waves"] for v in vs} >= {1, 2, 4}
    for v in vs:
        assert v["waves"] * v["group"] in (3, 4, 8, 16)
