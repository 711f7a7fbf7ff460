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
    # 6 int32 + 8 doubles + 2 doubles, naturally aligned
    assert ctypes.sizeof(rb.Params) == 6 * 4 + 10 * 8
    assert rb.Params.vel.offset == 24


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
