"""rbfsl_weights_noalloc (the entry point that allocates nothing, for callers
that cannot allocate device memory) against rbfsl_weights on the same inputs:
two calls in a row, the second smaller, each bit for bit equal to the
allocating entry point (which the parity tests check against the oracle);
inputs beyond its fixed scratch and host arrays are refused before anything
runs.  Device memory for the test comes from the HIP runtime the library is
bound to (whichever copy the process loaded first)."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import paper_1804_01609_amd as rb
from paper_1804_01609_amd import workloads as W

pytestmark = pytest.mark.gpu

H2D, D2H = 1, 2


def say(*a):
    print(*a, file=sys.stderr, flush=True)


class Dev:
    """Device buffers through the process's HIP runtime (freed at close)."""

    def __init__(self):
        rb.lib()  # the library binds the runtime; this gets the same one by soname
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        self.hip.hipFree.argtypes = [ctypes.c_void_p]
        self.bufs = []

    def put(self, a):
        a = np.ascontiguousarray(a)
        p = ctypes.c_void_p()
        assert self.hip.hipMalloc(ctypes.byref(p), max(a.nbytes, 8)) == 0
        self.bufs.append(p)
        assert self.hip.hipMemcpy(p, a.ctypes.data_as(ctypes.c_void_p), a.nbytes, H2D) == 0
        return p.value

    def get(self, ptr, shape, dtype):
        out = np.empty(shape, dtype=dtype)
        assert self.hip.hipDeviceSynchronize() == 0
        assert self.hip.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(ptr), out.nbytes, D2H) == 0
        return out

    def close(self):
        for p in self.bufs:
            self.hip.hipFree(p)
        self.bufs = []


def test_noalloc_weights_equal_allocating_entry_point_twice():
    d = Dev()
    try:
        # the second call is smaller than the first
        for N, n, L, k, count in [(40962, 84, 5, 3, 3000), (10242, 31, 3, 2, 700)]:
            say(f"[noalloc] N={N} n={n} L={L} k={k} count={count}")
            X = W.fibonacci_nodes(N)
            Qp = W.random_sphere_points(count, seed=N + count)
            idx, d2 = oracle.knn(X, Qp, n)
            idx = idx.astype(np.int32)
            s2 = d2[:, -1].copy()
            ref_w, ref_st = rb.weights(X, idx, Qp, s2, Qp, n, L, k)
            w = d.put(np.full((count, n), np.nan))
            st = d.put(np.full(count, 77, dtype=np.int32))
            code = rb.weights_noalloc_ptr(d.put(X), N, d.put(idx), d.put(Qp), d.put(s2), d.put(Qp), count,
                                          n, L, k, w, st)
            assert code == rb.RBFSL_OK
            wg = d.get(w, (count, n), np.float64)
            sg = d.get(st, (count,), np.int32)
            assert np.array_equal(sg, ref_st) and np.all(sg == 0)
            assert np.abs(wg - ref_w).max() <= 1e-11 * np.abs(ref_w).max()
            assert np.array_equal(wg, ref_w)
    finally:
        d.close()


def test_noalloc_refuses_inputs_beyond_its_scratch_and_host_arrays():
    cap = rb.weights_noalloc_capacity()
    assert cap == 1 << 21
    d = Dev()
    try:
        n, N = 4, 1024
        X = d.put(W.fibonacci_nodes(N))
        count = (cap - N) // 2 + 1  # N + 2 count just above the capacity
        idx = d.put(np.zeros((count, n), dtype=np.int32))
        pts = d.put(np.zeros((count, 3)))
        s2 = d.put(np.ones(count))
        w = d.put(np.zeros((count, n)))
        assert rb.weights_noalloc_ptr(X, N, idx, pts, s2, pts, count, n, 1, 1, w) == rb.RBFSL_E_CAPACITY
        # a host array where device memory is required
        host = np.zeros((N, 3))
        assert rb.weights_noalloc_ptr(host.ctypes.data, N, idx, pts, s2, pts, 10, n, 1, 1, w) == rb.RBFSL_E_INVAL
    finally:
        d.close()
