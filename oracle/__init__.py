"""ctypes wrapper of the plain FP64 CPU oracle (``oracle.c``).

Test infrastructure only: the tests, the smoke check and the CPU-baseline leg
of the benchmark are the only callers.  Nothing here imports the product
package, and the product package never imports this module.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

ORC_OK, ORC_SINGULAR, ORC_NONFINITE, ORC_INVAL = 0, 1, 2, 3
VEL_ZERO, VEL_SOLID, VEL_DEFORM, VEL_NL2010 = 0, 1, 2, 3
RK4, RK5F = 0, 1

# -O3 with the x86-64-v3 instruction set (AVX2 + FMA) rather than
# -march=native: the library is built on one host and may be loaded on another
# (the GPU machine's), and every x86-64 server of the last decade has v3.
# Vector code does not change any result: no contraction, no reassociation.
CFLAGS = ["-O3", "-march=x86-64-v3", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp"]


def build(force=True):
    """Compile liboracle.so with gcc (strict FP64: no contraction)."""
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO)
    return _SO


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int), ("L", ctypes.c_int), ("k", ctypes.c_int),
        ("mode", ctypes.c_int), ("vel_id", ctypes.c_int), ("ntr", ctypes.c_int),
        ("rk", ctypes.c_int), ("reserved", ctypes.c_int),
        ("vp", ctypes.c_double * 8), ("dt", ctypes.c_double), ("t0", ctypes.c_double),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_SO)
        L.orc_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_velocity.argtypes = [ctypes.c_int, _D, ctypes.c_double, _D, _D]
        L.orc_trace.argtypes = [ctypes.c_int64, _D, ctypes.c_int, _D, ctypes.c_int, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int64, _D]
        L.orc_knn.argtypes = [ctypes.c_int64, _D, ctypes.c_int64, _D, ctypes.c_int, _I32, _D]
        L.orc_gauss_solve.argtypes = [ctypes.c_int, _D, _D]
        L.orc_gauss_solve.restype = ctypes.c_int
        L.orc_assemble.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D,
                                   ctypes.c_double, _D, _D, _D]
        L.orc_weights.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D,
                                  ctypes.c_double, _D, _D]
        L.orc_weights.restype = ctypes.c_int
        L.orc_step_sample.argtypes = [ctypes.c_int64, _D, ctypes.POINTER(Params), ctypes.c_int64,
                                      ctypes.c_int64, _I64, _D, _D, _I32, _D, _D, _I32]
        L.orc_step_sample.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.c_int64, _D, ctypes.POINTER(Params), ctypes.c_int64,
                              ctypes.c_int64, _D, _I64]
        L.orc_run.restype = ctypes.c_int
        L.orc_bspline.argtypes = [ctypes.c_double]
        L.orc_bspline.restype = ctypes.c_double
        L.orc_patch_coef.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_double, _D, _D]
        L.orc_patch_coef.restype = ctypes.c_int
        L.orc_patch_eval.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _D, _D, ctypes.c_double, _D, _D]
        L.orc_patch_eval.restype = ctypes.c_double
        L.orc_pu_patches.argtypes = [ctypes.c_int64, _D, ctypes.c_int64, _D, ctypes.c_double, _I64, _I32]
        L.orc_pu_step.argtypes = [ctypes.c_int64, _D, ctypes.c_int64, _D, ctypes.c_double, _I64, _I32,
                                  ctypes.POINTER(Params), ctypes.c_int64, ctypes.c_int64, _I64, _D, _D, _D, _I32]
        L.orc_pu_step.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def threads():
    return lib().orc_threads()


def set_threads(n):
    """Threads of the oracle's later parallel loops."""
    lib().orc_set_threads(int(n))


def make_params(n, L, k, mode=0, vel_id=VEL_ZERO, vp=(), dt=0.0, t0=0.0, ntr=1, rk=RK4):
    p = Params()
    p.n, p.L, p.k, p.mode, p.vel_id, p.ntr = int(n), int(L), int(k), int(mode), int(vel_id), int(ntr)
    p.rk = int(rk)
    v = list(vp) + [0.0] * (8 - len(vp))
    for i in range(8):
        p.vp[i] = float(v[i])
    p.dt, p.t0 = float(dt), float(t0)
    return p


def velocity(vel_id, vp, t, x):
    x = _f64(x, (3,))
    vpa = _f64(list(vp) + [0.0] * (8 - len(vp)))
    u = np.zeros(3)
    lib().orc_velocity(int(vel_id), _d(vpa), float(t), _d(x), _d(u))
    return u


def trace(nodes, vel_id, vp, t0, dt, m, rk=RK4):
    nodes = _f64(nodes)
    N = nodes.shape[0]
    vpa = _f64(list(vp) + [0.0] * (8 - len(vp)))
    xi = np.zeros((N, 3))
    lib().orc_trace(N, _d(nodes), int(vel_id), _d(vpa), int(rk), float(t0), float(dt), int(m), _d(xi))
    return xi


def knn(nodes, queries, n):
    nodes = _f64(nodes)
    queries = _f64(queries).reshape(-1, 3)
    Q = queries.shape[0]
    idx = np.zeros((Q, n), dtype=np.int32)
    d2 = np.zeros((Q, n))
    lib().orc_knn(nodes.shape[0], _d(nodes), Q, _d(queries), int(n),
                  idx.ctypes.data_as(_I32), _d(d2))
    return idx, d2


def gauss_solve(A, b):
    A = _f64(A).copy()
    b = _f64(b).copy()
    st = lib().orc_gauss_solve(A.shape[0], _d(A), _d(b))
    return b, st


def assemble(n, L, k, xs, center, s2, xi):
    M = n + (L + 1) ** 2
    A = np.zeros((M, M))
    r = np.zeros(M)
    lib().orc_assemble(n, L, k, _d(_f64(xs)), _d(_f64(center)), float(s2), _d(_f64(xi)), _d(A), _d(r))
    return A, r


def weights(n, L, k, xs, center, s2, xi):
    w = np.zeros(n)
    st = lib().orc_weights(n, L, k, _d(_f64(xs)), _d(_f64(center)), float(s2), _d(_f64(xi)), _d(w))
    return w, st


def step_sample(nodes, params, m, jl, q_in=None):
    """One step for target nodes jl.  Returns dict(xi, S, w, q, status)."""
    nodes = _f64(nodes)
    N = nodes.shape[0]
    jl = np.ascontiguousarray(jl, dtype=np.int64)
    J = jl.shape[0]
    n, ntr = params.n, params.ntr
    xi = np.zeros((J, 3))
    S = np.zeros((J, n), dtype=np.int32)
    w = np.zeros((J, n))
    st = np.zeros(J, dtype=np.int32)
    qo = None
    qp = None
    if q_in is not None:
        q_in = _f64(q_in).reshape(ntr, N)
        qo = np.zeros((ntr, J))
        qp = _d(q_in)
    lib().orc_step_sample(N, _d(nodes), ctypes.byref(params), int(m), J, jl.ctypes.data_as(_I64),
                          qp, _d(xi), S.ctypes.data_as(_I32), _d(w),
                          _d(qo) if qo is not None else None, st.ctypes.data_as(_I32))
    return dict(xi=xi, S=S, w=w, q=qo, status=st)


def run(nodes, params, q0, nsteps, m0=0):
    """Full run; returns (q, status, fail_step)."""
    nodes = _f64(nodes)
    N = nodes.shape[0]
    q = _f64(q0).reshape(params.ntr, N).copy()
    fs = ctypes.c_int64(-1)
    st = lib().orc_run(N, _d(nodes), ctypes.byref(params), int(m0), int(nsteps), _d(q), ctypes.byref(fs))
    return q, st, fs.value


# ---------------------------------------------------------------- RBF-PU


def bspline(r):
    """The cubic B-spline weight function (eq. bspline)."""
    return lib().orc_bspline(float(r))


def pu_radius(n, N):
    """One patch radius for every patch, R = 2 sqrt(n/N) (eq. rad_patches)."""
    return 2.0 * np.sqrt(n / N)


def pu_count(a, n, N):
    """Number of patches, ceil(a N / n) (eq. num_patches)."""
    return int(np.ceil(a * N / n))


def pu_patches(nodes, centers, R):
    """Patch membership: (counts, offsets, idx) with the nodes of patch l in
    idx[offsets[l]:offsets[l+1]], in (d^2, index) order."""
    nodes, centers = _f64(nodes), _f64(centers)
    Mp = centers.shape[0]
    counts = np.zeros(Mp, dtype=np.int64)
    lib().orc_pu_patches(nodes.shape[0], _d(nodes), Mp, _d(centers), float(R),
                         counts.ctypes.data_as(_I64), None)
    idx = np.zeros(max(int(counts.sum()), 1), dtype=np.int32)
    lib().orc_pu_patches(nodes.shape[0], _d(nodes), Mp, _d(centers), float(R),
                         counts.ctypes.data_as(_I64), idx.ctypes.data_as(_I32))
    offsets = np.concatenate([[0], np.cumsum(counts)])
    return counts, offsets, idx


def patch_coef(L, k, xs, omega, R2, qv):
    xs = _f64(xs).reshape(-1, 3)
    n = xs.shape[0]
    coef = np.zeros(n + (L + 1) ** 2)
    st = lib().orc_patch_coef(n, L, k, _d(xs), _d(_f64(omega)), float(R2), _d(_f64(qv)), _d(coef))
    return coef, st


def patch_eval(L, k, xs, omega, R2, coef, x):
    xs = _f64(xs).reshape(-1, 3)
    return lib().orc_patch_eval(xs.shape[0], L, k, _d(xs), _d(_f64(omega)), float(R2), _d(_f64(coef)),
                                _d(_f64(x)))


def pu_step(nodes, centers, R, patches, params, m, jl, q_in):
    """One RBF-PU step for the target nodes jl; patches from pu_patches.
    Returns dict(xi, q, status)."""
    nodes, centers = _f64(nodes), _f64(centers)
    N = nodes.shape[0]
    counts, _, idx = patches
    counts = np.ascontiguousarray(counts, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    jl = np.ascontiguousarray(jl, dtype=np.int64)
    J = jl.shape[0]
    q_in = _f64(q_in).reshape(params.ntr, N)
    xi = np.zeros((J, 3))
    qo = np.zeros((params.ntr, J))
    st = np.zeros(J, dtype=np.int32)
    lib().orc_pu_step(N, _d(nodes), centers.shape[0], _d(centers), float(R), counts.ctypes.data_as(_I64),
                      idx.ctypes.data_as(_I32), ctypes.byref(params), int(m), J, jl.ctypes.data_as(_I64),
                      _d(q_in), _d(xi), _d(qo), st.ctypes.data_as(_I32))
    return dict(xi=xi, q=qo, status=st)


def pu_run(nodes, centers, R, params, q0, nsteps, m0=0):
    """Full RBF-PU run; returns (q, status, fail_step)."""
    nodes = _f64(nodes)
    N = nodes.shape[0]
    patches = pu_patches(nodes, centers, R)
    q = _f64(q0).reshape(params.ntr, N).copy()
    jl = np.arange(N, dtype=np.int64)
    for m in range(m0, m0 + nsteps):
        o = pu_step(nodes, centers, R, patches, params, m, jl, q)
        bad = np.flatnonzero(o["status"])
        if bad.size:
            return q, int(o["status"][bad[0]]), m
        q = o["q"]
    return q, ORC_OK, -1
