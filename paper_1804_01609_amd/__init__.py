"""Python binding of librbfsl (the MI355X local-stencil RBF semi-Lagrangian
transport library): argument marshalling over the C ABI of include/rbfsl.h.

Host arrays are numpy float64/int32; device arrays are torch CUDA (HIP)
tensors, passed by pointer together with the current torch stream.  Every
step of the method runs in the library's HIP kernels; there is no CPU path
here, and loading fails loudly when the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# RBFSL_LIB_PATH selects another build of the same sources (the tests load a
# host-sanitized build this way)
LIB_PATH = os.environ.get("RBFSL_LIB_PATH") or os.path.join(_HERE, "librbfsl.so")

RBFSL_OK = 0
RBFSL_E_INVAL = -1
RBFSL_E_NOMEM = -2
RBFSL_E_DEVICE = -3
RBFSL_E_SINGULAR = -4
RBFSL_E_NONFINITE = -5
RBFSL_E_STATE = -6
RBFSL_E_SEARCH = -7
RBFSL_E_BUDGET = -8
RBFSL_E_CAPACITY = -9

VEL_ZERO, VEL_SOLID_BODY, VEL_DEFORM, VEL_NL2010 = 0, 1, 2, 3
STENCIL_PU = 2  # RBF-PU (PuTransport)
RK4, RK5_FEHLBERG = 0, 1

EXPORTS = [
    "rbfsl_create", "rbfsl_set_q", "rbfsl_step", "rbfsl_run", "rbfsl_steps_per_launch", "rbfsl_get_q",
    "rbfsl_get_state",
    "rbfsl_get_failures", "rbfsl_profile", "rbfsl_phase_times", "rbfsl_debug_departure", "rbfsl_debug_stencils", "rbfsl_debug_weights",
    "rbfsl_debug_sample", "rbfsl_source_hash", "rbfsl_weights_noalloc", "rbfsl_weights_noalloc_capacity",
    "rbfsl_knn", "rbfsl_weights", "rbfsl_max_system", "rbfsl_strerror", "rbfsl_last_error",
    "rbfsl_destroy", "rbfsl_create_pu", "rbfsl_pu_info", "rbfsl_debug_patches",
    "rbfsl_pool_create", "rbfsl_pool_run_bytes", "rbfsl_pool_add", "rbfsl_pool_step", "rbfsl_pool_run_info",
    "rbfsl_pool_get_q", "rbfsl_pool_remove", "rbfsl_pool_info", "rbfsl_pool_variants", "rbfsl_pool_set_variant",
    "rbfsl_pool_tune", "rbfsl_pool_serve", "rbfsl_pool_last_error", "rbfsl_pool_destroy",
]


class RbfslError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__(f"rbfsl error {code}: {msg}")


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("L", ctypes.c_int32), ("k", ctypes.c_int32),
        ("stencil_mode", ctypes.c_int32), ("velocity_id", ctypes.c_int32),
        ("n_tracers", ctypes.c_int32), ("integrator", ctypes.c_int32), ("cache_factors", ctypes.c_int32),
        ("vel", ctypes.c_double * 8),
        ("dt", ctypes.c_double), ("t0", ctypes.c_double),
    ]


class PoolConfig(ctypes.Structure):
    _fields_ = [("max_runs", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("hbm_budget", ctypes.c_int64),
                ("log_requests", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PoolStats(ctypes.Structure):
    _fields_ = [("runs", ctypes.c_int32), ("active", ctypes.c_int32),
                ("bytes_used", ctypes.c_int64), ("bytes_budget", ctypes.c_int64),
                ("steps_launched", ctypes.c_int64), ("items_per_step", ctypes.c_int64 * 4),
                ("blocks", ctypes.c_int32 * 4), ("graph", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("variant", ctypes.c_int32), ("ms_per_step", ctypes.c_float),
                ("chosen", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("arrival", ctypes.c_double), ("nodes_xyz", ctypes.c_void_p), ("N", ctypes.c_int64),
                ("params", Params), ("q0", ctypes.c_void_p), ("nsteps", ctypes.c_int64),
                ("q_out", ctypes.c_void_p)]


class RequestResult(ctypes.Structure):
    _fields_ = [("admitted", ctypes.c_double), ("finished", ctypes.c_double), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("steps", ctypes.c_int64)]


_lib = None
_P = ctypes.c_void_p


def lib():
    """Load librbfsl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1804_01609_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        L.rbfsl_source_hash.restype = ctypes.c_char_p
        from . import build as _build
        built, here = L.rbfsl_source_hash().decode(), _build.source_hash()
        if built != here:
            raise RuntimeError(f"{LIB_PATH} was built from other sources (hash {built[:12]}, sources "
                               f"{here[:12]}): rebuild it with `python -m paper_1804_01609_amd.build`")
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.rbfsl_create.argtypes = [_P, i64, ctypes.c_int, ctypes.POINTER(Params), _P, ctypes.POINTER(_P)]
        L.rbfsl_set_q.argtypes = [_P, _P, ctypes.c_int]
        L.rbfsl_step.argtypes = [_P]
        L.rbfsl_run.argtypes = [_P, i64]
        L.rbfsl_steps_per_launch.argtypes = [_P, i64]
        L.rbfsl_steps_per_launch.restype = i64
        L.rbfsl_get_q.argtypes = [_P, _P, ctypes.c_int]
        L.rbfsl_get_state.argtypes = [_P, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
        L.rbfsl_get_failures.argtypes = [_P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.rbfsl_profile.argtypes = [_P, ctypes.c_int]
        L.rbfsl_phase_times.argtypes = [_P, _P, ctypes.POINTER(i64)]
        L.rbfsl_debug_departure.argtypes = [_P, _P]
        L.rbfsl_debug_stencils.argtypes = [_P, _P]
        L.rbfsl_debug_weights.argtypes = [_P, _P]
        L.rbfsl_debug_sample.argtypes = [_P, _P, i64, _P, _P, _P]
        L.rbfsl_create_pu.argtypes = [_P, i64, ctypes.c_int, _P, i64, ctypes.c_double, ctypes.POINTER(Params), _P,
                                      ctypes.POINTER(_P)]
        L.rbfsl_pu_info.argtypes = [_P, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_double)]
        L.rbfsl_debug_patches.argtypes = [_P, _P, _P]
        L.rbfsl_knn.argtypes = [_P, i64, _P, i64, i32, _P, _P, ctypes.c_int, _P]
        L.rbfsl_weights.argtypes = [_P, i64, _P, _P, _P, _P, i64, i32, i32, i32, _P, _P, ctypes.c_int, _P]
        L.rbfsl_weights_noalloc.argtypes = [_P, i64, _P, _P, _P, _P, i64, i32, i32, i32, _P, _P, _P]
        L.rbfsl_weights_noalloc_capacity.restype = i64
        L.rbfsl_max_system.restype = ctypes.c_int
        L.rbfsl_strerror.restype = ctypes.c_char_p
        L.rbfsl_strerror.argtypes = [ctypes.c_int]
        L.rbfsl_last_error.restype = ctypes.c_char_p
        L.rbfsl_last_error.argtypes = [_P]
        L.rbfsl_destroy.argtypes = [_P]
        L.rbfsl_destroy.restype = None
        L.rbfsl_pool_create.argtypes = [ctypes.POINTER(PoolConfig), ctypes.POINTER(_P)]
        L.rbfsl_pool_run_bytes.argtypes = [i64, ctypes.POINTER(Params), i64]
        L.rbfsl_pool_run_bytes.restype = i64
        L.rbfsl_pool_add.argtypes = [_P, _P, i64, ctypes.c_int, ctypes.POINTER(Params), _P, ctypes.c_int, i64,
                                     ctypes.POINTER(i64)]
        L.rbfsl_pool_step.argtypes = [_P, i64]
        L.rbfsl_pool_run_info.argtypes = [_P, i64, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                          ctypes.POINTER(ctypes.c_int)]
        L.rbfsl_pool_get_q.argtypes = [_P, i64, _P, ctypes.c_int]
        L.rbfsl_pool_remove.argtypes = [_P, i64]
        L.rbfsl_pool_info.argtypes = [_P, ctypes.POINTER(PoolStats)]
        L.rbfsl_pool_variants.argtypes = [_P, _P, _P, _P, i32]
        L.rbfsl_pool_set_variant.argtypes = [_P, i32, i32]
        L.rbfsl_pool_tune.argtypes = [_P, i32, _P, i32, ctypes.POINTER(i32)]
        L.rbfsl_pool_serve.argtypes = [_P, _P, i64, _P, ctypes.POINTER(ctypes.c_double)]
        L.rbfsl_pool_last_error.restype = ctypes.c_char_p
        L.rbfsl_pool_last_error.argtypes = [_P]
        L.rbfsl_pool_destroy.argtypes = [_P]
        L.rbfsl_pool_destroy.restype = None
        _lib = L
    return _lib


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, on_device, keepalive) for a numpy array or torch tensor."""
    if x is None:
        return None, 0, None
    if _is_torch(x):
        import torch
        tdt = torch.float64 if dtype == np.float64 else torch.int32
        if x.dtype != tdt or not x.is_contiguous():
            raise TypeError(f"expected a contiguous {tdt} tensor")
        return ctypes.c_void_p(x.data_ptr()), (1 if x.is_cuda else 0), x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(ctypes.c_void_p), 0, a


def _stream(on_device):
    if not on_device:
        return None
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(code, ctx=None, pool=None):
    if code != RBFSL_OK:
        L = lib()
        msg = L.rbfsl_strerror(code).decode()
        extra = ""
        if ctx:
            extra = L.rbfsl_last_error(ctx).decode()
        elif pool:
            extra = L.rbfsl_pool_last_error(pool).decode()
        if extra:
            msg += ": " + extra
        raise RbfslError(code, msg)


def make_params(n, L=-1, k=-1, stencil_mode=0, velocity_id=VEL_ZERO, vel=(), dt=0.1, t0=0.0,
                n_tracers=1, integrator=RK4, cache_factors=0):
    p = Params()
    p.n, p.L, p.k = int(n), int(L), int(k)
    p.stencil_mode, p.velocity_id, p.n_tracers = int(stencil_mode), int(velocity_id), int(n_tracers)
    p.integrator = int(integrator)
    p.cache_factors = int(cache_factors)
    v = list(vel) + [0.0] * (8 - len(vel))
    for i in range(8):
        p.vel[i] = float(v[i])
    p.dt, p.t0 = float(dt), float(t0)
    return p


class Transport:
    """One transport problem on the GPU: nodes, parameters and the state q^m.

    nodes: (N, 3) numpy array or CUDA tensor; q arrays are (n_tracers, N).
    `stream` is a raw hipStream_t (int) or None for torch's current stream
    when device tensors are used, else the default stream.
    """

    def __init__(self, nodes, params, stream=None):
        L = lib()
        ptr, dev, keep = _ptr(nodes, np.float64)
        self.N = int(nodes.shape[0])
        self.params = params
        self.ntr = params.n_tracers
        s = ctypes.c_void_p(stream) if stream is not None else _stream(dev)
        self._ctx = _P()
        code = L.rbfsl_create(ptr, self.N, dev, ctypes.byref(params), s, ctypes.byref(self._ctx))
        if code != RBFSL_OK:
            self._ctx = None
            _check(code)

    def close(self):
        if getattr(self, "_ctx", None):
            lib().rbfsl_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_q(self, q):
        ptr, dev, keep = _ptr(q, np.float64)
        _check(lib().rbfsl_set_q(self._ctx, ptr, dev), self._ctx)

    def step(self):
        _check(lib().rbfsl_step(self._ctx), self._ctx)

    def run(self, nsteps):
        _check(lib().rbfsl_run(self._ctx, int(nsteps)), self._ctx)

    def steps_per_launch(self, nsteps):
        """Steps per launch that run(nsteps) takes (1: step by step)."""
        return int(lib().rbfsl_steps_per_launch(self._ctx, int(nsteps)))

    def run_status(self, nsteps):
        """run() returning the status code instead of raising."""
        return lib().rbfsl_run(self._ctx, int(nsteps))

    def get_q(self, out=None):
        if out is None:
            out = np.zeros((self.ntr, self.N))
        ptr, dev, keep = _ptr(out, np.float64)
        _check(lib().rbfsl_get_q(self._ctx, ptr, dev), self._ctx)
        return out

    def state(self):
        m = ctypes.c_int64()
        t = ctypes.c_double()
        _check(lib().rbfsl_get_state(self._ctx, ctypes.byref(m), ctypes.byref(t)))
        return m.value, t.value

    def failures(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().rbfsl_get_failures(self._ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def profile(self, enable=True):
        _check(lib().rbfsl_profile(self._ctx, int(bool(enable))), self._ctx)

    def phase_times(self):
        """Accumulated device ms per phase (trace, search, solve, apply) and steps."""
        ms = np.zeros(4)
        st = ctypes.c_int64()
        _check(lib().rbfsl_phase_times(self._ctx, ms.ctypes.data_as(_P), ctypes.byref(st)), self._ctx)
        return ms, st.value

    def departure(self):
        xi = np.zeros((self.N, 3))
        _check(lib().rbfsl_debug_departure(self._ctx, xi.ctypes.data_as(_P)), self._ctx)
        return xi

    def stencils(self):
        S = np.zeros((self.N, self.params.n), dtype=np.int32)
        _check(lib().rbfsl_debug_stencils(self._ctx, S.ctypes.data_as(_P)), self._ctx)
        return S

    def weights(self):
        w = np.zeros((self.N, self.params.n))
        _check(lib().rbfsl_debug_weights(self._ctx, w.ctypes.data_as(_P)), self._ctx)
        return w

    def sample(self, jl):
        """Departure points, stencils and weights of the last step at nodes jl."""
        jl = np.ascontiguousarray(jl, dtype=np.int64)
        J = jl.shape[0]
        xi = np.zeros((J, 3))
        S = np.zeros((J, self.params.n), dtype=np.int32)
        w = np.zeros((J, self.params.n))
        _check(lib().rbfsl_debug_sample(self._ctx, jl.ctypes.data_as(_P), J, xi.ctypes.data_as(_P),
                                        S.ctypes.data_as(_P), w.ctypes.data_as(_P)), self._ctx)
        return xi, S, w


class PuTransport(Transport):
    """RBF-PU transport (Sections 2.3 and 3.3.3): patches are the caps of
    radius R around `centers` (Mp x 3); by default the paper's choices,
    R = 2 sqrt(n/N) and ceil(a N / n) quasi-uniform centres, come from
    `pu_radius` / `pu_count` and the caller's point set.  params.stencil_mode
    must be STENCIL_PU."""

    def __init__(self, nodes, centers, R, params, stream=None):
        L = lib()
        ptr, dev, keep = _ptr(nodes, np.float64)
        cptr, cdev, ckeep = _ptr(centers, np.float64)
        if cdev != dev:
            raise ValueError("nodes and centers must both be host arrays or both device tensors")
        self.N = int(nodes.shape[0])
        self.params = params
        self.ntr = params.n_tracers
        s = ctypes.c_void_p(stream) if stream is not None else _stream(dev)
        self._ctx = _P()
        code = L.rbfsl_create_pu(ptr, self.N, dev, cptr, int(centers.shape[0]), float(R), ctypes.byref(params), s,
                                 ctypes.byref(self._ctx))
        if code != RBFSL_OK:
            self._ctx = None
            _check(code)

    def info(self):
        Mp, ncap, nmax, R = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(lib().rbfsl_pu_info(self._ctx, ctypes.byref(Mp), ctypes.byref(ncap), ctypes.byref(nmax),
                                   ctypes.byref(R)), self._ctx)
        return dict(patches=Mp.value, ncap=ncap.value, nmax=nmax.value, R=R.value)

    def patches(self):
        """(counts, list of node-index arrays) of every patch."""
        inf = self.info()
        counts = np.zeros(inf["patches"], dtype=np.int32)
        idx = np.zeros((inf["patches"], inf["ncap"]), dtype=np.int32)
        _check(lib().rbfsl_debug_patches(self._ctx, counts.ctypes.data_as(_P), idx.ctypes.data_as(_P)), self._ctx)
        return counts, [idx[l, :counts[l]] for l in range(counts.shape[0])]


def pu_radius(n, N):
    """The patch radius R = 2 sqrt(n/N) (eq. rad_patches)."""
    return 2.0 * np.sqrt(n / N)


def pu_count(a, n, N):
    """The patch count ceil(a N / n) (eq. num_patches)."""
    return int(np.ceil(a * N / n))


def knn(nodes, queries, n):
    """Exact n nearest nodes of every query (host numpy in, host numpy out)."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    queries = np.ascontiguousarray(queries, dtype=np.float64).reshape(-1, 3)
    Q = queries.shape[0]
    idx = np.zeros((Q, n), dtype=np.int32)
    d2 = np.zeros((Q, n))
    _check(lib().rbfsl_knn(nodes.ctypes.data_as(_P), nodes.shape[0], queries.ctypes.data_as(_P), Q,
                           int(n), idx.ctypes.data_as(_P), d2.ctypes.data_as(_P), 0, None))
    return idx, d2


def weights(nodes, idx, centers, s2, evals, n, L, k):
    """Batched stencil weights (host numpy in/out); returns (w, status)."""
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, n)
    count = idx.shape[0]
    centers = np.ascontiguousarray(centers, dtype=np.float64).reshape(count, 3)
    evals = np.ascontiguousarray(evals, dtype=np.float64).reshape(count, 3)
    s2 = np.ascontiguousarray(s2, dtype=np.float64).reshape(count)
    w = np.zeros((count, n))
    st = np.zeros(count, dtype=np.int32)
    _check(lib().rbfsl_weights(nodes.ctypes.data_as(_P), nodes.shape[0], idx.ctypes.data_as(_P),
                               centers.ctypes.data_as(_P), s2.ctypes.data_as(_P),
                               evals.ctypes.data_as(_P), count, int(n), int(L), int(k),
                               w.ctypes.data_as(_P), st.ctypes.data_as(_P), 0, None))
    return w, st


def weights_noalloc_ptr(nodes, N, idx, centers, s2, evals, count, n, L, k, w, status=0, stream=0):
    """rbfsl_weights_noalloc on raw device addresses (ints): nodes N x 3,
    idx count x n (int32), centers and evals count x 3, s2 count, outputs w
    count x n and status count (0: none); enqueued on `stream` (0: default).
    Returns the status code without raising."""
    P = ctypes.c_void_p
    return lib().rbfsl_weights_noalloc(P(nodes), int(N), P(idx), P(centers), P(s2), P(evals), int(count), int(n),
                                       int(L), int(k), P(w), P(status) if status else None,
                                       P(stream) if stream else None)


def weights_noalloc_code(nodes, idx, centers, s2, evals, n, L, k, w, status=None, stream=None):
    """rbfsl_weights_noalloc on device tensors (torch, float64 / int32,
    contiguous): nodes (N, 3), idx (count, n), centers and evals (count, 3),
    s2 (count,), outputs w (count, n) and status (count,) or None.  Work is
    enqueued on `stream` (raw hipStream_t) or torch's current stream; returns
    the status code without raising."""
    args = []
    for x, dt in ((nodes, np.float64), (idx, np.int32), (centers, np.float64), (s2, np.float64),
                  (evals, np.float64), (w, np.float64)):
        if not _is_torch(x):
            raise TypeError("rbfsl_weights_noalloc takes device tensors")
        args.append(_ptr(x, dt)[0])
    st = _ptr(status, np.int32)[0] if status is not None else None
    count = int(idx.shape[0])
    s = ctypes.c_void_p(stream) if stream is not None else _stream(1)
    return lib().rbfsl_weights_noalloc(args[0], int(nodes.shape[0]), args[1], args[2], args[3], args[4], count,
                                       int(n), int(L), int(k), args[5], st, s)


def weights_noalloc_capacity():
    return lib().rbfsl_weights_noalloc_capacity()


def max_system():
    return lib().rbfsl_max_system()


def pool_variants():
    """Compiled solver variants of the pooled kernels: list of dicts
    (index, mcap, waves per stencil, stencils per workgroup, panel width)."""
    L = lib()
    nv = L.rbfsl_pool_variants(None, None, None, None, 0)
    a = [np.zeros(nv, dtype=np.int32) for _ in range(4)]
    L.rbfsl_pool_variants(*[x.ctypes.data_as(_P) for x in a], nv)
    return [dict(index=i, mcap=int(a[0][i]), waves=int(a[1][i]), group=int(a[2][i]), panel=int(a[3][i]))
            for i in range(nv)]


def pool_run_bytes(N, params, nsteps):
    return int(lib().rbfsl_pool_run_bytes(int(N), ctypes.byref(params), int(nsteps)))


class Pool:
    """Many independent runs resident on the GPU and stepped together
    (batched form), or fed by a request stream (served form)."""

    def __init__(self, max_runs=64, hbm_budget=0, use_graph=True, log_requests=False):
        cfg = PoolConfig(int(max_runs), int(bool(use_graph)), int(hbm_budget), int(bool(log_requests)), 0)
        self._p = _P()
        code = lib().rbfsl_pool_create(ctypes.byref(cfg), ctypes.byref(self._p))
        if code != RBFSL_OK:
            self._p = None
            _check(code)
        self._shape = {}

    def close(self):
        if getattr(self, "_p", None):
            lib().rbfsl_pool_destroy(self._p)
            self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _chk(self, code):
        _check(code, pool=self._p)

    def add(self, nodes, params, q0, nsteps):
        """Admit a run; returns its id (raises RbfslError with code RBFSL_E_BUDGET when it does not fit)."""
        nptr, ndev, nk = _ptr(nodes, np.float64)
        qptr, qdev, qk = _ptr(q0, np.float64)
        rid = ctypes.c_int64()
        self._chk(lib().rbfsl_pool_add(self._p, nptr, int(nodes.shape[0]), ndev, ctypes.byref(params), qptr, qdev,
                                       int(nsteps), ctypes.byref(rid)))
        self._shape[rid.value] = (params.n_tracers, int(nodes.shape[0]))
        return rid.value

    def step(self, nsteps=1):
        self._chk(lib().rbfsl_pool_step(self._p, int(nsteps)))

    def info(self, rid):
        """(steps done, steps requested, status code) of a run."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        self._chk(lib().rbfsl_pool_run_info(self._p, int(rid), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def get_q(self, rid, out=None):
        if out is None:  # an unknown id is the library's to reject
            out = np.zeros(self._shape.get(rid, (1,)))
        ptr, dev, keep = _ptr(out, np.float64)
        self._chk(lib().rbfsl_pool_get_q(self._p, int(rid), ptr, dev))
        return out

    def remove(self, rid):
        self._chk(lib().rbfsl_pool_remove(self._p, int(rid)))
        self._shape.pop(rid, None)

    def stats(self):
        st = PoolStats()
        self._chk(lib().rbfsl_pool_info(self._p, ctypes.byref(st)))
        return dict(runs=st.runs, active=st.active, bytes_used=st.bytes_used, bytes_budget=st.bytes_budget,
                    steps_launched=st.steps_launched, items_per_step=list(st.items_per_step),
                    blocks=list(st.blocks), graph=bool(st.graph))

    def set_variant(self, M, variant):
        self._chk(lib().rbfsl_pool_set_variant(self._p, int(M), int(variant)))

    def tune(self, trials=2):
        """Autotune the solver variant per system size; returns the trials."""
        cap = 256
        res = (TuneResult * cap)()
        cnt = ctypes.c_int32()
        self._chk(lib().rbfsl_pool_tune(self._p, int(trials), res, cap, ctypes.byref(cnt)))
        return [dict(M=r.M, variant=r.variant, ms_per_step=r.ms_per_step, chosen=bool(r.chosen))
                for r in res[:cnt.value]]

    def serve(self, requests):
        """requests: list of dicts (arrival, nodes, params, q0, nsteps).  Runs
        the stream with continuous batching; returns (results, q_outs, wall_s)."""
        nreq = len(requests)
        req = (Request * max(nreq, 1))()
        res = (RequestResult * max(nreq, 1))()
        keep, outs = [], []
        for i, r in enumerate(requests):
            nodes = np.ascontiguousarray(r["nodes"], dtype=np.float64)
            q0 = np.ascontiguousarray(r["q0"], dtype=np.float64)
            out = np.zeros_like(q0)
            keep += [nodes, q0]
            outs.append(out)
            req[i].arrival = float(r["arrival"])
            req[i].nodes_xyz = nodes.ctypes.data
            req[i].N = nodes.shape[0]
            req[i].params = r["params"]
            req[i].q0 = q0.ctypes.data
            req[i].nsteps = int(r["nsteps"])
            req[i].q_out = out.ctypes.data
        wall = ctypes.c_double()
        self._chk(lib().rbfsl_pool_serve(self._p, req, nreq, res, ctypes.byref(wall)))
        results = [dict(admitted=res[i].admitted, finished=res[i].finished, status=res[i].status,
                        steps=res[i].steps) for i in range(nreq)]
        return results, outs, wall.value
