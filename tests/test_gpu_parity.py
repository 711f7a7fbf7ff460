"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  The bar is bit-exact for stencil indices; the weights
must agree to 1e-11 relative and q to 1e-9 after a full run -- and because
both sides perform the same correctly rounded operations in the same order,
they are expected to agree bit for bit, which the tests also record."""
import math
import sys

import numpy as np
import pytest

import oracle
import paper_1804_01609_amd as rb
from paper_1804_01609_amd import workloads as W

pytestmark = pytest.mark.gpu

W_TOL = 1e-11
Q_TOL = 1e-9


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def orc_params(cfg, mode=0, ntr=None):
    return oracle.make_params(cfg["n"], cfg["L"], cfg["k"], mode, cfg["vel_id"], cfg["vp"], cfg["dt"],
                              0.0, ntr if ntr is not None else cfg["ntr"])


def gpu_params(cfg, mode=0, ntr=None):
    return rb.make_params(cfg["n"], cfg["L"], cfg["k"], mode, cfg["vel_id"], cfg["vp"], cfg["dt"], 0.0,
                          ntr if ntr is not None else cfg["ntr"])


# ---------------------------------------------------------------- kNN

@pytest.mark.parametrize("N,n,Q", [(1024, 31, 500), (40962, 84, 3000), (10000, 56, 777),
                                   (655362, 120, 1500), (300, 300, 20), (97, 5, 64)])
def test_knn_bit_exact_against_brute_force(N, n, Q):
    say(f"[knn] N={N} n={n} Q={Q}")
    X = W.fibonacci_nodes(N)
    Qp = W.random_sphere_points(Q, seed=N + n)
    gi, gd = rb.knn(X, Qp, n)
    oi, od = oracle.knn(X, Qp, n)
    assert np.array_equal(gi, oi)
    assert np.array_equal(gd, od)


def test_knn_ties_and_degenerate_sets():
    say("[knn] ties")
    V = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, -1]], dtype=float)
    X = V[[4, 0, 2, 5, 1, 3]]
    Qp = np.concatenate([V, [[0.0, 0.0, 1.0], [1 / math.sqrt(2), 1 / math.sqrt(2), 0.0]]])
    for n in (1, 3, 6):
        gi, gd = rb.knn(X, Qp, n)
        oi, od = oracle.knn(X, Qp, n)
        assert np.array_equal(gi, oi) and np.array_equal(gd, od)
    # queries exactly at nodes, at cell corners, and duplicated nodes
    F = W.fibonacci_nodes(2000)
    F = np.concatenate([F, F[[3, 77, 1500]]])
    Qp = np.concatenate([F[:200], np.array([[0.0, 0.0, 1.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0]])])
    gi, gd = rb.knn(F, Qp, 40)
    oi, od = oracle.knn(F, Qp, 40)
    assert np.array_equal(gi, oi) and np.array_equal(gd, od)
    # clustered (non-uniform) nodes force the search radius to adapt
    C = W.random_sphere_points(3000, 5)
    C = C[C[:, 2] > 0.6]
    C = np.concatenate([C, W.random_sphere_points(50, 6)])
    Qp = W.random_sphere_points(300, 7)
    gi, gd = rb.knn(C, Qp, 31)
    oi, od = oracle.knn(C, Qp, 31)
    assert np.array_equal(gi, oi) and np.array_equal(gd, od)


# ---------------------------------------------------------------- weights

@pytest.mark.parametrize("N,n,L,k", [(1024, 31, 3, 2), (4096, 56, 4, 2), (40962, 84, 5, 3),
                                     (2562, 17, 1, 1), (655362, 120, 7, 4), (5000, 40, 4, 2),
                                     (8000, 100, 5, 3), (800, 9, 1, 0)])
def test_weights_match_oracle(N, n, L, k):
    say(f"[weights] N={N} n={n} L={L} k={k}")
    X = W.fibonacci_nodes(N)
    Qp = W.random_sphere_points(300, seed=n)
    idx, d2 = oracle.knn(X, Qp, n)
    s2 = d2[:, -1].copy()
    gw, st = rb.weights(X, idx, Qp, s2, Qp, n, L, k)
    assert np.all(st == 0)
    ow = np.zeros_like(gw)
    for t in range(Qp.shape[0]):
        ow[t], ost = oracle.weights(n, L, k, X[idx[t]], Qp[t], s2[t], Qp[t])
        assert ost == 0
    assert rel_err(gw, ow) <= W_TOL
    assert np.array_equal(gw, ow), "weights differ in the last bits"


def test_weights_off_centre_evaluation():
    # centre at a node, evaluation elsewhere (the paper's centre-point mode)
    say("[weights] off-centre")
    N, n, L, k = 40962, 84, 5, 3
    X = W.fibonacci_nodes(N)
    Qp = W.random_sphere_points(200, seed=3)
    K, _ = oracle.knn(X, Qp, 1)
    C = X[K[:, 0]]
    idx, d2 = oracle.knn(X, C, n)
    gw, st = rb.weights(X, idx, C, d2[:, -1].copy(), Qp, n, L, k)
    assert np.all(st == 0)
    for t in range(0, 200, 7):
        ow, _ = oracle.weights(n, L, k, X[idx[t]], C[t], d2[t, -1], Qp[t])
        assert np.array_equal(gw[t], ow)


def test_weights_singular_stencil_flagged():
    say("[weights] singular")
    X = W.fibonacci_nodes(1024)
    X = np.concatenate([X, X[[10]]])  # node 1024 duplicates node 10
    idx, d2 = oracle.knn(X, X[[10, 500]], 31)
    gw, st = rb.weights(X, idx, X[[10, 500]], d2[:, -1].copy(), X[[10, 500]], 31, 3, 2)
    assert st[0] == rb.RBFSL_E_SINGULAR and st[1] == 0


# ---------------------------------------------------------------- one step

def _one_step_check(cfg, X, q0, mode, jl=None):
    p = gpu_params(cfg, mode)
    with rb.Transport(X, p) as tr:
        tr.set_q(q0)
        tr.step()
        xi, S, w, q1 = tr.departure(), tr.stencils(), tr.weights(), tr.get_q()
    op = orc_params(cfg, mode)
    if jl is None:
        jl = np.arange(X.shape[0])
    o = oracle.step_sample(X, op, 0, jl, q0)
    assert np.all(o["status"] == 0)
    assert np.array_equal(xi[jl], o["xi"]), "departure points differ"
    assert np.array_equal(S[jl], o["S"]), "stencils differ"
    assert rel_err(w[jl], o["w"]) <= W_TOL
    assert np.array_equal(w[jl], o["w"])
    assert np.abs(q1[:, jl] - o["q"]).max() <= Q_TOL
    assert np.array_equal(q1[:, jl], o["q"])


@pytest.mark.parametrize("mode", [0, 1])
def test_one_step_c1_all_nodes(mode):
    say(f"[step] c1 mode={mode}")
    cfg = W.CONFIGS["c1"]
    X = W.fibonacci_nodes(cfg["N"])
    _one_step_check(cfg, X, W.initial_q(cfg, X), mode)


def test_one_step_c2_sampled():
    say("[step] c2 sampled")
    cfg = W.CONFIGS["c2"]
    X = W.fibonacci_nodes(cfg["N"])
    jl = np.unique(np.random.default_rng(0).integers(0, cfg["N"], 400))
    jl = np.concatenate([[0, 1, cfg["N"] - 1], jl])
    _one_step_check(cfg, X, W.initial_q(cfg, X), 0, jl)


def test_one_step_c3_sampled_eight_tracers():
    say("[step] c3 sampled")
    cfg = W.CONFIGS["c3"]
    X = W.fibonacci_nodes(cfg["N"])
    jl = np.unique(np.random.default_rng(1).integers(0, cfg["N"], 150))
    _one_step_check(cfg, X, W.initial_q(cfg, X), 0, jl)


def test_weights_at_a_late_step_c2():
    # trace, stencils and weights do not depend on q: compare them at step 300
    say("[step] c2 step 300 weights")
    cfg = W.CONFIGS["c2"]
    X = W.fibonacci_nodes(cfg["N"])
    p = gpu_params(cfg)
    with rb.Transport(X, p) as tr:
        tr.set_q(W.initial_q(cfg, X))
        tr.run(301)
        xi, S, w = tr.departure(), tr.stencils(), tr.weights()
    jl = np.arange(0, cfg["N"], 211)
    o = oracle.step_sample(X, orc_params(cfg), 300, jl)
    assert np.array_equal(xi[jl], o["xi"]) and np.array_equal(S[jl], o["S"])
    assert rel_err(w[jl], o["w"]) <= W_TOL


# ---------------------------------------------------------------- full runs

@pytest.mark.parametrize("mode", [0, 1])
def test_full_run_c1_matches_oracle(mode):
    say(f"[run] c1 mode={mode}")
    cfg = W.CONFIGS["c1"]
    X = W.fibonacci_nodes(cfg["N"])
    q0 = W.initial_q(cfg, X)
    with rb.Transport(X, gpu_params(cfg, mode)) as tr:
        tr.set_q(q0)
        tr.run(cfg["nsteps"])
        qg = tr.get_q()
        assert tr.state()[0] == cfg["nsteps"]
    qo, st, _ = oracle.run(X, orc_params(cfg, mode), q0, cfg["nsteps"])
    assert st == 0
    assert np.abs(qg - qo).max() <= Q_TOL
    assert np.array_equal(qg, qo)


@pytest.mark.parametrize("n,L,k,N,steps", [(84, 5, 3, 2562, 40), (56, 4, 2, 2000, 30),
                                           (120, 7, 4, 3000, 12)])
def test_full_run_deformational_matches_oracle(n, L, k, N, steps):
    say(f"[run] deform n={n} L={L} N={N}")
    cfg = dict(n=n, L=L, k=k, vel_id=W.VEL_DEFORM, vp=W.deform_vp(), dt=5.0 / steps, ntr=2)
    X = W.fibonacci_nodes(N)
    q0 = W.tracer_set(X, 2)
    with rb.Transport(X, gpu_params(cfg)) as tr:
        tr.set_q(q0)
        tr.run(steps)
        qg = tr.get_q()
    qo, st, _ = oracle.run(X, orc_params(cfg), q0, steps)
    assert st == 0
    assert np.abs(qg - qo).max() <= Q_TOL
    assert np.array_equal(qg, qo)


def test_c2_flow_returns_and_converges():
    # the deformational flow returns every parcel at t = T, so q(T) = q0 up to
    # the interpolation error, which must fall as N grows (C2's n, L, k, dt)
    say("[run] c2 flow, N = 10242 and 40962")
    cfg = W.CONFIGS["c2"]
    errs = []
    for N in (10242, cfg["N"]):
        X = W.fibonacci_nodes(N)
        q0 = W.initial_q(cfg, X)
        with rb.Transport(X, gpu_params(cfg)) as tr:
            tr.set_q(q0)
            tr.run(cfg["nsteps"])
            q = tr.get_q()
        errs.append(np.linalg.norm(q - q0) / np.linalg.norm(q0))
        say(f"  N={N}: relative l2 error at T = {errs[-1]:.3e}")
    assert errs[1] < 0.5 * errs[0]


def test_run_is_deterministic_and_resumable():
    say("[run] determinism")
    cfg = W.CONFIGS["c1"]
    X = W.fibonacci_nodes(cfg["N"])
    q0 = W.initial_q(cfg, X)
    with rb.Transport(X, gpu_params(cfg)) as a, rb.Transport(X, gpu_params(cfg)) as b:
        a.set_q(q0)
        b.set_q(q0)
        a.run(20)
        b.run(7)
        b.run(13)
        assert np.array_equal(a.get_q(), b.get_q())


def test_singular_step_is_not_committed():
    say("[run] singular")
    cfg = W.CONFIGS["c1"]
    X = W.fibonacci_nodes(cfg["N"])
    X = np.concatenate([X, X[[17]]])
    q0 = W.c1_bump(X)[None]
    with rb.Transport(X, gpu_params(cfg)) as tr:
        tr.set_q(q0)
        code = tr.run_status(5)
        assert code == rb.RBFSL_E_SINGULAR
        assert tr.state()[0] == 0
        assert np.array_equal(tr.get_q(), q0)
        assert tr.failures()[0] > 0
