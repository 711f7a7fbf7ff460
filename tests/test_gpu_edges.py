"""Edge cases of the HIP path against the oracle: empty inputs, the smallest
and largest systems, a stencil of all nodes, the degenerate one-node
interpolant, a query far from every node, and the pool's error paths."""
import sys

import numpy as np
import pytest

import oracle
import paper_1804_01609_amd as rb
from paper_1804_01609_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_empty_query_and_weight_batches():
    say("[edges] empty batches")
    X = W.fibonacci_nodes(300)
    idx, d2 = rb.knn(X, np.zeros((0, 3)), 10)
    assert idx.shape == (0, 10)
    w, st = rb.weights(X, np.zeros((0, 10), np.int32), np.zeros((0, 3)), np.zeros(0), np.zeros((0, 3)), 10, 1, 1)
    assert w.shape == (0, 10) and st.shape == (0,)


def test_stencil_of_every_node():
    # n = N: the stencil is the whole node set, ordered by distance
    say("[edges] n = N")
    X = W.fibonacci_nodes(100)
    Q = W.random_sphere_points(20, 9)
    idx, _ = rb.knn(X, Q, 100)
    io, _ = oracle.knn(X, Q, 100)
    assert np.array_equal(idx, io)
    p = rb.make_params(100, 2, 2, 0, rb.VEL_SOLID_BODY, W.tc1_vp(), 0.05, 0.0, 1)
    po = oracle.make_params(100, 2, 2, 0, oracle.VEL_SOLID, W.tc1_vp(), 0.05, 0.0, 1)
    q0 = W.c1_bump(X)[None]
    with rb.Transport(X, p) as tr:
        tr.set_q(q0)
        tr.run(3)
        q = tr.get_q()
    qo, st, _ = oracle.run(X, po, q0, 3)
    assert st == 0 and np.array_equal(q, qo)


def test_one_node_stencil_is_nearest_node_semi_lagrangian():
    # n = 1, L = 0, k = 0: a 2 x 2 system whose weight is exactly 1
    say("[edges] n = 1")
    X = W.fibonacci_nodes(400)
    q0 = W.c1_bump(X)[None]
    p = rb.make_params(1, 0, 0, 0, rb.VEL_SOLID_BODY, W.tc1_vp(), 0.1, 0.0, 1)
    po = oracle.make_params(1, 0, 0, 0, oracle.VEL_SOLID, W.tc1_vp(), 0.1, 0.0, 1)
    with rb.Transport(X, p) as tr:
        tr.set_q(q0)
        tr.run(2)
        q = tr.get_q()
        w = tr.weights()
        S = tr.stencils()
        xi = tr.departure()
    assert np.all(w == 1.0)
    qo, st, _ = oracle.run(X, po, q0, 2)
    assert st == 0 and np.array_equal(q, qo)
    assert np.array_equal(S[:, 0], oracle.knn(X, xi, 1)[0][:, 0])


def test_largest_supported_system():
    # M = n + (L+1)^2 = 192 exactly: the biggest solver variant, full capacity
    say("[edges] M = 192")
    M = rb.max_system()
    assert M >= 192
    n, L, k = 128, 7, 4
    assert n + (L + 1) ** 2 == 192
    X = W.fibonacci_nodes(3000)
    E = W.random_sphere_points(40, 21)
    idx, d2 = rb.knn(X, E, n)
    w, st = rb.weights(X, idx, E, d2[:, -1], E, n, L, k)
    wo = np.array([oracle.weights(n, L, k, X[idx[t]], E[t], d2[t, -1], E[t])[0] for t in range(len(E))])
    assert (st == 0).all()
    assert np.array_equal(w, wo)
    # one past the largest is refused before any device work
    with pytest.raises(rb.RbfslError):
        rb.Transport(X, rb.make_params(129, 7, 4))


def test_far_query_needs_a_wide_search():
    # a query point far from the sphere (the search radius has to grow)
    say("[edges] far query")
    X = W.fibonacci_nodes(2000)
    Q = np.array([[0.0, 0.0, 3.0], [1.2, -0.4, 0.1]])
    idx, _ = rb.knn(X, Q, 40)
    io, _ = oracle.knn(X, Q, 40)
    assert np.array_equal(idx, io)


def test_pool_error_paths_and_empty_steps():
    say("[edges] pool errors")
    with rb.Pool(max_runs=2, hbm_budget=1 << 28) as pl:
        pl.step(3)  # nothing admitted: a no-op
        with pytest.raises(rb.RbfslError) as e:
            pl.get_q(12345)
        assert e.value.code == rb.RBFSL_E_INVAL
        X = W.fibonacci_nodes(500)
        bad = rb.make_params(31, 3, 2, 1, rb.VEL_SOLID_BODY, W.tc1_vp(), 0.1, 0.0, 1)  # centre mode
        with pytest.raises(rb.RbfslError) as e:
            pl.add(X, bad, W.c1_bump(X)[None], 4)
        assert e.value.code == rb.RBFSL_E_INVAL
        assert pl.stats()["runs"] == 0
        with pytest.raises(rb.RbfslError) as e:
            pl.remove(7)
        assert e.value.code == rb.RBFSL_E_INVAL
