"""Pins of the oracle's Gaussian elimination and brute-force neighbour search
against independent references (LAPACK via numpy, numpy sorting, hand-built
tie configurations)."""
import numpy as np
import pytest

import oracle
from paper_1804_01609_amd import workloads as W


@pytest.mark.parametrize("M", [1, 2, 5, 17, 47, 64])
def test_ge_matches_lapack_on_random_systems(M):
    rng = np.random.default_rng(M)
    A = rng.standard_normal((M, M)) + M * np.eye(M) * 0.1
    b = rng.standard_normal(M)
    z, st = oracle.gauss_solve(A, b)
    assert st == oracle.ORC_OK
    ref = np.linalg.solve(A, b)
    assert np.abs(z - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_ge_saddle_system_needs_pivoting():
    # zero diagonal in both blocks: no elimination without row exchanges
    rng = np.random.default_rng(1)
    n, m = 12, 4
    B = rng.standard_normal((n, n))
    A = B + B.T
    np.fill_diagonal(A, 0.0)
    P = rng.standard_normal((n, m))
    K = np.block([[A, P], [P.T, np.zeros((m, m))]])
    r = rng.standard_normal(n + m)
    z, st = oracle.gauss_solve(K, r)
    assert st == oracle.ORC_OK
    ref = np.linalg.solve(K, r)
    assert np.abs(z - ref).max() <= 1e-11 * np.abs(ref).max()


def test_ge_permutation_matrix_is_solved_exactly():
    M = 9
    perm = np.array([3, 7, 0, 8, 1, 5, 2, 6, 4])
    A = np.zeros((M, M))
    A[np.arange(M), perm] = np.arange(1, M + 1, dtype=float)
    b = np.arange(M, dtype=float) + 0.5
    z, st = oracle.gauss_solve(A, b)
    assert st == oracle.ORC_OK
    ref = np.zeros(M)
    ref[perm] = b / np.arange(1, M + 1)
    # multipliers are exact zeros, so only the reciprocal product rounds
    assert np.abs(z - ref).max() <= 2.3e-16 * np.abs(ref).max()


def test_ge_detects_singular_systems():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((6, 6))
    A[4] = A[1]  # duplicated row: exactly singular, elimination hits a 0 pivot
    _, st = oracle.gauss_solve(A, rng.standard_normal(6))
    assert st == oracle.ORC_SINGULAR
    _, st = oracle.gauss_solve(np.zeros((3, 3)), np.ones(3))
    assert st == oracle.ORC_SINGULAR
    B = np.eye(3)
    B[:, 1] = np.nan
    _, st = oracle.gauss_solve(B, np.ones(3))
    assert st == oracle.ORC_SINGULAR


def _numpy_knn(X, q, n):
    d = X - q
    d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    order = np.lexsort((np.arange(X.shape[0]), d2))
    return order[:n], d2[order[:n]]


@pytest.mark.parametrize("N,n", [(1024, 31), (2562, 84), (500, 500)])
def test_knn_matches_numpy_sort(N, n):
    X = W.fibonacci_nodes(N)
    Q = W.random_sphere_points(40, seed=N)
    idx, d2 = oracle.knn(X, Q, n)
    for q in range(Q.shape[0]):
        ref_i, ref_d = _numpy_knn(X, Q[q], n)
        assert np.array_equal(idx[q], ref_i)
        assert np.array_equal(d2[q], ref_d)


def test_knn_ties_break_by_index():
    # octahedron vertices, shuffled: from the pole, the four equatorial
    # vertices are at exactly the same distance
    V = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, -1]], dtype=float)
    perm = np.array([4, 0, 2, 5, 1, 3])
    X = V[perm]
    idx, d2 = oracle.knn(X, np.array([[0.0, 0.0, 1.0]]), 6)
    pole = int(np.where(perm == 0)[0][0])
    south = int(np.where(perm == 5)[0][0])
    eq = sorted(int(i) for i in np.where((perm >= 1) & (perm <= 4))[0])
    assert idx[0].tolist() == [pole] + eq + [south]
    assert d2[0, 0] == 0.0 and np.all(d2[0, 1:5] == 2.0) and d2[0, 5] == 4.0
    # a query exactly at a node returns that node first
    X2 = W.fibonacci_nodes(300)
    idx2, d22 = oracle.knn(X2, X2[[17, 250]], 5)
    assert idx2[0, 0] == 17 and idx2[1, 0] == 250 and d22[0, 0] == 0.0


def test_knn_duplicate_points_ordered_by_index():
    X = W.fibonacci_nodes(64)
    X = np.concatenate([X, X[[10, 3]]])  # nodes 64, 65 duplicate 10 and 3
    idx, _ = oracle.knn(X, X[[10]], 3)
    assert idx[0, :2].tolist() == [10, 64]


@pytest.mark.parametrize("n", [1, 2, 31, 120, 700])
def test_knn_selection_orders_of_arrival(n):
    # the brute force keeps the n smallest keys while it scans the nodes in
    # index order; Fibonacci nodes run from the north to the south pole, so
    # queries at the poles see their neighbours arrive last (south) or first
    # (north), and equatorial ones in the middle of the scan
    X = W.fibonacci_nodes(700)
    Q = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, -1.0, 0.0]])
    Q = np.concatenate([Q, W.random_sphere_points(6, seed=n)])
    idx, d2 = oracle.knn(X, Q, n)
    for q in range(Q.shape[0]):
        ref_i, ref_d = _numpy_knn(X, Q[q], n)
        assert np.array_equal(idx[q], ref_i)
        assert np.array_equal(d2[q], ref_d)
