"""Pins of the oracle's local interpolation weights (eq. rbf_poly and
rbf_poly_linsys) against what the method fixes: reproduction of the degree-L
harmonic space, partition of unity, interpolation at nodes, closed-form special
cases, invariance under basis change and scaling, the paper's coefficient form,
and a 40-digit solve in a different (global) basis."""
import math

import mpmath
import numpy as np
import pytest

import oracle
from paper_1804_01609_amd import workloads as W


def stencil(N, n, q):
    X = W.fibonacci_nodes(N)
    idx, d2 = oracle.knn(X, q[None], n)
    return X[idx[0]], d2[0, -1]


def monomials(L, P):
    out = []
    for a in range(L + 1):
        for b in range(L + 1 - a):
            for c in range(L + 1 - a - b):
                out.append(P[..., 0] ** a * P[..., 1] ** b * P[..., 2] ** c)
    return np.array(out)


# (N, n, L, k): C1, a degree-one case, C2, the batched (56, 4, 2), and C3's
# (120, 7, 4) on its 655,362 nodes, whose system has cond(A~) ~ 1.2e10.  The
# partition-of-unity and reproduction residuals are rows of the system, which
# backward-stable elimination satisfies to a few units of roundoff whatever
# the conditioning (measured at C3: 1.1e-15 and 3.4e-16 sum|w|), so the same
# bounds hold for every case.
CASES = [(1024, 31, 3, 2), (2562, 17, 1, 1), (40962, 84, 5, 3), (4096, 56, 4, 2), (655362, 120, 7, 4)]


@pytest.mark.parametrize("N,n,L,k", CASES)
def test_partition_of_unity_and_harmonic_reproduction(N, n, L, k):
    for q in W.random_sphere_points(6, seed=N + n):
        xs, s2 = stencil(N, n, q)
        w, st = oracle.weights(n, L, k, xs, q, s2, q)
        assert st == oracle.ORC_OK
        assert abs(w.sum() - 1.0) < 2e-14
        F = monomials(L, xs)          # every x^a y^b z^c with a+b+c <= L
        f0 = monomials(L, q[None])[:, 0]
        err = np.abs(F @ w - f0).max()
        assert err < 5e-13 * np.abs(w).sum()


@pytest.mark.parametrize("N,n,L,k", [CASES[0], CASES[2], CASES[4]])
def test_degree_above_L_is_not_reproduced(N, n, L, k):
    # the reproduction pin has teeth: in coordinates centred at xi and scaled
    # by the stencil radius s (the space of degree <= L is invariant under
    # both), every monomial of degree <= L is reproduced to roundoff, while
    # some monomial of degree L + 1 leaves an O(1e-5..1e-3) residual
    # (measured at C1, C2, C3: 7e-4, 1e-5, 1.8e-5 against 7e-16, 2e-14, 1e-13)
    q = W.random_sphere_points(1, seed=3)[0]
    xs, s2 = stencil(N, n, q)
    w, st = oracle.weights(n, L, k, xs, q, s2, q)
    assert st == 0
    Y = (xs - q) / np.sqrt(s2)
    sw = np.abs(w).sum()
    res = []
    for deg in (L, L + 1):
        F = monomials(deg, Y)
        f0 = monomials(deg, np.zeros((1, 3)))[:, 0]
        res.append(np.abs(F @ w - f0).max())
    assert res[0] < 1e-11 * sw
    assert res[1] > 1e-7 * sw


@pytest.mark.parametrize("N,n,L,k", CASES[:2])
def test_interpolation_at_a_node(N, n, L, k):
    X = W.fibonacci_nodes(N)
    j = 123
    idx, d2 = oracle.knn(X, X[[j]], n)
    w, st = oracle.weights(n, L, k, X[idx[0]], X[j], d2[0, -1], X[j])
    assert st == 0 and idx[0, 0] == j
    e = np.zeros(n)
    e[0] = 1.0
    assert np.abs(w - e).max() < 1e-13


def test_single_node_constant_basis_is_nearest_neighbour():
    X = W.fibonacci_nodes(200)
    q = W.random_sphere_points(1, 9)[0]
    xs, s2 = stencil(200, 1, q)
    w, st = oracle.weights(1, 0, 0, xs, q, s2, q)
    assert st == 0 and w.tolist() == [1.0]


def test_four_nodes_degree_one_gives_affine_coordinates():
    # n = (L+1)^2 = 4: the moment conditions force c = 0, so the weights are
    # the unique w with sum w = 1 and sum w x_a = xi  (a 4x4 linear system)
    for seed in range(5):
        q = W.random_sphere_points(1, 100 + seed)[0]
        xs, s2 = stencil(642, 4, q)
        for k in (0, 1):
            w, st = oracle.weights(4, 1, k, xs, q, s2, q)
            assert st == 0
            B = np.vstack([np.ones(4), xs.T])
            ref = np.linalg.solve(B, np.concatenate([[1.0], q]))
            assert np.abs(w - ref).max() < 1e-12 * np.abs(ref).max()


def test_weights_invariant_under_scale():
    q = W.random_sphere_points(1, 5)[0]
    xs, s2 = stencil(1024, 31, q)
    w1, _ = oracle.weights(31, 3, 2, xs, q, s2, q)
    for f in (0.25, 3.0):
        w2, _ = oracle.weights(31, 3, 2, xs, q, s2 * f, q)
        assert np.abs(w1 - w2).max() < 1e-11 * np.abs(w1).max()


def global_basis(L, x):
    """{x^a y^b z^e : e in {0,1}, a+b+e <= L}: a basis of the degree-L
    polynomials restricted to the sphere (z^2 = 1 - x^2 - y^2)."""
    out = []
    for e in (0, 1):
        for d in range(L + 1 - e):
            for a in range(d + 1):
                out.append(x[0] ** a * x[1] ** (d - a) * x[2] ** e)
    return out


def test_paper_coefficient_form_equals_cardinal_weights():
    # the paper solves A~ [c; d] = [f; 0] and evaluates s(xi); the oracle
    # evaluates sum_a w_a f_a.  Build the paper's system independently
    # (global basis, unscaled PHS, LAPACK) and compare.
    n, L, k = 31, 3, 2
    rng = np.random.default_rng(7)
    for q in W.random_sphere_points(3, 21):
        xs, s2 = stencil(1024, n, q)
        w, _ = oracle.weights(n, L, k, xs, q, s2, q)
        mL = (L + 1) ** 2
        A = np.zeros((n + mL, n + mL))
        D = np.linalg.norm(xs[:, None, :] - xs[None, :, :], axis=2)
        A[:n, :n] = D ** (2 * k + 1)
        P = np.array([global_basis(L, x) for x in xs])
        A[:n, n:] = P
        A[n:, :n] = P.T
        f = rng.standard_normal(n)
        cd = np.linalg.solve(A, np.concatenate([f, np.zeros(mL)]))
        s = cd[:n] @ (np.linalg.norm(xs - q, axis=1) ** (2 * k + 1)) + cd[n:] @ np.array(global_basis(L, q))
        assert abs(s - w @ f) < 1e-10 * np.abs(f).max()


def mp_weights(xs, q, n, L, k, dps=40):
    """40-digit weights in the global basis, with the nodes projected exactly
    onto the sphere (the space is defined on the sphere)."""
    mpmath.mp.dps = dps

    def proj(v):
        v = [mpmath.mpf(float(t)) for t in v]
        r = mpmath.sqrt(sum(t * t for t in v))
        return [t / r for t in v]

    xm = [proj(r) for r in xs]
    qm = proj(q)
    mL = (L + 1) ** 2
    M = n + mL
    A = mpmath.zeros(M, M)
    r = mpmath.zeros(M, 1)
    for a in range(n):
        for b in range(n):
            A[a, b] = mpmath.sqrt(sum((xm[a][i] - xm[b][i]) ** 2 for i in range(3))) ** (2 * k + 1)
        P = global_basis(L, xm[a])
        for c in range(mL):
            A[a, n + c] = P[c]
            A[n + c, a] = P[c]
        r[a] = mpmath.sqrt(sum((xm[a][i] - qm[i]) ** 2 for i in range(3))) ** (2 * k + 1)
    Pq = global_basis(L, qm)
    for c in range(mL):
        r[n + c] = Pq[c]
    z = mpmath.lu_solve(A, r)
    return np.array([float(z[a]) for a in range(n)])


# Forward error of the weights is bounded by about cond(A~) u (u = 1.1e-16):
# C1 cond ~ 1e3, C2 ~ 6e7 (cond u = 7e-9), C3 ~ 1.2e10 (cond u = 1.3e-6);
# each tolerance is cond u / 100, well above what is measured (C3: 3e-10) and
# far below the O(1) change a dropped term, wrong sign or index would cause.
@pytest.mark.parametrize("N,n,L,k,tol", [(1024, 31, 3, 2, 1e-12), (40962, 84, 5, 3, 1e-10),
                                         pytest.param(655362, 120, 7, 4, 1e-8, marks=pytest.mark.slow)])
def test_weights_match_40_digit_global_basis_solve(N, n, L, k, tol):
    q = W.random_sphere_points(1, 5)[0]
    xs, s2 = stencil(N, n, q)
    w, st = oracle.weights(n, L, k, xs, q, s2, q)
    assert st == 0
    ref = mp_weights(xs, q, n, L, k)
    assert np.abs(w - ref).max() < tol * np.abs(ref).max()


def test_centre_mode_weights_reproduce_harmonics():
    # the paper's mode: stencil of the nearest node K, centred at x_K, and the
    # interpolant evaluated at xi != x_K
    N, n, L, k = 2562, 31, 3, 2
    X = W.fibonacci_nodes(N)
    for q in W.random_sphere_points(4, 77):
        K, _ = oracle.knn(X, q[None], 1)
        idx, d2 = oracle.knn(X, X[K[0]], n)
        xs = X[idx[0]]
        w, st = oracle.weights(n, L, k, xs, X[K[0, 0]], d2[0, -1], q)
        assert st == 0
        F = monomials(L, xs)
        f0 = monomials(L, q[None])[:, 0]
        assert np.abs(F @ w - f0).max() < 1e-12 * np.abs(w).sum()


def test_duplicate_nodes_are_singular():
    q = W.random_sphere_points(1, 5)[0]
    xs, s2 = stencil(1024, 31, q)
    xs = xs.copy()
    xs[7] = xs[3]
    _, st = oracle.weights(31, 3, 2, xs, q, s2, q)
    assert st == oracle.ORC_SINGULAR
