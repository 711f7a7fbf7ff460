"""Pins of the oracle's RBF-PU interpolation (Section 2.3, eq. bspline,
eq. pu_func, eq. PU_interp) and its SL step (Section 3.3.3, eq. rad_patches,
eq. num_patches) against what the mathematics fixes: the B-spline is the
textbook centred cubic B-spline B(2r); patch membership is the cap
|x - omega| < R by brute force; the interpolant reproduces every polynomial of
degree <= L on the sphere (each patch interpolant reproduces them, and the PU
weights sum to one) and interpolates the data at the nodes; a point outside
every patch is reported; the error of a smooth rotation decreases with N."""
import math

import numpy as np
import oracle
from paper_1804_01609_amd import workloads as W


def textbook_cubic_bspline(x):
    # centred cubic B-spline with knots -2..2 (support |x| < 2)
    x = abs(x)
    if x < 1.0:
        return 2.0 / 3.0 - x * x + 0.5 * x ** 3
    if x < 2.0:
        return (2.0 - x) ** 3 / 6.0
    return 0.0


def test_bspline_is_the_textbook_cubic_bspline_scaled_to_the_unit_support():
    for r in np.concatenate([np.linspace(0.0, 1.2, 241), [0.5 - 1e-12, 0.5 + 1e-12, 1.0 - 1e-9]]):
        assert abs(oracle.bspline(r) - textbook_cubic_bspline(2.0 * r)) <= 4e-16
    assert oracle.bspline(0.0) == 2.0 / 3.0 and oracle.bspline(1.0) == 0.0 and oracle.bspline(3.0) == 0.0
    # C2 at the knot r = 1/2 (one-sided second differences)
    h = 1e-4
    left = (oracle.bspline(0.5 - 2 * h) - 2 * oracle.bspline(0.5 - h) + oracle.bspline(0.5)) / h ** 2
    right = (oracle.bspline(0.5) - 2 * oracle.bspline(0.5 + h) + oracle.bspline(0.5 + 2 * h)) / h ** 2
    assert abs(left - 4.0) < 1e-2 and abs(right - 4.0) < 1e-2


def test_patch_parameters_follow_the_area_estimates():
    assert oracle.pu_radius(84, 23042) == 2.0 * math.sqrt(84 / 23042)
    assert oracle.pu_count(2.5, 84, 23042) == math.ceil(2.5 * 23042 / 84)


def test_patch_membership_is_the_cap_by_brute_force():
    N, n, a = 2562, 31, 2.5
    X = W.fibonacci_nodes(N)
    R = oracle.pu_radius(n, N)
    C = W.fibonacci_nodes(oracle.pu_count(a, n, N))
    counts, off, idx = oracle.pu_patches(X, C, R)
    for l in range(0, C.shape[0], 17):
        d = X - C[l]
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        inside = np.flatnonzero(d2 < R * R)
        want = inside[np.lexsort((inside, d2[inside]))]
        assert np.array_equal(idx[off[l]:off[l + 1]], want)
    # about n nodes per patch (the area estimate of eq. rad_patches)
    assert abs(counts.mean() - n) < 0.1 * n


def _setup(N=2562, n=31, L=3, k=2, a=2.5):
    X = W.fibonacci_nodes(N)
    R = oracle.pu_radius(n, N)
    C = W.fibonacci_nodes(oracle.pu_count(a, n, N))
    return X, C, R, oracle.pu_patches(X, C, R)


def test_reproduces_polynomials_of_degree_L_at_departure_points():
    X, C, R, pt = _setup()
    rng = np.random.default_rng(4)
    coef = rng.standard_normal(10)

    def f(P):  # a polynomial of degree 3 = L in x, y, z
        x, y, z = P[:, 0], P[:, 1], P[:, 2]
        return (coef[0] + coef[1] * x + coef[2] * y * z + coef[3] * x * x * y + coef[4] * z ** 3
                + coef[5] * x * y * z + coef[6] * y * y)

    p = oracle.make_params(31, 3, 2, 0, oracle.VEL_SOLID, W.tc1_vp(), 0.3, 0.0, 1)
    o = oracle.pu_step(X, C, R, pt, p, 2, np.arange(X.shape[0]), f(X)[None])
    assert np.all(o["status"] == 0)
    assert np.abs(o["q"][0] - f(o["xi"])).max() <= 1e-12 * np.abs(f(X)).max()
    # degree L + 1 is not reproduced (the pin above is not trivially satisfied)
    g = X[:, 0] ** 4
    o = oracle.pu_step(X, C, R, pt, p, 2, np.arange(X.shape[0]), g[None])
    assert np.abs(o["q"][0] - o["xi"][:, 0] ** 4).max() > 1e-9


def test_interpolates_at_the_nodes_and_reproduces_constants():
    X, C, R, pt = _setup()
    q = np.exp(-3.0 * ((X - [0.3, -0.5, 0.81]) ** 2).sum(1))
    still = oracle.make_params(31, 3, 2, 0, oracle.VEL_ZERO, (), 0.1, 0.0, 2)
    o = oracle.pu_step(X, C, R, pt, still, 0, np.arange(X.shape[0]), np.stack([q, np.ones_like(q)]))
    assert np.all(o["status"] == 0)
    assert np.abs(o["q"][0] - q).max() <= 1e-13
    assert np.abs(o["q"][1] - 1.0).max() <= 1e-14


def test_point_outside_every_patch_is_reported():
    X = W.fibonacci_nodes(1000)
    C = W.fibonacci_nodes(6)           # too few patches to cover the sphere
    R = oracle.pu_radius(31, 1000)
    pt = oracle.pu_patches(X, C, R)
    p = oracle.make_params(31, 3, 2, 0, oracle.VEL_ZERO, (), 0.1, 0.0, 1)
    counts = pt[0]
    o = oracle.pu_step(X, C, R, pt, p, 0, np.arange(1000), np.ones((1, 1000)))
    covered = np.zeros(1000, bool)
    for l in range(6):
        covered[pt[2][pt[1][l]:pt[1][l + 1]]] = True
    assert counts.sum() > 0 and (~covered).any()
    assert np.all(o["status"][~covered] == oracle.ORC_INVAL)
    assert np.all(o["status"][covered] == 0)


def rodrigues(axis, angle):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def _rotation_error(N, n=31, L=3, k=2, a=2.5, steps=8):
    X = W.fibonacci_nodes(N)
    R = oracle.pu_radius(n, N)
    C = W.fibonacci_nodes(oracle.pu_count(a, n, N))
    vp = W.tc1_vp()
    T = vp[0]
    dt = T / 64
    p = oracle.make_params(n, L, k, 0, oracle.VEL_SOLID, vp, dt, 0.0, 1)
    c0 = np.array([1.0, 0.0, 0.0])
    q0 = np.exp(-4.0 * ((X - c0) ** 2).sum(1))
    q, st, _ = oracle.pu_run(X, C, R, p, q0[None], steps)
    assert st == 0
    back = X @ rodrigues(vp[1:4], -2 * math.pi / T * dt * steps).T
    exact = np.exp(-4.0 * ((back - c0) ** 2).sum(1))
    return np.abs(q[0] - exact).max()


def test_solid_body_rotation_error_decreases_with_N():
    e1, e4 = _rotation_error(1024), _rotation_error(4096)
    assert e4 < 2e-3
    assert e4 < e1 / 3, (e1, e4)
