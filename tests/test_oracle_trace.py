"""Pins of the oracle's velocity fields and RK4 departure tracer (Section 3.2)
against closed forms, an independent high-order ODE integration (scipy
DOP853) and the defining stream function."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_1804_01609_amd import workloads as W


def rodrigues(axis, angle):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def test_zero_flow_departure_is_the_projected_node():
    X = W.fibonacci_nodes(777)
    xi = oracle.trace(X, oracle.VEL_ZERO, [], 0.0, 0.1, 3)
    ref = X / np.linalg.norm(X, axis=1, keepdims=True)
    assert np.abs(xi - ref).max() <= 2.3e-16


def test_solid_body_departure_matches_rotation():
    X = W.fibonacci_nodes(1024)
    vp = W.tc1_vp()
    T = vp[0]
    dt = T / 128.0
    for m in (0, 77):
        xi = oracle.trace(X, oracle.VEL_SOLID, vp, 0.0, dt, m)
        R = rodrigues(vp[1:4], -2 * math.pi / T * dt)  # back by one step
        ref = X @ R.T
        err = np.abs(xi - ref).max()
        # RK4 local error for rotation at rate w: ~ (w dt)^5 / 120
        wdt = 2 * math.pi / T * dt
        assert err <= wdt ** 5 / 120 * 2 + 1e-15
        assert np.abs(np.linalg.norm(xi, axis=1) - 1).max() <= 4.5e-16


def _psi(x, t, vp):
    """the stream function of the deformational flow, from its definition"""
    T, a, kap = vp[0], np.asarray(vp[1:4]), vp[4]
    R = rodrigues(a, 2 * math.pi / T * t)
    y = R.T @ x
    return kap * math.cos(math.pi * t / T) * (y[0] * y[1] * y[2] + 0.5 * y[2] ** 2 * y[0])


@pytest.mark.parametrize("axis", [(0, 0, 1), (0.3, -0.5, 0.8)])
def test_deformational_velocity_is_x_cross_grad_psi_plus_rotation(axis):
    vp = W.deform_vp(5.0, axis)
    a = np.asarray(vp[1:4])
    Om = 2 * math.pi / vp[0]
    rng = np.random.default_rng(3)
    h = 1e-5
    for x in W.random_sphere_points(12, 4):
        t = float(rng.uniform(0, 5))
        g = np.zeros(3)
        for i in range(3):
            e = np.zeros(3)
            e[i] = h
            g[i] = (_psi(x + e, t, vp) - _psi(x - e, t, vp)) / (2 * h)
        ref = np.cross(x, g) + Om * np.cross(a, x)
        u = oracle.velocity(oracle.VEL_DEFORM, vp, t, x)
        assert np.abs(u - ref).max() < 1e-8
        assert abs(u @ x) < 1e-14  # tangent to the sphere


def _rhs(vel_id, vp):
    def f(t, y):
        return oracle.velocity(vel_id, vp, t, y)
    return f


def test_deformational_flow_returns_at_T():
    vp = W.deform_vp(5.0, (0.2, 0.4, 0.9))
    for x0 in W.random_sphere_points(4, 11):
        sol = solve_ivp(_rhs(oracle.VEL_DEFORM, vp), (0.0, 5.0), x0, method="DOP853",
                        rtol=1e-12, atol=1e-13)
        assert np.abs(sol.y[:, -1] - x0).max() < 1e-8
        mid = np.abs(sol.y[:, sol.y.shape[1] // 2] - x0).max()
        assert mid > 0.05  # it does move


def test_rk4_departure_converges_at_fifth_order_locally():
    vp = W.deform_vp()
    X = W.fibonacci_nodes(64)[::8]
    errs = []
    for dt in (0.08, 0.04):
        m = 7
        xi = oracle.trace(X, oracle.VEL_DEFORM, vp, 0.0, dt, m)
        t1, t0 = (m + 1) * dt, m * dt
        e = 0.0
        for j in range(X.shape[0]):
            sol = solve_ivp(_rhs(oracle.VEL_DEFORM, vp), (t1, t0), X[j], method="DOP853",
                            rtol=1e-13, atol=1e-14)
            ref = sol.y[:, -1] / np.linalg.norm(sol.y[:, -1])
            e = max(e, np.abs(xi[j] - ref).max())
        errs.append(e)
    assert errs[0] < 1e-6
    assert errs[0] / errs[1] > 16.0  # ~2^5 for a fifth-order local error
