"""Pins of the oracle's NL2010 deformational flow (Section 4.2) and of its
Fehlberg RK5 departure tracer (Section 3.2) against the flow's definition in
longitude/latitude components, its reversal at t = T (an independent DOP853
integration), the divergence of the spherical form, the closed-form solid-body
rotation and the integrator's order."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from paper_1804_01609_amd import workloads as W

T = 5.0


def spherical_velocity(x, t):
    """u from the longitude/latitude components of the NL2010 flow (with
    sin(2 lambda') in the latitude component) and the local basis vectors."""
    lam = math.atan2(x[1], x[0])
    th = math.asin(max(-1.0, min(1.0, x[2])))
    w = 2 * math.pi / T
    K = 10.0 / T * math.cos(math.pi * t / T)
    lp = lam - w * t
    ul = K * math.sin(lp) ** 2 * math.sin(2 * th) + w * math.cos(th)
    vt = K * math.sin(2 * lp) * math.cos(th)
    e_l = np.array([-math.sin(lam), math.cos(lam), 0.0])
    e_t = np.array([-math.sin(th) * math.cos(lam), -math.sin(th) * math.sin(lam), math.cos(th)])
    return ul * e_l + vt * e_t


def test_cartesian_form_matches_the_longitude_latitude_definition():
    vp = W.nl2010_vp()
    X = W.random_sphere_points(400, 11)
    X = X[np.abs(X[:, 2]) < 0.995]
    for t in (0.0, 0.7, 2.5, 3.9, 5.0):
        for x in X[:80]:
            u = oracle.velocity(oracle.VEL_NL2010, vp, t, x)
            ref = spherical_velocity(x, t)
            assert np.abs(u - ref).max() <= 2e-14 * max(1.0, np.abs(ref).max())
            assert abs(float(u @ x)) <= 1e-14  # tangent


def test_spherical_form_is_divergence_free():
    # surface divergence (1/cos th) [d u_l / d lam + d (v cos th) / d th] of the
    # oracle's velocity, by central differences in longitude and latitude
    vp = W.nl2010_vp()
    h = 1e-5
    rng = np.random.default_rng(2)

    def comps(lam, th, t):
        x = np.array([math.cos(th) * math.cos(lam), math.cos(th) * math.sin(lam), math.sin(th)])
        u = oracle.velocity(oracle.VEL_NL2010, vp, t, x)
        e_l = np.array([-math.sin(lam), math.cos(lam), 0.0])
        e_t = np.array([-math.sin(th) * math.cos(lam), -math.sin(th) * math.sin(lam), math.cos(th)])
        return float(u @ e_l), float(u @ e_t)

    for _ in range(20):
        lam, th, t = rng.uniform(-3, 3), rng.uniform(-1.3, 1.3), rng.uniform(0, 5)
        dul = (comps(lam + h, th, t)[0] - comps(lam - h, th, t)[0]) / (2 * h)
        dvc = (comps(lam, th + h, t)[1] * math.cos(th + h) - comps(lam, th - h, t)[1] * math.cos(th - h)) / (2 * h)
        assert abs((dul + dvc) / math.cos(th)) <= 1e-7


def test_flow_returns_every_parcel_at_t_equals_T():
    vp = W.nl2010_vp()
    for x0 in W.random_sphere_points(6, 5):
        sol = solve_ivp(lambda t, x: oracle.velocity(oracle.VEL_NL2010, vp, t, x / np.linalg.norm(x)),
                        (0.0, T), x0, method="DOP853", rtol=1e-12, atol=1e-13)
        assert np.abs(sol.y[:, -1] - x0).max() <= 1e-8
        # and it really moves: half way, far from the start
        mid = solve_ivp(lambda t, x: oracle.velocity(oracle.VEL_NL2010, vp, t, x / np.linalg.norm(x)),
                        (0.0, T / 2), x0, method="DOP853", rtol=1e-12, atol=1e-13)
        assert np.linalg.norm(mid.y[:, -1] - x0) > 0.05


def rodrigues(axis, angle):
    a = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def test_rk5_solid_body_matches_rotation():
    X = W.fibonacci_nodes(512)
    vp = W.tc1_vp()
    Tp = vp[0]
    for dt in (Tp / 32, Tp / 64):
        xi = oracle.trace(X, oracle.VEL_SOLID, vp, 0.0, dt, 3, rk=oracle.RK5F)
        ref = X @ rodrigues(vp[1:4], -2 * math.pi / Tp * dt).T
        wdt = 2 * math.pi / Tp * dt
        # fifth-order formula: local error ~ (w dt)^6 / 720
        assert np.abs(xi - ref).max() <= 4 * wdt ** 6 / 720 + 1e-15
        assert np.abs(np.linalg.norm(xi, axis=1) - 1).max() <= 4.5e-16


def _exact_departure(x, t1, dt, vp):
    sol = solve_ivp(lambda t, y: oracle.velocity(oracle.VEL_NL2010, vp, t, y / np.linalg.norm(y)),
                    (t1, t1 - dt), x, method="DOP853", rtol=1e-13, atol=1e-14)
    y = sol.y[:, -1]
    return y / np.linalg.norm(y)


def test_rk5_local_error_is_sixth_order_and_beats_rk4():
    vp = W.nl2010_vp()
    X = W.random_sphere_points(5, 8)
    X = X[np.abs(X[:, 2]) < 0.9]
    errs = {oracle.RK4: [], oracle.RK5F: []}
    for dt in (0.02, 0.01):  # in the asymptotic range of both formulas
        m = 7  # step from t = 8 dt back to 7 dt
        for rk in (oracle.RK4, oracle.RK5F):
            xi = oracle.trace(X, oracle.VEL_NL2010, vp, 0.0, dt, m, rk=rk)
            ref = np.array([_exact_departure(x, (m + 1) * dt, dt, vp) for x in X])
            errs[rk].append(np.abs(xi - ref).max())
    r5 = errs[oracle.RK5F][0] / errs[oracle.RK5F][1]
    r4 = errs[oracle.RK4][0] / errs[oracle.RK4][1]
    assert 48 <= r5 <= 96, r5      # local error O(dt^6): ratio ~ 64
    assert 24 <= r4 <= 48, r4      # local error O(dt^5): ratio ~ 32
    assert errs[oracle.RK5F][0] < errs[oracle.RK4][0]


def test_rk5_tableau_is_consistent():
    # one step of the formula for a uniform rotation (a linear ODE, where the
    # order conditions reduce to the Taylor series of the exponential) agrees
    # with the exact angle through the dt^5 term
    x = np.array([1.0, 0.0, 0.0])
    vp = [2 * math.pi, 0.0, 0.0, 1.0]
    dt = 0.3
    xi = oracle.trace(x[None], oracle.VEL_SOLID, vp, 0.0, dt, 0, rk=oracle.RK5F)[0]
    err = abs(math.atan2(xi[1], xi[0]) + dt)
    assert err <= dt ** 6 / 720 * 2
