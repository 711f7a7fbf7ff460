"""GPU parity at the configured sizes: full runs against the oracle's stored
result, every step of a C2 run and the first steps of C3 on sampled nodes
(the oracle fed the GPU's own q^m, so every step is checked on its own), each
compiled solver capacity against the oracle, and the largest harmonic degree
in the cached-factor mode.

Bar: stencil indices bit-exact; weights within 1e-11 relative and q within
1e-9 absolute (Algorithm 1 over the whole run); both sides perform the same
correctly rounded operations in the same order, so the tests also assert bit
equality."""
import importlib.util
import json
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1804_01609_amd as rb
from paper_1804_01609_amd import workloads as W

pytestmark = pytest.mark.gpu

W_TOL = 1e-11
Q_TOL = 1e-9
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _golden_module():
    spec = importlib.util.spec_from_file_location("make_full_run_golden",
                                                  os.path.join(GOLDEN, "make_full_run_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def gpu_params(cfg, mode=0, ntr=None, **kw):
    return rb.make_params(cfg["n"], cfg["L"], cfg["k"], mode, cfg["vel_id"], cfg["vp"], cfg["dt"], 0.0,
                          ntr if ntr is not None else cfg["ntr"], **kw)


def orc_params(cfg, mode=0, ntr=None):
    return oracle.make_params(cfg["n"], cfg["L"], cfg["k"], mode, cfg["vel_id"], cfg["vp"], cfg["dt"],
                              0.0, ntr if ntr is not None else cfg["ntr"])


# ---------------------------------------------------------------- full runs

@pytest.mark.parametrize("name", ["c1", "c2"])
def test_full_run_matches_stored_oracle_result(name):
    g = _golden_module()
    qpath, jpath = g.paths(name)
    with open(jpath) as f:
        meta = json.load(f)
    cfg = W.CONFIGS[name]
    X = W.fibonacci_nodes(cfg["N"])
    q0 = W.initial_q(cfg, X)
    assert g.input_hash(cfg, X, q0) == meta["input_sha256"], "inputs changed: regenerate the stored result"
    qo = np.load(qpath, allow_pickle=False)
    say(f"[size] {name}: full run of {cfg['nsteps']} steps, N={cfg['N']}")
    with rb.Transport(X, gpu_params(cfg)) as tr:
        tr.set_q(q0)
        tr.run(cfg["nsteps"])
        assert tr.state()[0] == cfg["nsteps"]
        qg = tr.get_q()
    err = float(np.abs(qg - qo).max())
    say(f"  max |q_gpu - q_oracle| = {err:.3e}")
    assert err <= Q_TOL
    assert np.array_equal(qg, qo)


# ---------------------------------------------------------------- every step, sampled

def _stepwise(cfg, steps, per_step, seed):
    """Run `steps` steps one at a time; after each, compare the departure
    points, stencils, weights and q^{m+1} of `per_step` random nodes with the
    oracle's step m from the same q^m."""
    X = W.fibonacci_nodes(cfg["N"])
    op = orc_params(cfg)
    rng = np.random.default_rng(seed)
    worst_w, worst_q = 0.0, 0.0
    with rb.Transport(X, gpu_params(cfg)) as tr:
        tr.set_q(W.initial_q(cfg, X))
        for m in range(steps):
            qm = tr.get_q()
            tr.step()
            q1 = tr.get_q()
            jl = np.sort(rng.choice(cfg["N"], per_step, replace=False)).astype(np.int64)
            xi, S, w = tr.sample(jl)
            o = oracle.step_sample(X, op, m, jl, qm)
            assert np.all(o["status"] == 0)
            assert np.array_equal(xi, o["xi"]), f"departure points differ at step {m}"
            assert np.array_equal(S, o["S"]), f"stencils differ at step {m}"
            worst_w = max(worst_w, rel_err(w, o["w"]))
            worst_q = max(worst_q, float(np.abs(q1[:, jl] - o["q"]).max()))
            assert worst_w <= W_TOL and worst_q <= Q_TOL, f"step {m}"
            assert np.array_equal(w, o["w"]), f"weights differ in the last bits at step {m}"
            assert np.array_equal(q1[:, jl], o["q"]), f"q differs in the last bits at step {m}"
            if m % 40 == 39:
                say(f"  step {m + 1}/{steps} ok")
    return worst_w, worst_q


def test_c2_every_step_on_sampled_nodes():
    cfg = W.CONFIGS["c2"]
    say(f"[size] c2: all {cfg['nsteps']} steps, 64 sampled nodes each")
    ww, wq = _stepwise(cfg, cfg["nsteps"], 64, seed=20)
    say(f"  worst weight rel err {ww:.2e}, worst q err {wq:.2e}")


def test_c3_first_forty_steps_on_sampled_nodes():
    cfg = W.CONFIGS["c3"]
    say("[size] c3: 40 steps, 64 sampled nodes each, 8 tracers")
    ww, wq = _stepwise(cfg, 40, 64, seed=30)
    say(f"  worst weight rel err {ww:.2e}, worst q err {wq:.2e}")


# ---------------------------------------------------------------- each solver capacity

# (N, n, L, k): systems of n + (L+1)^2 unknowns that land in every compiled
# capacity (48, 64, 81, 96, 120, 128, 192); 1,500 systems per launch, more
# than the 1,024 up to which the smallest capacity uses four waves per system
CAPACITY_CASES = [(10242, 31, 3, 2), (10242, 39, 4, 2), (10242, 56, 4, 2), (20000, 60, 5, 3),
                  (40962, 84, 5, 3), (20000, 79, 6, 3), (655362, 120, 7, 4), (40962, 90, 8, 4)]


@pytest.mark.parametrize("N,n,L,k", CAPACITY_CASES)
def test_weights_each_capacity_against_oracle(N, n, L, k):
    count = 1500
    say(f"[size] weights N={N} n={n} L={L} k={k} M={n + (L + 1) ** 2} count={count}")
    X = W.fibonacci_nodes(N)
    Qp = W.random_sphere_points(count, seed=N + 7 * n + L)
    idx, d2 = oracle.knn(X, Qp, n)
    s2 = d2[:, -1].copy()
    gw, st = rb.weights(X, idx, Qp, s2, Qp, n, L, k)
    assert np.all(st == 0)
    ow = np.zeros_like(gw)
    for t in range(count):
        ow[t], ost = oracle.weights(n, L, k, X[idx[t]], Qp[t], s2[t], Qp[t])
        assert ost == 0
    assert rel_err(gw, ow) <= W_TOL
    assert np.array_equal(gw, ow)


def test_cached_factors_at_degree_eight():
    # (n, L) = (90, 8): 81 harmonic terms, the most a system of at most 192
    # unknowns can carry, through the stored-factorization replay
    N, n, L, k = 10242, 90, 8, 4
    cfg = dict(n=n, L=L, k=k, vel_id=W.VEL_DEFORM, vp=W.deform_vp(), dt=5.0 / 200, ntr=2)
    X = W.fibonacci_nodes(N)
    q0 = W.tracer_set(X, 2)
    say(f"[size] cached factors n={n} L={L}")
    out = {}
    for cache in (0, 1):
        with rb.Transport(X, gpu_params(cfg, 1, cache_factors=cache)) as tr:
            tr.set_q(q0)
            tr.run(3)
            qm = tr.get_q()
            tr.step()
            jl = np.arange(0, N, 37, dtype=np.int64)
            out[cache] = (qm, tr.get_q(), tr.sample(jl), jl)
    assert np.array_equal(out[0][1], out[1][1])
    qm, q1, (xi, S, w), jl = out[1]
    o = oracle.step_sample(X, orc_params(cfg, 1), 3, jl, qm)
    assert np.all(o["status"] == 0)
    assert np.array_equal(xi, o["xi"]) and np.array_equal(S, o["S"])
    assert rel_err(w, o["w"]) <= W_TOL
    assert np.array_equal(w, o["w"])
    assert np.array_equal(q1[:, jl], o["q"])
