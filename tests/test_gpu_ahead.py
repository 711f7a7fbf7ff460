"""Runs go in chunks of steps whose searches, solves and field updates overlap
on three streams, small problems with several steps per launch (the
departure points, stencils and weights of a step do not depend on the
transported field): a run of m steps must give, bit for bit, what m single
steps give, in both stencil
modes, with several tracers, across chunk boundaries, with the debug taps
showing the last step.  The single-step path is itself checked against the oracle by
the parity tests (and the 128-step run of the N=1,024 workload against the
oracle's stored result)."""
import sys

import numpy as np
import pytest

import paper_1804_01609_amd as rb
from paper_1804_01609_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def params(n, L, k, mode, ntr, dt, vel=None):
    vel_id, vp = vel if vel is not None else (W.VEL_DEFORM, W.deform_vp())
    return rb.make_params(n, L, k, mode, vel_id, vp, dt, 0.0, ntr)


def both(X, q0, p, nsteps, chunks=None):
    """(run in the given chunks, then nsteps single steps) from the same start"""
    with rb.Transport(X, p) as a:
        a.set_q(q0)
        for c in (chunks or [nsteps]):
            a.run(c)
        ra = (a.get_q(), a.state(), a.departure(), a.stencils(), a.weights())
    with rb.Transport(X, p) as b:
        b.set_q(q0)
        for _ in range(nsteps):
            b.step()
        rb_ = (b.get_q(), b.state(), b.departure(), b.stencils(), b.weights())
    return ra, rb_


CASES = [
    # N, n, L, k, mode, ntr, steps
    (1024, 31, 3, 2, 0, 1, 40),
    (1024, 31, 3, 2, 1, 1, 40),
    (1024, 31, 3, 2, 0, 8, 24),
    (5000, 39, 4, 2, 0, 1, 30),    # chunks of 15, 8, 7 steps
    (2562, 56, 4, 2, 1, 2, 60),
    (70000, 31, 3, 2, 0, 1, 5),    # N > 65,536: step by step
    (70000, 56, 4, 2, 1, 2, 4),
]


@pytest.mark.parametrize("N,n,L,k,mode,ntr,steps", CASES)
def test_run_equals_single_steps(N, n, L, k, mode, ntr, steps):
    say(f"[ahead] N={N} n={n} mode={mode} ntr={ntr} steps={steps}")
    X = W.fibonacci_nodes(N)
    q0 = W.tracer_set(X, ntr)
    (qa, sa, xa, Sa, wa), (qb, sb, xb, Sb, wb) = both(X, q0, params(n, L, k, mode, ntr, 5.0 / 200), steps)
    assert sa == sb
    assert np.array_equal(qa, qb)
    assert np.array_equal(xa, xb) and np.array_equal(Sa, Sb) and np.array_equal(wa, wb)


def test_chunk_boundaries_and_resumed_runs():
    # runs of 300 = 128 + 128 + 44, and 129 = 65 + 32 + 32 then 171 = 86 + 43 + 42 steps
    N, n, L, k = 1024, 31, 3, 2
    X = W.fibonacci_nodes(N)
    q0 = W.c1_bump(X)[None]
    p = params(n, L, k, 0, 1, 2.0 * np.pi / 128, (W.VEL_SOLID, W.tc1_vp()))
    for chunks in ([300], [129, 171]):
        say(f"[ahead] chunks {chunks}")
        (qa, sa, *_), (qb, sb, *_) = both(X, q0, p, 300, chunks)
        assert sa == sb == (300, sb[1])
        assert np.array_equal(qa, qb)


def test_singular_run_stops_at_the_first_step_in_both_paths():
    cfg = W.CONFIGS["c1"]
    X = W.fibonacci_nodes(cfg["N"])
    X = np.concatenate([X, X[[17]]])
    q0 = W.c1_bump(X)[None]
    p = rb.make_params(cfg["n"], cfg["L"], cfg["k"], 0, cfg["vel_id"], cfg["vp"], cfg["dt"], 0.0, 1)
    for nsteps in (1, 5, 200):
        say(f"[ahead] singular run of {nsteps}")
        with rb.Transport(X, p) as tr:
            tr.set_q(q0)
            assert tr.run_status(nsteps) == rb.RBFSL_E_SINGULAR
            assert tr.state()[0] == 0
            assert np.array_equal(tr.get_q(), q0)
            assert tr.failures()[0] > 0
