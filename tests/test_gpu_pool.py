"""GPU tests of the pooled (batched and served) forms through the C ABI.

Every pooled node runs the same arithmetic as the single-run path, so the
pool must reproduce the CPU oracle on small runs and the single-run GPU path
bit for bit on larger ones, whatever solver variant, graph mode, mix of other
runs or admission order it meets."""
import sys

import numpy as np
import pytest

import oracle
import paper_1804_01609_amd as rb
from paper_1804_01609_amd import workloads as W

pytestmark = pytest.mark.gpu

Q_TOL = 1e-9


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_spec(N, n, L, k, deform, seed, nsteps, ntr=1, T=None):
    """A seeded run description (flow axis and period from splitmix64)."""
    g = W.SplitMix64(seed)
    alpha, beta = np.pi * g.uniform(), 2 * np.pi * g.uniform()
    T = T if T is not None else 1.0 + 9.0 * g.uniform()
    ax = (np.sin(alpha) * np.cos(beta), np.sin(alpha) * np.sin(beta), np.cos(alpha))
    if deform:
        vel_id, vp = W.VEL_DEFORM, W.deform_vp(T, ax)
    else:
        vel_id, vp = W.VEL_SOLID, W.solid_body_vp(T, alpha, beta)
    X = W.fibonacci_nodes(N)
    fields = W.tracer_set(X, 8)
    q0 = np.stack([fields[(seed + t) % 8] for t in range(ntr)])
    return dict(X=X, q0=q0, n=n, L=L, k=k, vel_id=vel_id, vp=vp, dt=T / 256, nsteps=nsteps, ntr=ntr)


def gparams(r):
    return rb.make_params(r["n"], r["L"], r["k"], 0, r["vel_id"], r["vp"], r["dt"], 0.0, r["ntr"])


def oparams(r):
    return oracle.make_params(r["n"], r["L"], r["k"], 0, r["vel_id"], r["vp"], r["dt"], 0.0, r["ntr"])


def plain(r, nsteps=None):
    with rb.Transport(r["X"], gparams(r)) as tr:
        tr.set_q(r["q0"])
        code = tr.run_status(r["nsteps"] if nsteps is None else nsteps)
        return tr.get_q(), code, tr.state()[0]


def test_pool_matches_oracle_small_mix():
    specs = [run_spec(600, 31, 3, 2, False, 1, 7), run_spec(900, 56, 4, 2, True, 2, 5),
             run_spec(700, 84, 5, 3, True, 3, 6, ntr=2), run_spec(800, 120, 7, 4, True, 4, 3)]
    say("[pool] oracle mix", [(r["X"].shape[0], r["n"], r["nsteps"]) for r in specs])
    with rb.Pool(max_runs=8, hbm_budget=1 << 30) as pl:
        ids = [pl.add(r["X"], gparams(r), r["q0"], r["nsteps"]) for r in specs]
        pl.step(10)
        for r, i in zip(specs, ids):
            steps, want, code = pl.info(i)
            assert (steps, code) == (r["nsteps"], rb.RBFSL_OK)
            q = pl.get_q(i)
            qo, st, _ = oracle.run(r["X"], oparams(r), r["q0"], r["nsteps"])
            assert st == 0
            err = float(np.abs(q - qo).max())
            say(f"  N={r['X'].shape[0]} n={r['n']} max|q_pool - q_oracle| = {err:.3e}")
            assert err <= Q_TOL
            assert np.array_equal(q, qo)


def test_pool_equals_plain_path_every_variant():
    specs = [run_spec(5000, 31, 3, 2, True, 11, 12), run_spec(7000, 56, 4, 2, True, 12, 12, ntr=3),
             run_spec(6000, 84, 5, 3, True, 13, 12), run_spec(3000, 120, 7, 4, True, 14, 6)]
    ref = []
    for r in specs:
        say("[pool] plain reference", r["X"].shape[0], r["n"])
        q, code, _ = plain(r)
        assert code == rb.RBFSL_OK
        ref.append(q)
    variants = rb.pool_variants()
    sizes = [r["n"] + (r["L"] + 1) ** 2 for r in specs]
    # every variant able to solve each size, one pool per choice
    for pick in range(max(len([v for v in variants if v["mcap"] >= M]) for M in sizes)):
        with rb.Pool(max_runs=8, hbm_budget=2 << 30, use_graph=(pick % 2 == 0)) as pl:
            chosen = []
            for M in sizes:
                fit = [v["index"] for v in variants if v["mcap"] >= M]
                chosen.append(fit[min(pick, len(fit) - 1)])
                pl.set_variant(M, chosen[-1])
            say("[pool] variants", chosen, "graph" if pick % 2 == 0 else "direct")
            ids = [pl.add(r["X"], gparams(r), r["q0"], r["nsteps"]) for r in specs]
            pl.step(12)
            for r, i, qr in zip(specs, ids, ref):
                assert pl.info(i)[2] == rb.RBFSL_OK
                assert np.array_equal(pl.get_q(i), qr), (r["n"], chosen)


def test_pool_ragged_lengths_admission_and_removal():
    a = run_spec(4000, 84, 5, 3, True, 21, 9)
    b = run_spec(9000, 31, 3, 2, False, 22, 4)
    c = run_spec(2500, 56, 4, 2, True, 23, 6)
    say("[pool] ragged")
    with rb.Pool(max_runs=2, hbm_budget=1 << 30) as pl:
        ia = pl.add(a["X"], gparams(a), a["q0"], a["nsteps"])
        ib = pl.add(b["X"], gparams(b), b["q0"], b["nsteps"])
        with pytest.raises(rb.RbfslError) as e:
            pl.add(c["X"], gparams(c), c["q0"], c["nsteps"])
        assert e.value.code == rb.RBFSL_E_BUDGET
        pl.step(3)
        assert pl.info(ia)[0] == 3 and pl.info(ib)[0] == 3
        pl.step(5)  # b stops at its own 4 steps
        assert pl.info(ia)[0] == 8 and pl.info(ib)[0] == 4
        assert np.array_equal(pl.get_q(ib), plain(b)[0])
        pl.remove(ib)
        ic = pl.add(c["X"], gparams(c), c["q0"], c["nsteps"])  # joins a run in flight
        pl.step(10)
        assert pl.info(ia)[0] == 9 and pl.info(ic)[0] == 6
        assert np.array_equal(pl.get_q(ia), plain(a)[0])
        assert np.array_equal(pl.get_q(ic), plain(c)[0])


def test_pool_budget_is_enforced():
    a = run_spec(20000, 84, 5, 3, True, 31, 4)
    need = rb.pool_run_bytes(20000, gparams(a), 4)
    say("[pool] budget", need)
    with rb.Pool(max_runs=8, hbm_budget=int(need * 1.5)) as pl:
        ia = pl.add(a["X"], gparams(a), a["q0"], 4)
        with pytest.raises(rb.RbfslError) as e:
            pl.add(a["X"], gparams(a), a["q0"], 4)
        assert e.value.code == rb.RBFSL_E_BUDGET
        assert pl.stats()["bytes_used"] >= need
        pl.remove(ia)
        assert pl.stats()["bytes_used"] == 0
        ib = pl.add(a["X"], gparams(a), a["q0"], 4)
        pl.step(4)
        assert np.array_equal(pl.get_q(ib), plain(a)[0])


def test_pool_singular_run_fails_alone():
    good = run_spec(3000, 56, 4, 2, True, 41, 5)
    bad = run_spec(1500, 31, 3, 2, False, 42, 5)
    bad["X"] = np.concatenate([bad["X"], bad["X"][[17]]])
    bad["q0"] = np.concatenate([bad["q0"], bad["q0"][:, [17]]], axis=1)
    say("[pool] singular")
    q_plain, code, step = plain(bad)
    assert code == rb.RBFSL_E_SINGULAR
    with rb.Pool(max_runs=4, hbm_budget=1 << 30) as pl:
        ig = pl.add(good["X"], gparams(good), good["q0"], 5)
        ib = pl.add(bad["X"], gparams(bad), bad["q0"], 5)
        pl.step(5)
        sb = pl.info(ib)
        assert sb[2] == rb.RBFSL_E_SINGULAR and sb[0] == step
        assert np.array_equal(pl.get_q(ib), q_plain)
        assert pl.info(ig) == (5, 5, rb.RBFSL_OK)
        assert np.array_equal(pl.get_q(ig), plain(good)[0])


def test_pool_tuner_keeps_results():
    specs = [run_spec(6000, 31, 3, 2, True, 51, 3), run_spec(6000, 84, 5, 3, True, 52, 3)]
    say("[pool] tune")
    with rb.Pool(max_runs=4, hbm_budget=1 << 30) as pl:
        ids = [pl.add(r["X"], gparams(r), r["q0"], r["nsteps"]) for r in specs]
        trials = pl.tune(trials=1)
        sizes = {t["M"] for t in trials}
        assert sizes == {47, 120}
        for M in sizes:
            assert sum(t["chosen"] for t in trials if t["M"] == M) == 1
        say("  ", [(t["M"], t["variant"], round(t["ms_per_step"], 3), t["chosen"]) for t in trials])
        pl.step(3)
        for r, i in zip(specs, ids):
            assert pl.info(i)[:2] == (3, 3)
            assert np.array_equal(pl.get_q(i), plain(r)[0])


def test_served_results_equal_alone_and_in_the_mix():
    reqs = W.served_requests(10, rate=40.0, seed=5, nmin=1500, nmax=6000, smin=4, smax=12)
    say("[serve] mix", [(r["N"], r["n"], r["nsteps"], r["ntr"]) for r in reqs])
    items = []
    for r in reqs:
        X = W.fibonacci_nodes(r["N"])
        items.append(dict(arrival=r["arrival"], nodes=X,
                          params=rb.make_params(r["n"], r["L"], r["k"], 0, r["vel_id"], r["vp"], r["dt"], 0.0,
                                                r["ntr"]),
                          q0=W.request_q0(r, X), nsteps=r["nsteps"]))
    # budget for about three runs at once: admissions wait for retirements
    big = max(rb.pool_run_bytes(it["nodes"].shape[0], it["params"], it["nsteps"]) for it in items)
    with rb.Pool(max_runs=4, hbm_budget=3 * big) as pl:
        res, outs, wall = pl.serve(items)
    say(f"  wall {wall:.3f} s")
    for it, r, q in zip(items, res, outs):
        assert r["status"] == rb.RBFSL_OK and r["steps"] == it["nsteps"]
        assert r["admitted"] >= it["arrival"] - 1e-6 and r["finished"] >= r["admitted"]
        with rb.Transport(it["nodes"], it["params"]) as tr:
            tr.set_q(it["q0"])
            tr.run(it["nsteps"])
            alone = tr.get_q()
        assert np.array_equal(q, alone)
        # and the oracle on the same request: a fault shared by both GPU
        # paths (search, solver, apply) cannot hide behind the comparison above
        pr = it["params"]
        op = oracle.make_params(pr.n, pr.L, pr.k, 0, pr.velocity_id, list(pr.vel), pr.dt, pr.t0, pr.n_tracers)
        qo, st, _ = oracle.run(it["nodes"], op, it["q0"], it["nsteps"])
        assert st == oracle.ORC_OK
        assert np.abs(q - qo).max() <= 1e-9
        assert np.array_equal(q, qo)


def test_served_small_request_passes_a_large_one():
    # both arrive at once; the small one has far less remaining work, so the
    # scheduler steps it alone and it completes first, while the large one's
    # state waits untouched: both results are still the ones they get alone
    specs = [(60000, 84, 5, 3, 40), (2000, 31, 3, 2, 40)]
    items = []
    for N, n, L, k, ns in specs:
        X = W.fibonacci_nodes(N)
        p = rb.make_params(n, L, k, 0, W.VEL_DEFORM, W.deform_vp(5.0), 5.0 / 80, 0.0, 1)
        items.append(dict(arrival=0.0, nodes=X, params=p, q0=W.two_gaussians(X)[None], nsteps=ns))
    say("[serve] large and small at t = 0")
    with rb.Pool(max_runs=4, hbm_budget=4 << 30) as pl:
        res, outs, _ = pl.serve(items)
    big, small = res
    say(f"  finished: large {big['finished']:.3f} s, small {small['finished']:.3f} s")
    assert big["status"] == small["status"] == rb.RBFSL_OK
    assert big["steps"] == small["steps"] == 40
    assert small["finished"] < big["finished"]
    for it, q in zip(items, outs):
        with rb.Transport(it["nodes"], it["params"]) as tr:
            tr.set_q(it["q0"])
            tr.run(it["nsteps"])
            assert np.array_equal(q, tr.get_q())
