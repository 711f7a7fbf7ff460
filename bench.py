#!/usr/bin/env python3
"""Throughput of the local-stencil RBF semi-Lagrangian transport step on one
MI355X: departure interpolations per second (N x steps / s).

One step = the whole hot path for every node: RK4 departure point, exact
n-nearest-neighbour stencil, assembly and partial-pivot LU of the augmented
PHS + spherical-harmonic system, back substitution, gather-and-dot apply.
Inputs are synthetic (spherical Fibonacci nodes, analytic flow, Gaussian
fields) and resident in HBM before the timed region.

The headline (the JSON line's value) is the largest configuration that fits
one GPU: N = 655,362 nodes, (n, L, k) = (120, 7, 4) (M = 184 unknowns per
system), eight tracers sharing each step's weights, deformational flow.

Sections (all by default):
  plain   -- the headline: one run, one launch sequence per step;
  c2, c1  -- the same for N = 40,962, (84, 5, 3) and N = 1,024, (31, 3, 2);
  batched -- 64 independent ragged runs advanced together by the pool (one
             search pass and one persistent solve launch per kernel family
             and step, graph-replayed, autotuned), against the same runs
             stepped one after another on the plain path;
  centre  -- the paper's centre-point stencils with every node's factorization
             computed once and replayed each step (N = 40,962);
  pu      -- the N = 40,962 workload interpolated by RBF-PU (patches factored
             once; per step: patch search, patch coefficients,
             partition-of-unity blend);
  served  -- a Poisson stream of transport requests (arrival rate 0.8 x the
             capacity calibrated on the request mix) through the pool's
             continuous-batching loop under a 200 GB HBM budget: p50/p99
             request latency and aggregate throughput, against the same
             requests run one after another on the plain path.

Prints one JSON line.  `--gpus N` with N > 1 is refused: this build runs on a
single GPU (see the design notes on sharding).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_1804_01609_amd as rb  # noqa: E402
from paper_1804_01609_amd import workloads as W  # noqa: E402

METRIC = "departure interpolations/sec (N x steps/s) batched vs plain; p50/p99 run latency"
PEAK_FP64_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz


def say(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(msg, file=sys.stderr, flush=True)


def solve_flops(M):
    """Algorithmic flops of one stencil's elimination + back substitution:
    step k updates M-1-k rows, each one multiplier product and M-k fused
    multiply-adds (columns k+1..M, right-hand side included); unknown k of the
    back substitution costs one product and k fused multiply-adds."""
    elim = sum((M - 1 - k) * (1 + 2 * (M - k)) for k in range(M))
    back = sum(1 + 2 * k for k in range(M))
    return elim + back


def assembly_flops(n, L, k):
    """Algorithmic flops of one stencil's assembly: the symmetric PHS block,
    n^2/2 entries of (10 + k) flops (difference, squared distance, square
    root, k products), and 3 n (L+1)^2 for the harmonic basis block."""
    return n * n * (10 + k) // 2 + 3 * n * (L + 1) ** 2


def stencil_flops(n, L, k):
    return assembly_flops(n, L, k) + solve_flops(n + (L + 1) ** 2)


def solver_sources_sha256(M):
    """Hash of the solver sources the counters were taken on (kernel + instantiation)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1804_01609_amd", "csrc")
    cap = {47: 48, 184: 192}.get(M, M)
    h = hashlib.sha256()
    for f in ("k_solve.h", f"k_solve_m{cap}.hip"):
        path = os.path.join(csrc, f)
        if not os.path.exists(path):
            return None
        h.update(open(path, "rb").read())
    return h.hexdigest()


def measured_traffic(cfg, M, spl):
    """HBM bytes per k_solve launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a known-size copy kernel), or None
    when the summary is missing, the solver sources changed since it was taken,
    or its launches covered another number of steps than `spl`."""
    key = cfg["name"].split("-")[0]
    path = os.path.join(ROOT, "profiles", f"k_solve_{key}_N{cfg['N']}_M{M}_counters.txt")
    if not os.path.exists(path):
        return None
    kv = dict(line.strip().split("=", 1) for line in open(path) if "=" in line and not line.startswith("#"))
    if kv.get("source_sha256") != solver_sources_sha256(M) or int(kv.get("steps_per_launch", 1)) != spl:
        return None
    return float(kv["hbm_bytes_per_launch"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, X, q0, target_s):
    """The oracle, as it stands, on a bounded sample of one step's nodes: on
    all host threads (the value) and on one thread."""
    import oracle
    p = oracle.make_params(cfg["n"], cfg["L"], cfg["k"], 0, cfg["vel_id"], cfg["vp"], cfg["dt"], 0.0, cfg["ntr"])
    rng = np.random.default_rng(0)
    nthr = oracle.threads()

    def rate(threads, seconds, probe):
        oracle.set_threads(threads)
        t = time.perf_counter()
        oracle.step_sample(X, p, 0, rng.integers(0, X.shape[0], probe), q0)
        dt = time.perf_counter() - t
        J = int(min(X.shape[0], max(probe, probe * seconds / max(dt, 1e-6))))
        t = time.perf_counter()
        oracle.step_sample(X, p, 0, rng.integers(0, X.shape[0], J), q0)
        dt = time.perf_counter() - t
        return J / dt, J, dt

    one, J1, t1 = rate(1, target_s / 4, 16)
    allr, J, dt = rate(nthr, target_s, 16 * nthr)
    oracle.set_threads(nthr)
    return {"value": allr, "unit": "interpolations/s", "cores": nthr, "kind": "oracle",
            "single_core_value": one, "cpu_model": cpu_model(),
            "sample": f"one step (step 0) of {cfg['name']} for {J} randomly drawn nodes, {dt:.1f} s on "
                      f"{nthr} OpenMP threads (one thread: {J1} nodes, {t1:.1f} s); per node: brute-force "
                      f"n nearest of all N nodes kept in a heap, assembly, elimination, apply"}


# steps and warm-up steps when not given: the headline configuration is timed
# over a few steps (0.5 s each), the small ones over a full run
STEP_DEFAULTS = {"c1": (128, 10), "c2": (480, 10), "c3": (20, 2)}


def bench_plain(name, steps, warmup, sync):
    """One run of configuration `name`: `steps` timed steps after `warmup`."""
    cfg = W.CONFIGS[name]
    N, n, L, k = cfg["N"], cfg["n"], cfg["L"], cfg["k"]
    M = n + (L + 1) ** 2
    X = W.fibonacci_nodes(N)
    q0 = W.initial_q(cfg, X)
    p = rb.make_params(n, L, k, 0, cfg["vel_id"], cfg["vp"], cfg["dt"], 0.0, cfg["ntr"])
    tr = rb.Transport(X, p)
    tr.set_q(q0)
    if warmup:
        tr.run(warmup)
    tr.profile(True)
    spl = tr.steps_per_launch(steps)
    sync()
    t0 = time.perf_counter()
    tr.run(steps)  # one host synchronisation at the end
    sync()
    t1 = time.perf_counter()
    phase_ms, nrec = tr.phase_times()
    tr.profile(False)
    tr.close()
    elapsed = t1 - t0
    solve_ms = phase_ms[2] / max(nrec, 1)
    fl = stencil_flops(n, L, k) * N
    achieved = fl / (solve_ms * 1e-3) / 1e12
    return {
        "workload": cfg["name"], "N": N, "n": n, "L": L, "k": k, "M": M, "tracers": cfg["ntr"], "dt": cfg["dt"],
        "steps": steps, "warmup": warmup, "value": N * steps / elapsed, "unit": "interpolations/s",
        "ms_per_step": 1e3 * elapsed / steps,
        "phase_ms_per_step": {nm: phase_ms[i] / max(nrec, 1) for i, nm in enumerate(["trace", "knn", "solve", "apply"])},
        "roofline": {"kernel": "k_solve", "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic(cfg, M, spl), "traffic_unit": "bytes/launch",
                     "flops_per_launch": fl * spl, "flops_per_stencil": stencil_flops(n, L, k),
                     "launch_ms": solve_ms * spl, "steps_per_launch": spl},
    }, X, q0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--config", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--sections", default="plain,c2,c1,centre,pu,batched,batched_small,served")
    ap.add_argument("--batched-steps", type=int, default=24)
    ap.add_argument("--served-requests", type=int, default=10)
    ap.add_argument("--served-step-scale", type=float, default=0.25,
                    help="scale of the requests' step counts (1.0: 64..512 steps)")
    ap.add_argument("--served-load", type=float, default=0.8,
                    help="arrival rate as a fraction of the capacity calibrated on the request mix")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run 5 device-to-device copies of BYTES (a known-size copy kernel "
                         "that calibrates the HBM byte counters) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        src = torch.ones(args.calibrate_copy // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": args.calibrate_copy, "copies": 5}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                                   "(multi-GPU sharding is described in the design notes, not built)"}))
        sys.exit(2)

    try:
        import torch
        sync = torch.cuda.synchronize if torch.cuda.is_available() else (lambda: None)
    except Exception:
        sync = lambda: None  # noqa: E731

    steps = args.steps if args.steps is not None else STEP_DEFAULTS.get(args.config, (20, 2))[0]
    warmup = args.warmup if args.warmup is not None else STEP_DEFAULTS.get(args.config, (20, 2))[1]
    head, X, q0 = bench_plain(args.config, steps, warmup, sync)
    cfg = W.CONFIGS[args.config]
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "interpolations/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "N": head["N"], "n": head["n"], "L": head["L"], "k": head["k"],
                   "M": head["M"], "tracers": head["tracers"], "dt": head["dt"],
                   "mode": "plain, one run per launch sequence"},
        "phase_ms_per_step": head["phase_ms_per_step"],
        "roofline": head["roofline"],
    }
    say(f"plain {cfg['name']}: {head['value']:.4g} interpolations/s, {head['ms_per_step']:.3f} ms/step, "
        f"k_solve {head['roofline']['launch_ms']:.2f} ms = {head['roofline']['frac']:.4f} of FP64 peak")
    sections = set(args.sections.split(","))
    for nm in ("c2", "c1"):
        if nm in sections and nm != args.config:
            st, wu = (100, 5) if nm == "c2" else STEP_DEFAULTS[nm]
            r, _, _ = bench_plain(nm, st, wu, sync)
            out[nm] = r
            say(f"plain {r['workload']}: {r['value']:.4g} interpolations/s, {r['ms_per_step']:.3f} ms/step")
    c2 = W.CONFIGS["c2"]
    if "centre" in sections or "pu" in sections:
        X2 = W.fibonacci_nodes(c2["N"])
        q2 = W.initial_q(c2, X2)
    if "centre" in sections:
        out["centre"] = bench_centre(c2, X2, q2, sync)
        say(f"centre (cached factors): {out['centre']['value']:.4g} interpolations/s, "
            f"{out['centre']['ms_per_step']:.3f} ms/step")
    if "pu" in sections:
        out["pu"] = bench_pu(c2, X2, q2, sync)
        say(f"RBF-PU: {out['pu']['value']:.4g} interpolations/s, {out['pu']['ms_per_step']:.3f} ms/step")
    if "batched" in sections:
        out["batched"] = bench_batched(args.batched_steps, sync)
        say(f"batched: {out['batched']['value']:.4g} interpolations/s "
            f"({out['batched']['speedup_vs_plain']:.3f}x the plain path)")
    if "batched_small" in sections:
        out["batched_small"] = bench_batched(args.batched_steps, sync, BATCHED_SMALL)
        say(f"batched, small runs: {out['batched_small']['value']:.4g} interpolations/s "
            f"({out['batched_small']['speedup_vs_plain']:.3f}x the plain path)")
    if "served" in sections:
        out["served"] = bench_served(args.served_requests, args.served_load, args.served_step_scale)
        sv = out["served"]
        say(f"served: p50 {sv['p50_s']:.2f} s, p99 {sv['p99_s']:.2f} s (single-run FIFO on the same arrivals: "
            f"p50 {sv['plain_fifo']['p50_s']:.2f} s, p99 {sv['plain_fifo']['p99_s']:.2f} s; results equal: "
            f"{sv['plain_fifo']['results_equal_pool']})")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, X, q0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_centre(cfg, X, q0, sync, steps=100):
    """C2 with the paper's centre-point stencils (Section 3.3.2) and cached
    factorizations: one factorization per node at create, then per step the
    search for the nearest node, the right-hand side and the stored
    elimination replayed (HBM-bound: 8 M^2 bytes per point)."""
    N, n, L, k = cfg["N"], cfg["n"], cfg["L"], cfg["k"]
    M = n + (L + 1) ** 2
    p = rb.make_params(n, L, k, 1, cfg["vel_id"], cfg["vp"], cfg["dt"], 0.0, cfg["ntr"], cache_factors=1)
    sync()
    t = time.perf_counter()
    tr = rb.Transport(X, p)
    sync()
    create_s = time.perf_counter() - t
    tr.set_q(q0)
    tr.run(2)
    tr.profile(True)
    sync()
    t = time.perf_counter()
    tr.run(steps)
    sync()
    dt = time.perf_counter() - t
    ph, nrec = tr.phase_times()
    tr.close()
    solve_ms = ph[2] / max(nrec, 1)
    bytes_solve = 8.0 * M * M * N
    return {"workload": cfg["name"] + "-centre-point-stencils-cached-factors", "steps": steps,
            "value": N * steps / dt, "unit": "interpolations/s", "ms_per_step": 1e3 * dt / steps,
            "create_s_incl_factorization": create_s, "factor_bytes": 8 * M * M * N,
            "phase_ms_per_step": {nm: ph[i] / max(nrec, 1) for i, nm in enumerate(["trace", "knn", "solve", "apply"])},
            "roofline_solve": {"kernel": "k_solve_cached", "bound": "hbm",
                               "achieved": bytes_solve / (solve_ms * 1e-3) / 1e9, "peak": 8000.0,
                               "unit": "GB/s", "frac": bytes_solve / (solve_ms * 1e-3) / 8e12,
                               "algorithmic_bytes_per_launch": bytes_solve}}


def bench_pu(cfg, X, q0, sync, steps=200, a=2.5):
    """C2's nodes, flow and (n, L, k) with RBF-PU interpolation (Sections 2.3
    and 3.3.3): ceil(a N / n) patches of radius 2 sqrt(n/N) around
    quasi-uniform centres, factored once at create; per step the patch search
    of every departure point, every patch's coefficients from its stored
    factorization (HBM: 8 M_l^2 bytes per patch and tracer) and the
    partition-of-unity blend (FP64 ALU: per containing patch, n_l PHS terms and
    (L+1)^2 basis terms)."""
    N, n, L, k = cfg["N"], cfg["n"], cfg["L"], cfg["k"]
    R = rb.pu_radius(n, N)
    C = W.fibonacci_nodes(rb.pu_count(a, n, N))
    p = rb.make_params(n, L, k, rb.STENCIL_PU, cfg["vel_id"], cfg["vp"], cfg["dt"], 0.0, cfg["ntr"])
    sync()
    t = time.perf_counter()
    tr = rb.PuTransport(X, C, R, p)
    sync()
    create_s = time.perf_counter() - t
    counts, _ = tr.patches()
    tr.set_q(q0)
    tr.run(2)
    tr.profile(True)
    sync()
    t = time.perf_counter()
    tr.run(steps)
    sync()
    dt = time.perf_counter() - t
    ph, nrec = tr.phase_times()
    tr.close()
    mL = (L + 1) ** 2
    coef_ms, eval_ms = ph[2] / max(nrec, 1), ph[3] / max(nrec, 1)
    coef_bytes = 8.0 * float(((counts.astype(np.float64) + mL) ** 2).sum()) * cfg["ntr"]
    return {"workload": f"{cfg['name']}-rbfpu-a{a}", "patches": int(C.shape[0]), "R": R,
            "nodes_per_patch": [int(counts.min()), float(counts.mean()), int(counts.max())],
            "steps": steps, "value": N * steps / dt, "unit": "interpolations/s", "ms_per_step": 1e3 * dt / steps,
            "create_s_incl_factorization": create_s,
            "phase_ms_per_step": {nm: ph[i] / max(nrec, 1)
                                  for i, nm in enumerate(["trace", "patch_search", "coef", "eval"])},
            "roofline_coef": {"kernel": "k_pu_coef", "bound": "hbm",
                              "achieved": coef_bytes / (coef_ms * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                              "frac": coef_bytes / (coef_ms * 1e-3) / 8e12,
                              "algorithmic_bytes_per_launch": coef_bytes}}


def _run_inputs(r):
    X = W.fibonacci_nodes(r["N"])
    p = rb.make_params(r["n"], r["L"], r["k"], 0, r["vel_id"], r["vp"], r["dt"], 0.0, r["ntr"])
    return X, p


BATCHED_C4 = ("c4-batched-64runs-N2048..65536-(31,3,2)/(56,4,2)/(84,5,3)-seed0", dict())
BATCHED_SMALL = ("batched-small-512runs-N256..2048-(31,3,2)/(56,4,2)/(84,5,3)-seed2",
                 dict(count=512, seed=2, nmin=256, nmax=2048))


def bench_batched(steps, sync, which=BATCHED_C4):
    """A batched workload: pool (tuned, graph-replayed) vs the same runs one
    after another on the plain path, `steps` steps each.  C4 (64 runs of
    2,048..65,536 nodes) is the configured one; the small-run mix (512 runs of
    256..2,048 nodes) is where launches, not arithmetic, bound the plain path."""
    name, kw = which
    runs = W.batched_runs(**kw)
    inputs = [(*_run_inputs(r), None) for r in runs]
    inputs = [(X, p, W.run_q0(r, X)) for r, (X, p, _) in zip(runs, inputs)]
    nodes = sum(r["N"] for r in runs)
    with rb.Pool(max_runs=len(runs), hbm_budget=32 << 30) as pl:
        for X, p, q0 in inputs:
            pl.add(X, p, q0, runs[0]["nsteps"])
        t = time.perf_counter()
        trials = pl.tune(trials=1)
        tune_s = time.perf_counter() - t
        pl.step(1)  # warm-up (graph capture)
        t = time.perf_counter()
        pl.step(steps)
        dt_pool = time.perf_counter() - t
        st = pl.stats()
    trs = []
    for X, p, q0 in inputs:  # set-up outside the timed region, as for the pool
        trs.append(rb.Transport(X, p))
        trs[-1].set_q(q0)
    sync()
    t = time.perf_counter()
    for tr in trs:
        tr.run(steps)
    sync()
    dt_plain = time.perf_counter() - t
    for tr in trs:
        tr.close()
    pool_v, plain_v = nodes * steps / dt_pool, nodes * steps / dt_plain
    return {"workload": name,
            "runs": len(runs), "nodes_per_step": nodes, "steps": steps,
            "value": pool_v, "unit": "interpolations/s", "ms_per_step": 1e3 * dt_pool / steps,
            "plain_value": plain_v, "plain_ms_per_step": 1e3 * dt_plain / steps,
            "speedup_vs_plain": pool_v / plain_v, "graph": st["graph"], "blocks": st["blocks"],
            "tune_s": tune_s,
            "tuned": {str(t_["M"]): t_["variant"] for t_ in trials if t_["chosen"]}}


def served_calibration(pairs, N=32768, steps=3):
    """Device ns per interpolation of each (n, L, k) class, measured in the
    pool (one run of N nodes per class, after one warm-up step)."""
    ns = {}
    for n, L, k in pairs:
        X = W.fibonacci_nodes(N)
        p = rb.make_params(n, L, k, 0, W.VEL_DEFORM, W.deform_vp(5.0), 5.0 / 256, 0.0, 1)
        with rb.Pool(max_runs=1, hbm_budget=2 << 30) as pl:
            pl.add(X, p, W.two_gaussians(X)[None], steps + 1)
            pl.step(1)
            t = time.perf_counter()
            pl.step(steps)
            ns[(n, L, k)] = 1e9 * (time.perf_counter() - t) / (N * steps)
    return ns


def bench_served(nreq, load, step_scale):
    """Served workload: Poisson arrivals at `load` x the capacity calibrated on
    the request mix (device time per request from per-class pool throughput),
    continuous batching in the pool under a 200 GB HBM budget."""
    pairs = ((31, 3, 2), (56, 4, 2), (84, 5, 3), (120, 7, 4))
    cal = served_calibration(pairs)
    smin, smax = max(1, int(round(64 * step_scale))), max(1, int(round(512 * step_scale)))
    probe = W.served_requests(nreq, rate=1.0, smin=smin, smax=smax)
    sec = float(np.mean([r["N"] * r["nsteps"] * cal[(r["n"], r["L"], r["k"])] * 1e-9 for r in probe]))
    rate = load / sec
    reqs = W.served_requests(nreq, rate=rate, smin=smin, smax=smax)
    items = []
    for r in reqs:
        X, p = _run_inputs(r)
        items.append(dict(arrival=r["arrival"], nodes=X, params=p, q0=W.request_q0(r, X), nsteps=r["nsteps"]))
    with rb.Pool(max_runs=64, hbm_budget=200 * 10 ** 9, log_requests=True) as pl:
        res, outs, wall = pl.serve(items)
    lat = np.array([x["finished"] - it["arrival"] for x, it in zip(res, items)])
    ok = all(x["status"] == rb.RBFSL_OK for x in res)
    total = sum(it["nodes"].shape[0] * it["nsteps"] for it in items)
    # the same requests on the single-run path, one after another in arrival
    # order (a first-come first-served server): each request's device run time
    # (context creation and the copies excluded), the latencies such a server
    # would give on the same arrivals, and the results, which must be the pool's
    plain_s, same = [], True
    for it, out in zip(items, outs):
        tr = rb.Transport(it["nodes"], it["params"])
        tr.set_q(it["q0"])
        tr.get_q()  # the upload has landed
        t0 = time.perf_counter()
        tr.run(it["nsteps"])  # returns once the run is complete
        plain_s.append(time.perf_counter() - t0)
        say(f"served, single-run path: request {len(plain_s) - 1} took {plain_s[-1]:.2f} s")
        same = same and np.array_equal(tr.get_q(), out)
        tr.close()
    free_at, plain_lat = 0.0, []
    for it, d in zip(items, plain_s):
        start = max(free_at, it["arrival"])
        free_at = start + d
        plain_lat.append(free_at - it["arrival"])
    plain_lat = np.array(plain_lat)
    return {"workload": f"c5-served-{nreq}req-N4096..262144-(31,3,2)/(56,4,2)/(84,5,3)/(120,7,4)"
                        f"-steps{smin}..{smax}-seed1",
            "requests": nreq, "load": load, "rate_per_s": rate, "mean_request_device_s": sec,
            "calibration_ns_per_interp": {f"{n},{L},{k}": v for (n, L, k), v in cal.items()},
            "all_ok": ok, "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "wall_s": wall,
            "value": total / wall, "unit": "interpolations/s", "hbm_budget_bytes": 200 * 10 ** 9,
            "plain_fifo": {"p50_s": float(np.percentile(plain_lat, 50)), "p99_s": float(np.percentile(plain_lat, 99)),
                           "mean_s": float(plain_lat.mean()), "busy_s": float(sum(plain_s)),
                           "interp_per_s_busy": total / sum(plain_s), "results_equal_pool": bool(same)}}


if __name__ == "__main__":
    main()
