#!/usr/bin/env python3
"""Throughput of the local-stencil RBF semi-Lagrangian transport step on one
MI355X: departure interpolations per second (N x steps / s).

One step = the whole hot path for every node: RK4 departure point, exact
n-nearest-neighbour stencil, assembly and partial-pivot LU of the augmented
PHS + spherical-harmonic system, back substitution, gather-and-dot apply.
Inputs are synthetic (spherical Fibonacci nodes, analytic flow, Gaussian
fields) and resident in HBM before the timed region.

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


def solve_flops(M):
    """Algorithmic flops of one stencil's elimination + back substitution:
    step k updates M-1-k rows, each one multiplier product and M-k fused
    multiply-adds (columns k+1..M, right-hand side included); unknown k of the
    back substitution costs one product and k fused multiply-adds."""
    elim = sum((M - 1 - k) * (1 + 2 * (M - k)) for k in range(M))
    back = sum(1 + 2 * k for k in range(M))
    return elim + back


def solver_sources_sha256(M):
    """Hash of the solver sources the counters were taken on (kernel + instantiation)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1804_01609_amd", "csrc")
    cap = {47: 48}.get(M, M)
    h = hashlib.sha256()
    for f in ("k_solve.h", f"k_solve_m{cap}.hip"):
        path = os.path.join(csrc, f)
        if not os.path.exists(path):
            return None
        h.update(open(path, "rb").read())
    return h.hexdigest()


def measured_traffic(cfg_key, M):
    """HBM bytes per k_solve launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a known-size copy kernel), or None
    when the summary is missing or the solver sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"k_solve_{cfg_key}_N40962_M120_counters.txt")
    if cfg_key != "c2" or not os.path.exists(path):
        return None
    kv = dict(line.strip().split("=", 1) for line in open(path) if "=" in line and not line.startswith("#"))
    if kv.get("source_sha256") != solver_sources_sha256(M):
        return None
    return float(kv["hbm_bytes_per_launch"])


def cpu_baseline(cfg, X, q0, target_s):
    """The oracle, as it stands, on a bounded sample of one step's nodes."""
    import oracle
    p = oracle.make_params(cfg["n"], cfg["L"], cfg["k"], 0, cfg["vel_id"], cfg["vp"], cfg["dt"], 0.0, cfg["ntr"])
    rng = np.random.default_rng(0)
    J = 512
    t = time.perf_counter()
    oracle.step_sample(X, p, 0, rng.integers(0, X.shape[0], J), q0)
    dt = time.perf_counter() - t
    J2 = int(min(X.shape[0], max(J, J * target_s / max(dt, 1e-6))))
    jl = rng.integers(0, X.shape[0], J2)
    t = time.perf_counter()
    oracle.step_sample(X, p, 0, jl, q0)
    dt2 = time.perf_counter() - t
    return {"value": J2 / dt2, "unit": "interpolations/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"one step (step 0) of {cfg['name']} for {J2} randomly drawn nodes, "
                      f"{dt2:.1f} s on {oracle.threads()} OpenMP threads"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=480)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
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

    cfg = W.CONFIGS[args.config]
    N, n, L, k = cfg["N"], cfg["n"], cfg["L"], cfg["k"]
    M = n + (L + 1) ** 2
    X = W.fibonacci_nodes(N)
    q0 = W.initial_q(cfg, X)
    p = rb.make_params(n, L, k, 0, cfg["vel_id"], cfg["vp"], cfg["dt"], 0.0, cfg["ntr"])

    try:
        import torch
        sync = torch.cuda.synchronize if torch.cuda.is_available() else (lambda: None)
    except Exception:
        sync = lambda: None  # noqa: E731

    tr = rb.Transport(X, p)
    tr.set_q(q0)
    if args.warmup:
        tr.run(args.warmup)
    tr.profile(True)
    sync()
    t0 = time.perf_counter()
    tr.run(args.steps)  # one host synchronisation at the end
    sync()
    t1 = time.perf_counter()
    phase_ms, nrec = tr.phase_times()
    tr.profile(False)
    tr.close()

    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = N * args.steps / elapsed
    solve_ms = phase_ms[2] / max(nrec, 1)
    fl = solve_flops(M) * N
    achieved = fl / (solve_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "interpolations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "N": N, "n": n, "L": L, "k": k, "M": M,
                   "tracers": cfg["ntr"], "dt": cfg["dt"], "mode": "plain, one run per launch sequence"},
        "phase_ms_per_step": {name: phase_ms[i] / max(nrec, 1)
                              for i, name in enumerate(["trace", "knn", "solve", "apply"])},
        "roofline": {"kernel": "k_solve", "bound": "alu", "achieved": achieved,
                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": measured_traffic(args.config, M), "traffic_unit": "bytes/launch",
                     "flops_per_launch": fl, "launch_ms": solve_ms},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, X, q0, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
