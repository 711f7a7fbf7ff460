"""Write the oracle's q after a full run of a configuration (Algorithm 1 over
all its steps) to tests/golden/, keyed by a hash of every input.

Only the CPU oracle (oracle/) computes anything here; the inputs come from the
seeded generators in paper_1804_01609_amd/workloads.py, which hold none of the
method's arithmetic.  Usage (repository root):

    python tests/golden/make_full_run_golden.py c2        # ~20 min on 8 cores
    python tests/golden/make_full_run_golden.py c1

Output: <config>_full_run_q.npy (ntr x N float64) and <config>_full_run.json
(input hash, steps, oracle source hash, wall time).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1804_01609_amd import workloads as W  # noqa: E402


def input_hash(cfg, X, q0):
    """sha256 over the node set, the initial field and every run parameter."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(X, dtype=np.float64).tobytes())
    h.update(np.ascontiguousarray(q0, dtype=np.float64).tobytes())
    keys = (cfg["N"], cfg["n"], cfg["L"], cfg["k"], cfg["vel_id"], cfg["ntr"], cfg["nsteps"])
    h.update(np.asarray(keys, dtype=np.int64).tobytes())
    h.update(np.asarray(list(cfg["vp"]) + [cfg["dt"], 0.0], dtype=np.float64).tobytes())
    return h.hexdigest()


def paths(name):
    return (os.path.join(HERE, f"{name}_full_run_q.npy"), os.path.join(HERE, f"{name}_full_run.json"))


def main(name, chunk=20):
    cfg = W.CONFIGS[name]
    X = W.fibonacci_nodes(cfg["N"])
    q = W.initial_q(cfg, X)
    hsh = input_hash(cfg, X, q)
    p = oracle.make_params(cfg["n"], cfg["L"], cfg["k"], 0, cfg["vel_id"], cfg["vp"], cfg["dt"], 0.0, cfg["ntr"])
    t0 = time.time()
    m = 0
    while m < cfg["nsteps"]:
        s = min(chunk, cfg["nsteps"] - m)
        q, st, fs = oracle.run(X, p, q, s, m0=m)
        if st != oracle.ORC_OK:
            raise SystemExit(f"oracle run failed at step {fs} with status {st}")
        m += s
        print(f"{name}: step {m}/{cfg['nsteps']}  {time.time() - t0:.0f} s", flush=True)
    qpath, jpath = paths(name)
    np.save(qpath, np.ascontiguousarray(q))
    with open(os.path.join(ROOT, "oracle", "oracle.c"), "rb") as f:
        osha = hashlib.sha256(f.read()).hexdigest()
    meta = dict(config=name, workload=cfg["name"], steps=cfg["nsteps"], input_sha256=hsh,
                oracle_c_sha256=osha, threads=oracle.threads(), wall_s=round(time.time() - t0, 1),
                command=f"python tests/golden/make_full_run_golden.py {name}")
    with open(jpath, "w") as f:
        json.dump(meta, f, indent=1)
        f.write("\n")
    print(json.dumps(meta))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c2")
