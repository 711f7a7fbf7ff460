"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code: the
oracle (every entry point, through oracle/sanitize_driver.c) and the host code
of the library (validation, buffer ownership and clean-up paths, the pool's
host checks), each run in a process of its own."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]


def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "driver")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-ffp-contract=off", *SAN,
                               os.path.join(ROOT, "oracle", "sanitize_driver.c"), "-o", exe, "-lm"])
        env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1")
        r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all calls ok" in r.stdout


# host calls that need no GPU: every one must return an error code, never
# crash, leak or overrun; on a machine without a device the valid create and
# pool calls fail in the HIP runtime and take the clean-up paths
HOST_CALLS = r'''
import ctypes, numpy as np
import paper_1804_01609_amd as rb
L = rb.lib()
out = ctypes.c_void_p()
vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
X = np.random.default_rng(0).standard_normal((500, 3))
X /= np.linalg.norm(X, axis=1, keepdims=True)
for n, Lh, k in [(31, 3, 2), (90, 8, 4), (120, 7, 4), (1, 0, 0), (200, 2, 2), (31, 5, 2), (31, 3, 4)]:
    p = rb.make_params(n, Lh, k, 0, rb.VEL_DEFORM, [5.0, 0, 0, 1, 1], 0.1)
    code = L.rbfsl_create(vp(X), 500, 0, ctypes.byref(p), None, ctypes.byref(out))
    assert code != rb.RBFSL_OK and not out.value, (n, Lh, k, code)
    assert rb.pool_run_bytes(1000, p, 64) != 0
cfg = rb.PoolConfig(8, 1, 1 << 20)
assert L.rbfsl_pool_create(ctypes.byref(cfg), ctypes.byref(out)) != rb.RBFSL_OK and not out.value
idx = np.zeros((4, 31), dtype=np.int32)
w = np.zeros((4, 31))
assert L.rbfsl_weights(vp(X), 500, vp(idx), vp(X), vp(np.ones(4)), vp(X), 4, 31, 3, 5, vp(w), None, 0, None) \
    == rb.RBFSL_E_INVAL
assert L.rbfsl_knn(vp(X), 500, vp(X), 4, 2000, vp(idx), None, 0, None) == rb.RBFSL_E_INVAL
for c in range(-9, 2):
    assert L.rbfsl_strerror(c)
print("host calls ok")
'''


@pytest.mark.slow
def test_library_host_code_under_address_and_undefined_behaviour_sanitizers():
    sys.path.insert(0, ROOT)
    from paper_1804_01609_amd import build as B
    lib = B.build_sanitized()
    env = dict(os.environ, RBFSL_LIB_PATH=lib, LD_PRELOAD=B.asan_runtime(), ASAN_OPTIONS="detect_leaks=0",
               HIP_VISIBLE_DEVICES=os.environ.get("HIP_VISIBLE_DEVICES", ""), PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")], env=env, cwd=ROOT,
                       capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    r = subprocess.run([sys.executable, "-c", HOST_CALLS], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "host calls ok" in r.stdout
