"""Build librbfsl.so (HIP kernels + C ABI) for gfx950 with hipcc.

Usage: python -m paper_1804_01609_amd.build   (or call build()).
Objects go to _build/ at the repository root; the library lands next to this
file so that it ships with the source tree.
"""
import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librbfsl.so")

SOURCES = ["k_pool4.hip", "k_pool3.hip", "k_pool8.hip", "k_pool16.hip", "k_pool_search.hip", "pool_api.hip", "k_solve_m192.hip", "k_solve_m128.hip", "k_solve_m120.hip", "k_solve_m96.hip", "k_solve_m81.hip", "k_solve_m64.hip", "k_solve_m48.hip",
           "k_solve.hip", "k_cached.hip", "k_pu.hip", "api.hip", "noalloc.hip", "k_trace.hip", "k_grid.hip", "k_knn.hip", "k_apply.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("RBFSL_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # every expression rounds as written; fused multiply-adds only via fma()
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep SimplifyCFG from merging the per-row-slot branches of the solver
    # into pointer phis, which would push its register arrays to scratch
    "-mllvm", "-simplifycfg-sink-common=false",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


def source_hash():
    """sha256 over every file the library is built from (kernels, host code,
    the C header and this build script, which holds the flags), in name
    order; the library embeds it and the binding refuses a library whose hash
    differs from the sources beside it."""
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".h")))
    h = hashlib.sha256()
    for name, path in [(f, os.path.join(CSRC, f)) for f in files] + [
            ("rbfsl.h", os.path.join(INCLUDE, "rbfsl.h")), ("build.py", os.path.abspath(__file__))]:
        with open(path, "rb") as fh:
            data = fh.read()
        h.update(name.encode() + b"\0" + str(len(data)).encode() + b"\0" + data)
    return h.hexdigest()


def build(verbose=False, jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    objs, procs = [], []
    shash = source_hash()
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, f'-DRBFSL_SOURCE_HASH="{shash}"', "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


# host units of the library: parameter validation, buffer ownership, the pool's
# arena and queues, the serve loop
HOST_UNITS = ["api.hip", "pool_api.hip"]
ASAN_LIB = os.path.join(BUILD, "asan", "librbfsl_asan.so")


def build_sanitized(verbose=False):
    """librbfsl with AddressSanitizer and UndefinedBehaviorSanitizer in the
    host code of HOST_UNITS (GPU code is built as usual; the sanitizers apply
    to the host pass only).  The other objects come from a regular build().
    For CPU tests of the host logic; load it with the compiler's ASan runtime
    preloaded."""
    objs = [os.path.join(BUILD, s.replace(".hip", ".o")) for s in SOURCES]
    if not all(os.path.exists(o) for o in objs):
        build(verbose=verbose)
    out = os.path.join(BUILD, "asan")
    os.makedirs(out, exist_ok=True)
    shash = source_hash()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    procs, repl = [], {}
    for src in HOST_UNITS:
        obj = os.path.join(out, src.replace(".hip", ".o"))
        repl[os.path.join(BUILD, src.replace(".hip", ".o"))] = obj
        cmd = [HIPCC, *FLAGS, *san, f'-DRBFSL_SOURCE_HASH="{shash}"', "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for p in procs:
        _wait(p)
    objs = [repl.get(o, o) for o in objs]
    rt = asan_runtime()
    subprocess.check_call([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan",
                           f"-Wl,-rpath,{os.path.dirname(rt)}", *objs, "-o", ASAN_LIB])
    return ASAN_LIB


def asan_runtime():
    """The compiler's shared AddressSanitizer runtime (to preload)."""
    out = subprocess.check_output([os.path.join(os.path.dirname(HIPCC), "..", "llvm", "bin", "clang"),
                                   "--print-file-name=libclang_rt.asan-x86_64.so"]).decode().strip()
    if not os.path.isabs(out):
        import glob
        hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        out = hits[0] if hits else out
    return out


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    # the host pass does not know the GPU-only target feature; that warning is harmless
    lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if p.returncode != 0:
        sys.stderr.write(text)
        raise RuntimeError(f"hipcc failed for {src}")
    if lines:
        sys.stderr.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
