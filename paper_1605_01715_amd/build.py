"""Build the HIP library libfmm_mi355x.so for gfx950 (in-tree)."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfmm_mi355x.so")
SOURCES = ["primitives.hip", "tree.hip", "gemm.hip", "m2l.hip", "operators.hip", "nbody.hip", "chebyshev.hip", "plan.hip",
           "gmres.hip", "dielectric.hip", "tune.hip", "probe.hip", "api.hip"]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-fopenmp",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, jobs=8):
    """Compile every source to an object, then link the shared library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [cc, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0), verbose)
    for p in procs:
        _wait(p, verbose)
    tmp = LIB + ".tmp"
    subprocess.check_call([cc, "-shared", "-fopenmp", "--offload-arch=gfx950", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


def build_sanitized(outdir, jobs=8):
    """Build the same library with AddressSanitizer and UndefinedBehaviorSanitizer
    instrumenting the host code only (device code is built as usual), for
    host-side checks of the C ABI on a machine without a GPU. Returns the path
    of the shared library (outdir/libfmm_mi355x_san.so)."""
    os.makedirs(outdir, exist_ok=True)
    cc = hipcc()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"] + san
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(outdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [cc, *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0), False)
    for p in procs:
        _wait(p, False)
    lib = os.path.join(outdir, "libfmm_mi355x_san.so")
    subprocess.check_call([cc, "-shared", "-fopenmp", "--offload-arch=gfx950", *san, "-o", lib, *objs])
    return lib


def _wait(item, verbose):
    src, p = item
    out = p.communicate()[0].decode(errors="replace")
    lines = [l for l in out.splitlines() if "not a recognized feature" not in l]
    if p.returncode != 0:
        sys.stderr.write("\n".join(lines) + "\n")
        raise RuntimeError(f"hipcc failed on {src}")
    if verbose and lines:
        sys.stderr.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    print(build(verbose=True))
