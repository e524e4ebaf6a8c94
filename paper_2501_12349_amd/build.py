"""Build libfpts.so (HIP for gfx950) in-tree.

Each source under csrc/ is compiled to an object in _build/ by hipcc, in
parallel, and the objects are linked into paper_2501_12349_amd/libfpts.so.
Packed FP32 instructions are disabled for all device code.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libfpts.so")
BUILD = os.path.join(ROOT, "_build")
ARCH = os.environ.get("FPTS_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]

SOURCES = ["kernels_newton.hip",
           "kernels_newton_line.hip",
           "kernels_find.hip", "kernels_eval.hip", "setup_device.hip", "lpt.hip", "api.cpp", "setup.cpp",
           "serve.cpp"]
# the device setup reproduces the host setup's rounding and the particle
# update rounds operation by operation: no contraction
EXTRA = {"setup_device.hip": ["-ffp-contract=off"], "lpt.hip": ["-ffp-contract=off"]}


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    lang = ["-x", "hip"]
    cmd = [HIPCC] + COMMON + EXTRA.get(src, []) + lang + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose=False, jobs=None):
    """Compile every source and link libfpts.so; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + \
        ["-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
