"""CPU-only sanitizer runs: the oracle (setup, find in all three modes,
eval) and the library's host setup (boxes, OBBs, local map) on small hex,
quad, surface and line meshes, built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no device is touched) and run
with every report fatal."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
BUILD = os.path.join(ROOT, "_build", "sanitize")


def _run(cmd, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr[-4000:])
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan():
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "oracle_driver")
    _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fopenmp", "-I", SAN, os.path.join(SAN, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "findpts_oracle.c"), "-o", exe, "-lm"])
    out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1"))
    assert out.count(":") == 4, out


def test_host_setup_under_asan_ubsan():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "setup_driver")
    csrc = os.path.join(ROOT, "paper_2501_12349_amd", "csrc")
    # sanitizers on the host side of the compilation only
    _run([hipcc, "-O1", "-g", "-std=c++17",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all",
          "-I", os.path.join(ROOT, "include"), "-I", csrc, "-I", SAN,
          "-x", "hip", "--offload-arch=gfx950", os.path.join(SAN, "setup_driver.cpp"),
          os.path.join(csrc, "setup.cpp"), "-o", exe])
    # the HIP runtime's own allocations are not ours to report
    out = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1"))
    assert out.count("status 0") == 4, out
