"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers are built for the host with -fsanitize=address,undefined and run:
  * tests/sanitize/oracle_driver.c -- the oracle (plain C, OpenMP) over
    small problems of every kind it covers and some it rejects;
  * tests/sanitize/abi_driver.cpp -- the C-ABI host code (lmep_abi.cpp, the
    kernel launchers replaced by tests/sanitize/abi_stubs.cpp) over weight
    counts, scratch sizes, options, plans and every entry point's argument
    checks, and a well-formed call that fails on the device of a machine
    without a GPU.
Any sanitizer report aborts the driver (-fno-sanitize-recover) and fails the
test.  Leak checking stays off for the ABI driver: the HIP runtime keeps
allocations for the life of the process."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
CLANG = "/opt/rocm/bin/amdclang++"


def _run(cmd, env=None, timeout=300):
    return subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_drv")
    r = _run(["gcc", "-std=gnu11", "-fopenmp", *FLAGS, "-I", os.path.join(ROOT, "oracle"),
              os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"])
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1")
    r = _run([exe], env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout


@pytest.mark.skipif(not os.path.exists(CLANG) or not os.path.exists("/opt/rocm/lib/libamdhip64.so"),
                    reason="ROCm host compiler or runtime not installed")
def test_abi_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "abi_drv")
    csrc = os.path.join(ROOT, "paper_2603_15964_amd", "csrc")
    r = _run([CLANG, "-std=c++17", *FLAGS, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
              "-I", os.path.join(ROOT, "include"), "-I", csrc, os.path.join(csrc, "lmep_abi.cpp"),
              os.path.join(SAN, "abi_stubs.cpp"), os.path.join(SAN, "abi_driver.cpp"), "-L/opt/rocm/lib",
              "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = _run([exe], env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout
