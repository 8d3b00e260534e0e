"""The C ABI's host code under the address and undefined-behaviour sanitizers.

pcop.cpp is compiled again with the sanitizers on its host pass only (the
device code is unchanged), linked with the kernels' ordinary objects and a
randomised driver (abi_fuzz.c) that calls everything that returns before
device work: option defaults, validation of random (mostly invalid) problems
and options, workspace sizing, and pcop_setup's argument checks.  Out-of-
bounds reads of the caller's arrays, integer overflow in the size arithmetic
and the like abort the driver with a report.  Runs on the CPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2410_22686_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitize")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# each sanitizer flag is for the host pass only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.fixture(scope="module")
def fuzz_binary():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    from paper_2410_22686_amd import build
    os.makedirs(OUT, exist_ok=True)
    # the kernels' ordinary objects (build() compiles them when absent)
    objs = [os.path.join(build.BUILD, os.path.splitext(s)[0] + ".o") for s in build.SOURCES if s != "pcop.cpp"]
    if not all(os.path.exists(o) for o in objs):
        build.build()
    pcop_obj = os.path.join(OUT, "pcop_san.o")
    _run([HIPCC, "-x", "hip", "-c", os.path.join(CSRC, "pcop.cpp"), "-o", pcop_obj, "-O1", "-g", "-std=c++17",
          "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include")] + HOST_SAN)
    drv_obj = os.path.join(OUT, "abi_fuzz.o")
    _run([HIPCC, "-x", "c", "-c", os.path.join(ROOT, "tests", "abi_fuzz.c"), "-o", drv_obj, "-O1", "-g",
          "-I", os.path.join(ROOT, "include")] + HOST_SAN)
    exe = os.path.join(OUT, "abi_fuzz")
    _run([HIPCC, "-o", exe, drv_obj, pcop_obj] + objs + ["--offload-arch=gfx950"] + HOST_SAN)
    return exe


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_host_abi_under_sanitizers(fuzz_binary, seed):
    env = dict(os.environ)
    # the HIP runtime keeps process-lifetime allocations; leaks are not what is checked here
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([fuzz_binary, "20000", str(seed)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-6000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
    assert "valid" in r.stdout
