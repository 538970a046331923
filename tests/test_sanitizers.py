"""AddressSanitizer / UndefinedBehaviorSanitizer builds on the CPU (gcc and
g++, no GPU code): the host runtime (argument checks, grids, plans of single
solves and batches for every dynamics and option, their host images, and a
tile-coverage count replaying the stage kernels' block mapping: every plane
element covered by exactly one tile) with the device launchers stubbed out,
and the oracle (small solves of every dynamics and mode, one-step
evaluation, costate-box helpers, time to reach in both orders).  Any
sanitizer report aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=600)
    assert res.returncode == 0 and res.stdout.strip().endswith("ok"), res.stdout[-4000:]


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.check_call(["gcc", "-std=c11", "-ffp-contract=off"] + SAN +
                          ["-o", exe, os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "odp_oracle.c"), "-lm"])
    _run(exe)


@pytest.mark.skipif(not os.path.exists("/opt/rocm/lib/libamdhip64.so") or shutil.which("g++") is None,
                    reason="needs g++ and the HIP runtime library to link the host code")
def test_host_runtime_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_asan")
    csrc = os.path.join(ROOT, "paper_2204_05520_amd", "csrc")
    srcs = [os.path.join(ROOT, "tests", "sanitize", f) for f in ("host_driver.cpp", "launch_stubs.cpp")]
    srcs += [os.path.join(csrc, f) for f in ("runtime.cpp", "plan.cpp", "tune.cpp", "solve.cpp", "serve.cpp")]
    subprocess.check_call(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                           "-I", os.path.join(ROOT, "include"), "-I", csrc] + SAN + ["-o", exe] + srcs +
                          ["-L", "/opt/rocm/lib", "-lamdhip64", "-lpthread", "-Wl,-rpath,/opt/rocm/lib"])
    _run(exe)
