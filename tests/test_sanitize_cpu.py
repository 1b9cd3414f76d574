"""The host-side index logic (fusion planner, reordering planner, pass-kernel
generator) built with AddressSanitizer and UndefinedBehaviorSanitizer and
run over many random gate lists, without a GPU.  Any out-of-bounds access,
use-after-free, overflow or other undefined behaviour aborts the run."""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1601_07195_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(not os.path.exists(CLANG), reason="needs the ROCm clang driver")
def test_planner_and_generator_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_harness")
    srcs = [os.path.join(ROOT, "tests", "sanitize", "plan_harness.cpp")] + \
        [os.path.join(CSRC, f) for f in ("qs_plan.cpp", "qs_reorder.cpp", "qs_jit.cpp")]
    cmd = [CLANG, "-x", "c++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, *srcs,
           "-L/opt/rocm/lib", "-lhiprtc", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe, "400"], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "kernels" in r.stdout and "ERROR" not in r.stderr
