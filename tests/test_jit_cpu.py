"""CPU-only checks of the compiled fused passes: the generator writes a
kernel for every fused pass of representative gate lists and hipRTC
compiles them for gfx950 (no GPU needed); kernels are cached by pass shape,
so the same circuit form with other angles compiles nothing new."""
from __future__ import annotations

import numpy as np
import pytest

import circuits as C


@pytest.fixture(scope="module")
def Q():
    import paper_1601_07195_amd.qs as Q
    return Q


def _plan_fused(Q, n, dtype, ops, theta=None):
    info, _, _ = Q.qs_plan(n, dtype, ops, theta)
    return info["fused"]


@pytest.mark.parametrize("name", ["c128", "c64"])
def test_every_fused_pass_compiles(Q, name):
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    n = 14
    rng = np.random.default_rng(5)
    lists = [
        C.random_circuit(n, 120, rng).ops,              # U / CU, remaps, controls everywhere
        C.qft_circuit(n).ops,                          # phase runs with tables
        C.iqft_circuit(n).ops,
    ]
    for ops in lists:
        nk = Q.qs_precompile(n, dtype, ops)
        assert nk == _plan_fused(Q, n, dtype, ops) and nk > 0


def test_adjoint_passes_compile_and_cache_by_shape(Q):
    n = 13
    circ, _ = C.workload_ansatz(n, 3, 5, seed=11)
    before = Q.qs_get_jit_stats()
    nk = Q.qs_precompile(n, Q.QS_C128, circ.ops, circ.theta, Q.QS_PRECOMPILE_ADJOINT)
    mid = Q.qs_get_jit_stats()
    assert nk > 0 and mid["kernels_compiled"] >= before["kernels_compiled"]
    # new angles, same circuit form: every kernel is already cached
    theta2 = np.random.default_rng(3).uniform(0, 2 * np.pi, circ.nparams)
    assert Q.qs_precompile(n, Q.QS_C128, circ.ops, theta2, Q.QS_PRECOMPILE_ADJOINT) == nk
    after = Q.qs_get_jit_stats()
    assert after["kernels_compiled"] == mid["kernels_compiled"]
    assert after["kernels_cached"] >= nk and after["compile_seconds"] > 0.0


def test_precompile_validates_its_arguments(Q):
    ops = C.random_circuit(12, 10, np.random.default_rng(1)).ops
    with pytest.raises(Q.QSError):
        Q.qs_precompile(12, 7, ops)
    with pytest.raises(Q.QSError):
        Q.qs_precompile(40, Q.QS_C128, ops)
    with pytest.raises(Q.QSError):
        Q.qs_precompile(12, Q.QS_C128, ops, flags=8)
    bad = ops.copy()
    bad[0]["target"] = 12
    with pytest.raises(Q.QSError):
        Q.qs_precompile(12, Q.QS_C128, bad)


def test_disk_cache_serves_a_second_process(tmp_path):
    """With QS_JIT_CACHE_DIR set, a second process finds every kernel the
    first compiled (its text compared in full) and compiles nothing."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys, json, numpy as np; sys.path.insert(0, %r)\n"
            "import circuits as C, paper_1601_07195_amd.qs as Q\n"
            "ops = C.random_circuit(13, 80, np.random.default_rng(21)).ops\n"
            "nk = Q.qs_precompile(13, Q.QS_C64, ops)\n"
            "print(json.dumps([nk, Q.qs_get_jit_stats()]))\n" % root)
    env = dict(os.environ, QS_JIT_CACHE_DIR=str(tmp_path))
    runs = [json.loads(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                      capture_output=True, text=True).stdout.strip().splitlines()[-1])
            for _ in range(2)]
    (nk1, s1), (nk2, s2) = runs
    assert nk1 == nk2 > 0
    assert s1["kernels_compiled"] == nk1 and s1["kernels_from_disk"] == 0
    assert s2["kernels_compiled"] == 0 and s2["kernels_from_disk"] == nk2


def test_hiprtc_fallback_compiles_too(tmp_path):
    """QS_JIT_COMPILER=hiprtc takes the in-process path; the default takes
    child clang processes when the ROCm driver exists."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys, json, numpy as np; sys.path.insert(0, %r)\n"
            "import circuits as C, paper_1601_07195_amd.qs as Q\n"
            "ops = C.random_circuit(12, 40, np.random.default_rng(23)).ops\n"
            "print(json.dumps([Q.qs_precompile(12, Q.QS_C128, ops), Q.qs_get_jit_stats()]))\n" % root)
    out = {}
    for mode in ("hiprtc", "default"):
        env = dict(os.environ)
        env.pop("QS_JIT_CACHE_DIR", None)
        if mode == "hiprtc":
            env["QS_JIT_COMPILER"] = "hiprtc"
        else:
            env.pop("QS_JIT_COMPILER", None)
        r = subprocess.run([sys.executable, "-c", code], env=env, check=True, capture_output=True, text=True)
        out[mode] = json.loads(r.stdout.strip().splitlines()[-1])
    nk, s = out["hiprtc"]
    assert nk > 0 and s["programs_hiprtc"] > 0 and s["programs_clang"] == 0
    nk2, s2 = out["default"]
    assert nk2 == nk
    if os.path.exists("/opt/rocm/llvm/bin/clang++"):
        assert s2["programs_clang"] > 0 and s2["programs_hiprtc"] == 0
