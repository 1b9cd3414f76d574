"""Host-side checks of the bench's bookkeeping: the counter-summary lookup
behind every `traffic` field (keyed lines, the source-hash gate) and the
per-kernel rooflines of the later sections."""
from __future__ import annotations

import hashlib
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _write_profile(tmp_path, src_rel, body):
    prof = tmp_path / "profiles"
    prof.mkdir(exist_ok=True)
    sha = hashlib.sha256(open(os.path.join(ROOT, src_rel), "rb").read()).hexdigest()
    (prof / "k_test_wl_traffic.md").write_text(
        f"# test\n\nsource_file: {src_rel}\nsource_sha256: {sha}\n\n" + body)
    return sha


def test_measured_traffic_keys_and_hash_gate(bench, tmp_path, monkeypatch):
    src = "paper_1601_07195_amd/csrc/qs_gates.hip"
    # the bench resolves profiles/ and sources against its ROOT: point
    # profiles at a temporary tree holding a link to the real source
    (tmp_path / "paper_1601_07195_amd" / "csrc").mkdir(parents=True)
    os.symlink(os.path.join(ROOT, src), tmp_path / src)
    _write_profile(tmp_path, src, "traffic_bytes_per_launch: 123\ntraffic_bytes_per_launch.a: 456\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("k_test", "wl") == 123.0
    assert bench.measured_traffic("k_test", "wl", "a") == 456.0
    assert bench.measured_traffic("k_test", "wl", "missing") is None
    assert bench.measured_traffic("k_none", "wl") is None
    # a stale hash (the source changed since the counters were taken) reads as unmeasured
    p = tmp_path / "profiles" / "k_test_wl_traffic.md"
    p.write_text(p.read_text().replace("source_sha256: ", "source_sha256: 0"))
    assert bench.measured_traffic("k_test", "wl") is None


def test_section_rooflines(bench):
    S30, S28 = (1 << 30) * 16, (1 << 28) * 16
    line = {
        "qft_fused_vs_unfused": {"c128": {"30": {"qft": {"fused_s": 0.032, "passes_fused": 5},
                                                 "iqft": {"fused_s": 0.034, "passes_fused": 5}}}},
        "adjoint_vs_param_shift": {"n28": {"sweeps": {"c128": {
            "forward_passes": 99, "forward_pass_ms": 1.5, "reverse_passes": 81, "reverse_pass_ms": 3.6}}}},
        "batch": {"c128": {"lds_bytes_model": 2.0e13, "batch_s": 0.4}},
    }
    r = bench.section_rooflines(line)
    q = r["qs_pass_* (QFT phase runs, n=30 c128)"]
    assert q["bytes_per_launch"] == 2 * S30 and q["launches_per_step"] == 5
    assert q["achieved_GBps"] == pytest.approx(2 * S30 / 0.0064 / 1e9, rel=1e-3)
    assert q["frac"] == pytest.approx(q["achieved_GBps"] / bench.PEAK_HBM_GBPS, rel=1e-3)
    rev = r["qs_pass_* (adjoint reverse sweep, n=28 c128)"]
    assert rev["bytes_per_launch"] == 4 * S28 and rev["mean_launch_ms"] == 3.6
    fwd = r["qs_pass_* (adjoint forward sweep, n=28 c128)"]
    assert fwd["bytes_per_launch"] == 2 * S28
    b = r["k_batch (4096 circuits, c128)"]
    assert b["bound"] == "lds" and b["peak_GBps"] == pytest.approx(bench.PEAK_LDS_GBPS)
    assert b["achieved_GBps"] == pytest.approx(2.0e13 / 0.4 / 1e9, rel=1e-3)
    # sections that did not run contribute nothing
    assert bench.section_rooflines({}) == {}
