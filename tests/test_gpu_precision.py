"""Precision: the random circuit (single-qubit Haar / controlled-U mix, 500
gates) followed by a QFT on all qubits, at n = 24, on a complex128 and a
complex64 state, against the FP64 oracle: maximum absolute amplitude error,
norm drift |<psi|psi> - 1| (accumulated in double precision on the GPU) and
per-qubit probabilities.  complex128 must match to 1e-12; the complex64
bound comes from single-precision rounding: each gate perturbs an amplitude
by a few units of 2^-24 of the pair it mixes, so the error grows like
sqrt(gates) * 2^-24 (scaled by a safety factor)."""
from __future__ import annotations

import math
import os

import numpy as np
import pytest

import circuits as C
import oracle as O
from tests.gpu_util import Q  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(params=["interpreted", "compiled"], autouse=True)
def fused_exec(request, monkeypatch):
    """Every test here runs twice: fused passes on the interpreter kernels and
    on kernels compiled per pass shape (QS_FUSED_EXEC drives states left in
    QS_EXEC_AUTO)."""
    monkeypatch.setenv("QS_FUSED_EXEC", request.param)
    return request.param

N = 24


@pytest.fixture(scope="module")
def reference():
    circ = C.workload_circuit_qft(N, 500)
    O.set_threads(max(1, min(16, os.cpu_count() or 1)))
    psi = O.run(circ.ops, N)
    p1, nrm, _ = O.probabilities(psi, N)
    return circ, psi, p1, nrm


@pytest.mark.parametrize("name", ["c128", "c64"])
def test_precision_random_plus_qft_n24(Q, reference, name):
    circ, psi, rp1, rnrm = reference
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    st = Q.State(N, dtype)
    st.run(circ.ops)
    p1, nrm, _ = st.probabilities()
    out = st.numpy()
    err = float(np.abs(out - psi).max())
    drift = abs(nrm - 1.0)
    perr = float(np.abs(p1 - rp1).max())
    print(f"{name} n={N} gates={len(circ)}: max |amp err| {err:.3e}, norm drift {drift:.3e} "
          f"(oracle {abs(rnrm - 1.0):.3e}), max |P1 err| {perr:.3e}")
    if name == "c128":
        assert err <= 1e-12 and drift <= 1e-12 and perr <= 1e-12
    else:
        bound = 8 * math.sqrt(len(circ)) * 2.0 ** -24
        assert err <= bound, (err, bound)
        assert drift <= 16 * math.sqrt(len(circ)) * 2.0 ** -24
        assert perr <= bound
