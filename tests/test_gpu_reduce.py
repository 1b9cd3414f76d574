"""GPU parity of the FP64 reductions: probabilities, Pauli-sum expectation,
H|psi>.  For complex64 states the reductions are checked against the oracle
run on the very same (complex64) amplitudes upcast to complex128, which pins
the double-precision accumulation itself."""
from __future__ import annotations

import numpy as np
import pytest

import circuits as C
import oracle as O
from tests.gpu_util import Q, random_state, to_gpu_state  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 3, 11, 13, 17])
def test_probabilities(Q, name, n):
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    psi = random_state(n, np.random.default_rng(n))
    st = to_gpu_state(Q, psi, dtype)
    held = st.numpy()  # exactly what the GPU holds
    p1, nrm, full = st.probabilities(full=True)
    rp1, rnrm, rfull = O.probabilities(held, n, full=True)
    assert np.abs(p1 - rp1).max() <= 1e-13
    assert abs(nrm - rnrm) <= 1e-13
    # |a|^2 = re^2 + im^2 may be FMA-contracted on the GPU (not in the
    # oracle): at most 2 ulp of a value <= 1 apart.
    assert np.abs(full.cpu().numpy() - rfull).max() <= 2 * 2.0 ** -52


@pytest.mark.parametrize("name", ["c128", "c64"])
def test_probabilities_basis_and_uniform(Q, name):
    n = 20
    x = 0b10110011100011110001
    st = Q.State(n, Q.QS_C128 if name == "c128" else Q.QS_C64, init=False).init_basis(x)
    p1, nrm, _ = st.probabilities()
    assert [int(v) for v in p1] == [(x >> k) & 1 for k in range(n)] and nrm == 1.0
    st.init_basis(0)
    for k in range(n):
        st.apply_1q(k, C.H_GATE)
    p1, nrm, _ = st.probabilities()
    tol = 1e-13 if name == "c128" else 1e-6
    assert np.abs(p1 - 0.5).max() <= tol and abs(nrm - 1.0) <= tol


def test_probabilities_reproducible(Q):
    n = 18
    st = to_gpu_state(Q, random_state(n, np.random.default_rng(5)), Q.QS_C128)
    a = st.probabilities()
    b = st.probabilities()
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]


def _with_special_terms(ham, n):
    codes = np.vstack([ham.codes, np.zeros((1, n), np.uint8), np.full((1, n), 3, np.uint8)])
    coeff = np.concatenate([ham.coeff, [0.75, -0.5]])
    return codes, coeff


@pytest.mark.parametrize("name", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 4, 12, 16])
def test_expect_pauli(Q, name, n):
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    rng = np.random.default_rng(40 + n)
    ham = C.random_pauli_sum(n, 25, rng)
    codes, coeff = _with_special_terms(ham, n)
    st = to_gpu_state(Q, random_state(n, rng), dtype)
    held = st.numpy()
    got = st.expect(codes, coeff)
    ref = O.expect_pauli(held, n, codes, coeff)
    assert abs(got - ref) <= 1e-12 * max(1.0, np.abs(coeff).sum())


@pytest.mark.parametrize("name", ["c128", "c64"])
def test_apply_pauli_sum(Q, name):
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    n = 11
    rng = np.random.default_rng(77)
    ham = C.random_pauli_sum(n, 30, rng)
    codes, coeff = _with_special_terms(ham, n)
    src = to_gpu_state(Q, random_state(n, rng), dtype)
    dst = Q.State(n, dtype, init=False)
    x, z = Q.pauli_masks(codes)
    Q.qs_apply_pauli_sum(src.handle, dst.handle, x, z, coeff)
    ref = O.apply_pauli_sum(src.numpy(), n, codes, coeff)
    tol = 1e-12 if name == "c128" else 2e-6
    assert np.abs(dst.numpy() - ref).max() <= tol


def test_expect_rejects_out_of_range_mask(Q):
    n = 5
    st = Q.State(n, Q.QS_C128)
    with pytest.raises(Q.QSError):
        Q.qs_expect_pauli(st.handle, np.array([1 << n], np.uint64), np.array([0], np.uint64), [1.0])
