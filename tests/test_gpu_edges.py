"""GPU edge cases through the C ABI: empty gate lists and observables, the
one-qubit state, and the largest states one MI355X holds (n = 33 complex128,
n = 34 complex64, 128 GiB each), where the oracle cannot run whole: there,
sampled amplitudes and per-qubit probabilities are checked against the
closed form of a product state (one-qubit factors from the oracle) with one
controlled gate on top, after the streaming kernels, a fused pass and a
qubit relabelling."""
from __future__ import annotations

import numpy as np
import pytest

import circuits as C
import oracle as O
from tests.gpu_util import Q, random_state, to_gpu_state  # noqa: F401

pytestmark = pytest.mark.gpu


def test_empty_lists_change_nothing(Q):
    import torch
    n = 12
    psi = random_state(n, np.random.default_rng(1800))
    st = to_gpu_state(Q, psi, Q.QS_C128)
    before = st.tensor.clone()
    st.run(C.empty_ops(0))
    assert torch.equal(st.tensor, before)
    info = st.run_reordered(C.empty_ops(0), n - 3)
    assert torch.equal(st.tensor, before)
    assert info["remaps"] == 0 and info["restore_swaps"] == 0 and info["global_gates"] == 0
    assert Q.qs_expect_pauli(st.handle, np.zeros(0, np.uint64), np.zeros(0, np.uint64), np.zeros(0)) == 0.0
    # an adjoint call with no gates: E = <0|H|0>, an empty gradient
    codes = np.zeros((2, n), dtype=np.uint8)
    codes[0, 3] = 3  # Z on qubit 3
    codes[1, 5] = 1  # X on qubit 5
    coeff = np.array([0.75, -2.0])
    lam = Q.State(n, Q.QS_C128, init=False)
    s0 = Q.State(n, Q.QS_C128)
    e, g = Q.grad_adjoint(s0, lam, C.empty_ops(0), np.zeros(0), codes, coeff)
    assert e == pytest.approx(0.75, abs=1e-15) and g.shape == (0,)


@pytest.mark.parametrize("name", ["c128", "c64"])
def test_one_qubit_state(Q, name):
    dt = Q.QS_C128 if name == "c128" else Q.QS_C64
    rng = np.random.default_rng(1810)
    psi = random_state(1, rng)
    u = C.haar_unitary(rng)
    st = to_gpu_state(Q, psi, dt)
    st.apply_1q(0, u)
    st.permute_qubits([0])
    ref = O.apply_1q(psi.astype(np.complex64).astype(np.complex128) if name == "c64" else psi.copy(), 1, 0, u)
    assert np.abs(st.numpy() - ref).max() <= (1e-15 if name == "c128" else 1e-6)
    p1, nrm, _ = st.probabilities()
    assert p1[0] == pytest.approx(abs(ref[1]) ** 2, abs=1e-6) and nrm == pytest.approx(1.0, abs=1e-6)


def _column(u):
    """The one-qubit state u|0>, computed by the oracle."""
    return O.apply_1q(O.basis_state(1, 0), 1, 0, u)


@pytest.mark.parametrize("name,n", [("c128", 33), ("c64", 34)])
def test_largest_states_product_form(Q, name, n):
    import torch
    dt = Q.QS_C128 if name == "c128" else Q.QS_C64
    tol = 1e-12 if name == "c128" else 2e-6
    rng = np.random.default_rng(1820 + n)
    st = Q.State(n, dt)  # |0...0>
    phi = {}
    # streaming kernels on low, middle and top targets
    for q in (0, 1, 6, 7, 12, 20, 27, n - 1):
        u = C.haar_unitary(rng)
        st.apply_1q(q, u)
        phi[q] = _column(u)
    # one fused pass of single-qubit gates on other qubits
    ops = C.empty_ops(0)
    for q in (3, 9, n - 2):
        u1, u2 = C.haar_unitary(rng), C.haar_unitary(rng)
        ops = np.concatenate([ops, C.op_u(q, u1), C.op_u(q, u2)])
        phi[q] = O.apply_1q(_column(u1), 1, 0, u2)
    info, _, _ = Q.qs_plan(n, dt, ops)
    assert info["fused"] == 1
    st.run(ops)
    # a controlled gate whose target is still |0>: control 20, target 25
    cu = C.haar_unitary(rng)
    st.apply_cu(20, 25, cu)
    ucol = _column(cu)
    touched = sorted(phi) + [25]

    def amp(i):
        a = 1.0 + 0j
        for q in range(n):
            b = (i >> q) & 1
            if q == 25:
                a *= ucol[b] if (i >> 20) & 1 else (1.0 if b == 0 else 0.0)
            elif q in phi:
                a *= phi[q][b]
            elif b:
                return 0j
        return a

    def sample(k):
        idx = np.zeros(k, dtype=np.int64)
        for q in touched:
            idx |= rng.integers(0, 2, k, dtype=np.int64) << q
        return np.concatenate([idx, rng.integers(0, 1 << n, 16, dtype=np.int64)])

    idx = sample(2048)
    got = st.tensor[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
    ref = np.array([amp(int(i)) for i in idx])
    assert np.abs(got - ref).max() <= tol
    # per-qubit probabilities of the product form
    p1, nrm, _ = st.probabilities()
    pref = np.zeros(n)
    for q, f in phi.items():
        pref[q] = abs(f[1]) ** 2
    pref[25] = abs(phi[20][1]) ** 2 * abs(ucol[1]) ** 2
    assert np.abs(p1 - pref).max() <= (1e-12 if name == "c128" else 1e-5)
    assert abs(nrm - 1.0) <= (1e-12 if name == "c128" else 1e-5)
    # a relabelling at full size: upper swaps, a block-bit swap, a cycle
    perm = list(range(n))
    perm[n - 1], perm[9] = 9, n - 1
    perm[0], perm[n - 3] = n - 3, 0
    perm[1], perm[2], perm[3] = 2, 3, 1
    st.permute_qubits(perm)
    dst = np.zeros_like(idx)
    for q, p in enumerate(perm):
        dst |= ((idx >> q) & 1) << p
    got = st.tensor[torch.from_numpy(dst).cuda()].cpu().numpy().astype(np.complex128)
    assert np.abs(got - ref).max() <= tol
    del st
    torch.cuda.empty_cache()
