"""Pins of the CPU oracle against things other than itself: dense Kronecker
operators (Eq. 1), closed forms, invariants and the paper's printed tables.
All CPU-only."""
from __future__ import annotations

import math
import os

import numpy as np
import pytest
import scipy.linalg

import circuits as C
import oracle as O
from tests import bruteforce as BF

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng(seed=0):
    return np.random.default_rng(seed)


# ----------------------------------------------------------- gates (Eq. 2, 3)

@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_1q_matches_kronecker(n):
    r = rng(n)
    for k in range(n):
        q = C.haar_unitary(r)
        psi = BF.random_state(n, r)
        ref = BF.kron_1q(n, k, q) @ psi
        got = O.apply_1q(psi.copy(), n, k, q)
        assert np.abs(got - ref).max() <= 1e-14


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_cu_matches_kronecker(n):
    r = rng(10 + n)
    for c in range(n):
        for t in range(n):
            if c == t:
                continue
            q = C.haar_unitary(r)
            psi = BF.random_state(n, r)
            ref = BF.kron_cu(n, c, t, q) @ psi
            got = O.apply_cu(psi.copy(), n, c, t, q)
            assert np.abs(got - ref).max() <= 1e-14, (c, t)


def test_random_circuit_matches_kronecker():
    n = 6
    circ = C.random_circuit(n, 60, rng(3))
    psi = BF.random_state(n, rng(4))
    ref = psi.copy()
    for op in circ.ops:
        q = C.row_to_mat(op["mat"])
        if op["kind"] == C.OP_U:
            ref = BF.kron_1q(n, op["target"], q) @ ref
        else:
            ref = BF.kron_cu(n, op["control"], op["target"], q) @ ref
    got = O.run(circ.ops, n, psi=psi.copy())
    assert np.abs(got - ref).max() <= 1e-13


@pytest.mark.parametrize("n", [1, 4, 9, 12])
def test_hadamard_on_all_gives_uniform(n):
    psi = O.basis_state(n)
    for k in range(n):
        O.apply_1q(psi, n, k, C.H_GATE)
    assert np.abs(psi - 2.0 ** (-n / 2)).max() <= 4 * n * 2.0 ** (-53) * 2.0 ** (-n / 2) * 4


def test_u_then_udagger_returns_input():
    n = 10
    circ = C.random_circuit(n, 200, rng(7))
    psi0 = BF.random_state(n, rng(8))
    psi = O.run(circ.ops, n, psi=psi0.copy())
    inv = circ.ops[::-1].copy()
    for op in inv:
        op["mat"] = C.mat_to_row(C.row_to_mat(op["mat"]).conj().T)
    O.run(inv, n, psi=psi)
    assert np.abs(psi - psi0).max() <= 1e-13


def test_norm_preserved():
    n = 12
    circ = C.random_circuit(n, 300, rng(9))
    psi = O.run(circ.ops, n)
    assert abs(np.vdot(psi, psi).real - 1.0) <= 1e-13


@pytest.mark.parametrize("c,t", [(0, 1), (1, 0), (3, 7), (7, 2), (9, 0)])
def test_cnot_is_exact_index_permutation(c, t):
    n = 10
    psi = BF.random_state(n, rng(c * 31 + t))
    got = O.apply_cu(psi.copy(), n, c, t, C.X_GATE)
    idx = np.arange(1 << n)
    perm = np.where((idx >> c) & 1, idx ^ (1 << t), idx)
    assert np.array_equal(got, psi[perm])


def test_identity_cu_is_noop():
    n = 8
    psi = BF.random_state(n, rng(5))
    got = O.apply_cu(psi.copy(), n, 2, 5, C.I_GATE)
    assert np.array_equal(got, psi)


def _bitrev(z, n):
    return int(format(z, "0%db" % n)[::-1], 2) if n else 0


def qft_closed_form(n, x):
    """QFT|x> without the output reversal: amplitude of |z> is
    2^(-n/2) exp(2 pi i (x * rev_n(z) mod 2^n) / 2^n), exponent reduced in
    integers first."""
    N = 1 << n
    z = np.arange(N)
    rev = np.array([_bitrev(v, n) for v in z], dtype=np.int64)
    ph = (x * rev) % N
    return np.exp(2j * np.pi * ph / N) / math.sqrt(N)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_qft_basis_state_closed_form(n):
    circ = C.qft_circuit(n)
    for x in range(1 << n):
        psi = O.run(circ.ops, n, psi=O.basis_state(n, x))
        assert np.abs(psi - qft_closed_form(n, x)).max() <= 1e-13, x


def test_iqft_inverts_qft():
    n = 7
    psi0 = BF.random_state(n, rng(11))
    psi = O.run(C.qft_circuit(n).ops, n, psi=psi0.copy())
    O.run(C.iqft_circuit(n).ops, n, psi=psi)
    assert np.abs(psi - psi0).max() <= 1e-13


def test_oracle_threads_do_not_change_results():
    n = 14
    circ = C.random_circuit(n, 50, rng(12))
    O.set_threads(1)
    a = O.run(circ.ops, n)
    perm = [int(x) for x in rng(13).permutation(n)]
    u5 = _haar(32, rng(14))
    a1 = O.permute_qubits(O.apply_kq(a.copy(), n, [0, 3, 7, 9, 13], u5), n, perm)
    O.set_threads(4)
    try:
        b = O.run(circ.ops, n)
        b1 = O.permute_qubits(O.apply_kq(b.copy(), n, [0, 3, 7, 9, 13], u5), n, perm)
    finally:
        O.set_threads(1)
    assert np.array_equal(a, b)
    assert np.array_equal(a1, b1)


# ------------------------------------------------------------- probabilities

def test_probabilities_bruteforce():
    n = 9
    psi = BF.random_state(n, rng(13))
    p1, nrm, full = O.probabilities(psi, n, full=True)
    pf = np.abs(psi) ** 2
    idx = np.arange(1 << n)
    for k in range(n):
        assert abs(p1[k] - pf[(idx >> k) & 1 == 1].sum()) <= 1e-15
    assert np.abs(full - pf).max() <= 1e-16
    assert abs(nrm - 1.0) <= 1e-14


def test_probabilities_special_states():
    n = 10
    psi = O.basis_state(n)
    for k in range(n):
        O.apply_1q(psi, n, k, C.H_GATE)
    p1, nrm, _ = O.probabilities(psi, n)
    assert np.abs(p1 - 0.5).max() <= 1e-14 and abs(nrm - 1) <= 1e-14
    x = 0b1011001101
    p1, nrm, full = O.probabilities(O.basis_state(n, x), n, full=True)
    assert [int(v) for v in p1] == [(x >> k) & 1 for k in range(n)]
    assert full[x] == 1.0 and full.sum() == 1.0


# ----------------------------------------------------------------- rotations

@pytest.mark.parametrize("kind,p", [(C.OP_RX, 1), (C.OP_RY, 2), (C.OP_RZ, 3)])
def test_rotation_matrix_is_exponential_of_generator(kind, p):
    for th in (0.0, 0.3, -1.7, 2.5, 6.1):
        ref = scipy.linalg.expm(-0.5j * th * BF.PAULI[p])
        assert np.abs(O.rotation_matrix(kind, th) - ref).max() <= 1e-15


# ----------------------------------------------------------- Pauli expectation

@pytest.mark.parametrize("n", [1, 3, 6])
def test_expect_pauli_kronecker(n):
    r = rng(20 + n)
    ham = C.random_pauli_sum(n, 12, r)
    psi = BF.random_state(n, r)
    hmat = BF.kron_hamiltonian(ham.codes, ham.coeff)
    ref = np.vdot(psi, hmat @ psi).real
    assert abs(O.expect_pauli(psi, n, ham.codes, ham.coeff) - ref) <= 1e-13
    lam = O.apply_pauli_sum(psi, n, ham.codes, ham.coeff)
    assert np.abs(lam - hmat @ psi).max() <= 1e-13


def test_expect_product_state_closed_forms():
    n = 5
    for a, b in [(0.4, 1.1), (2.9, -0.7), (5.5, 3.0)]:
        for q in range(n):
            ops = np.concatenate([C.op_rot(C.OP_RY, q, 0), C.op_rot(C.OP_RZ, q, 1)])
            psi = O.run(ops, n, np.array([a, b]))
            codes = np.zeros((3, n), dtype=np.uint8)
            codes[0, q], codes[1, q], codes[2, q] = 3, 1, 2
            ez, ex, ey = (O.expect_pauli(psi, n, codes[i:i + 1], [1.0]) for i in range(3))
            assert abs(ez - math.cos(a)) <= 1e-14
            assert abs(ex - math.sin(a) * math.cos(b)) <= 1e-14
            assert abs(ey - math.sin(a) * math.sin(b)) <= 1e-14


# ------------------------------------------------------------------ gradients

def test_param_shift_closed_form_single_qubit():
    # E(a, b) = <X> after RY(a) RZ(b) |0> = sin a cos b.
    ops = np.concatenate([C.op_rot(C.OP_RY, 0, 0), C.op_rot(C.OP_RZ, 0, 1)])
    codes = np.array([[1]], dtype=np.uint8)
    for a, b in [(0.3, 0.2), (1.9, -2.2), (4.0, 5.0)]:
        th = np.array([a, b])
        g = O.grad_param_shift(ops, 1, th, codes, [1.0])
        assert abs(g[0] - math.cos(a) * math.cos(b)) <= 1e-14
        assert abs(g[1] + math.sin(a) * math.sin(b)) <= 1e-14


def test_param_shift_matches_central_fd():
    n = 4
    circ, ham = C.workload_ansatz(n, layers=2, nterms=10, seed=99)
    gps = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    gfd = O.grad_central_fd(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    assert np.abs(gps - gfd).max() <= 1e-6 * max(np.abs(gfd).max(), 1.0)


def test_param_shift_dense_matrix_derivative():
    # Differentiate E through dense matrices with the analytic generator
    # dU/dtheta = -(i/2) P U, independent of the shift rule.
    n = 3
    circ, ham = C.workload_ansatz(n, layers=2, nterms=6, seed=5)
    hmat = BF.kron_hamiltonian(ham.codes, ham.coeff)
    mats = []
    for op in circ.ops:
        if op["kind"] == C.OP_CU:
            mats.append(BF.kron_cu(n, op["control"], op["target"], C.row_to_mat(op["mat"])))
        else:
            p = {C.OP_RX: 1, C.OP_RY: 2, C.OP_RZ: 3}[int(op["kind"])]
            u = scipy.linalg.expm(-0.5j * circ.theta[op["param"]] * BF.PAULI[p])
            mats.append(BF.kron_1q(n, op["target"], u))
    psi0 = np.zeros(1 << n, dtype=np.complex128)
    psi0[0] = 1
    ref = np.zeros(circ.nparams)
    for g, op in enumerate(circ.ops):
        if op["kind"] == C.OP_CU:
            continue
        p = {C.OP_RX: 1, C.OP_RY: 2, C.OP_RZ: 3}[int(op["kind"])]
        v = psi0
        dv = None
        for h, m in enumerate(mats):
            v = m @ v
            if h == g:
                dv = -0.5j * BF.kron_1q(n, op["target"], BF.PAULI[p]) @ v
            elif dv is not None:
                dv = m @ dv
        ref[op["param"]] += 2 * np.vdot(v, hmat @ dv).real
    got = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    assert np.abs(got - ref).max() <= 1e-12


def test_rz_on_basis_state_has_zero_gradient():
    n = 3
    ops = C.op_rot(C.OP_RZ, 1, 0)
    codes = np.array([[3, 3, 0], [0, 1, 3]], dtype=np.uint8)
    g = O.grad_param_shift(ops, n, np.array([0.77]), codes, [1.0, 0.5])
    assert g[0] == 0.0


# ------------------------------------------------------------- paper tables

def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_qft_gate_counts_match_table3():
    rows = _rows("table3_qft.txt")
    assert len(rows) == 12
    for n, ngates, total, per_gate in rows:
        assert len(C.qft_circuit(int(n))) == int(ngates) == int(n) * (int(n) + 1) // 2
        # the printed per-gate time is total / ngates rounded to 0.01 s
        assert abs(float(total) / int(ngates) - float(per_gate)) <= 0.006


def test_workload_generators_are_seeded():
    a = C.workload_gates(8, 30)
    b = C.workload_gates(8, 30)
    assert a.ops.tobytes() == b.ops.tobytes()
    for op in a.ops:
        q = C.row_to_mat(op["mat"])
        assert np.abs(q @ q.conj().T - np.eye(2)).max() <= 1e-14
        if op["kind"] == C.OP_CU:
            assert op["control"] != op["target"]
    circ, ham = C.workload_ansatz(6, 3, 20)
    assert circ.nparams == 2 * 6 * 3 and len(circ) == 3 * (3 * 6 - 1)
    w = (ham.codes > 0).sum(axis=1)
    assert w.min() >= 1 and w.max() <= 4


def test_inner_product_matches_vdot():
    n = 8
    a, b = BF.random_state(n, rng(30)), BF.random_state(n, rng(31))
    got = O.inner(a, b, n)
    ref = np.vdot(a, b)
    assert abs(got.real - ref.real) <= 1e-15 and abs(got.imag - ref.imag) <= 1e-15
    assert abs(O.inner(a, 1j * a, n) - 1j) <= 1e-15


# ------------------------------------------------------------ k-qubit gates

def _haar(dim, rng):
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _dense_kq(n, targets, u):
    """The full 2^n operator of u on `targets`, entry by entry from its
    definition: <i|M|j> = u[r(i), r(j)] when i and j agree outside the
    targets (r(x) = the target bits of x, bit j from qubit targets[j])."""
    N = 1 << n
    tmask = sum(1 << t for t in targets)
    def r(x):
        return sum(((x >> t) & 1) << j for j, t in enumerate(targets))
    m = np.zeros((N, N), dtype=np.complex128)
    for i in range(N):
        for j in range(N):
            if (i & ~tmask) == (j & ~tmask):
                m[i, j] = u[r(i), r(j)]
    return m


@pytest.mark.parametrize("n,targets", [(4, [0]), (4, [3, 1]), (5, [1, 4, 0]), (6, [5, 2, 0, 3]),
                                       (6, [0, 1, 2, 3, 4]), (6, [4, 0, 5, 1, 3])])
def test_kq_matches_dense_operator(n, targets):
    rng = np.random.default_rng(50 + n + len(targets))
    u = _haar(1 << len(targets), rng)
    psi = BF.random_state(n, rng)
    ref = _dense_kq(n, targets, u) @ psi
    out = O.apply_kq(psi.copy(), n, targets, u)
    assert np.abs(out - ref).max() <= 1e-14


def test_kq_index_order_matches_kronecker():
    """u = A (x) B with B on targets[0] and A on targets[1]: numpy's kron
    puts B on bit 0 of u's index, which is qubit targets[0]."""
    rng = np.random.default_rng(61)
    n = 5
    a, b = _haar(2, rng), _haar(2, rng)
    psi = BF.random_state(n, rng)
    out = O.apply_kq(psi.copy(), n, [3, 1], np.kron(a, b))
    ref = BF.kron_chain({3: b, 1: a}, n) @ psi
    assert np.abs(out - ref).max() <= 1e-14


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_kq_of_kronecker_product_equals_single_qubit_gates(k):
    rng = np.random.default_rng(70 + k)
    n = 9
    targets = [int(t) for t in rng.choice(n, k, replace=False)]
    qs = [_haar(2, rng) for _ in range(k)]
    u = np.ones((1, 1), dtype=np.complex128)
    for q in reversed(qs):  # qs[j] on bit j of u's index
        u = np.kron(u, q)
    psi = BF.random_state(n, rng)
    out = O.apply_kq(psi.copy(), n, targets, u)
    ref = psi.copy()
    for t, q in zip(targets, qs):
        O.apply_1q(ref, n, t, q)
    assert np.abs(out - ref).max() <= 1e-14


@pytest.mark.parametrize("c,t", [(0, 3), (4, 1), (2, 5)])
def test_kq_controlled_block_equals_cu(c, t):
    rng = np.random.default_rng(80 + c)
    n = 6
    q = _haar(2, rng)
    u = np.eye(4, dtype=np.complex128)
    u[2:, 2:] = q  # index bit 1 = control (targets[1]), bit 0 = target
    psi = BF.random_state(n, rng)
    out = O.apply_kq(psi.copy(), n, [t, c], u)
    ref = O.apply_cu(psi.copy(), n, c, t, q)
    assert np.abs(out - ref).max() <= 1e-15


def test_kq_then_inverse_returns_input():
    rng = np.random.default_rng(90)
    n = 10
    for k in (2, 3, 5):
        targets = [int(t) for t in rng.choice(n, k, replace=False)]
        u = _haar(1 << k, rng)
        psi = BF.random_state(n, rng)
        out = O.apply_kq(psi.copy(), n, targets, u)
        O.apply_kq(out, n, targets, u.conj().T)
        assert np.abs(out - psi).max() <= 1e-13


def test_kq_rejects_bad_targets():
    psi = BF.random_state(4, np.random.default_rng(1))
    for t in ([], [0, 0], [4], [-1], [0, 1, 2, 3, 0, 1]):
        with pytest.raises(ValueError):
            O.apply_kq(psi.copy(), 4, t, np.eye(1 << max(1, len(t))))


# ------------------------------------------- qubit reordering (Sec. 6)

def _product_state(vecs, n):
    """|phi_{n-1}> (x) ... (x) |phi_0>, qubit q's factor vecs[q] (qubit q is
    bit q of the index, so it is the last Kronecker factor for q = 0)."""
    out = np.ones(1, dtype=np.complex128)
    for q in reversed(range(n)):
        out = np.kron(out, vecs[q])
    return out


def _random_qubit_states(n, r):
    v = r.standard_normal((n, 2)) + 1j * r.standard_normal((n, 2))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_permute_moves_product_state_factors(n):
    """Relabelling qubit q as perm[q] puts qubit q's factor of a product state
    at position perm[q]."""
    r = rng(200 + n)
    for _ in range(4):
        vecs = _random_qubit_states(n, r)
        perm = [int(x) for x in r.permutation(n)]
        got = O.permute_qubits(_product_state(vecs, n), n, perm)
        moved = [None] * n
        for q in range(n):
            moved[perm[q]] = vecs[q]
        assert np.abs(got - _product_state(moved, n)).max() <= 1e-15


@pytest.mark.parametrize("n", [3, 6, 9])
def test_permute_is_a_tensor_axis_transpose(n):
    """On the state as an n-axis tensor (axis a = qubit n-1-a) the relabelling
    is numpy's axis transpose."""
    r = rng(210 + n)
    psi = BF.random_state(n, r)
    perm = [int(x) for x in r.permutation(n)]
    inv = [0] * n
    for q in range(n):
        inv[perm[q]] = q
    axes = [n - 1 - inv[n - 1 - b] for b in range(n)]
    ref = np.transpose(psi.reshape((2,) * n), axes).reshape(-1)
    assert np.array_equal(O.permute_qubits(psi.copy(), n, perm), ref)


@pytest.mark.parametrize("a,b", [(0, 1), (1, 0), (2, 6), (6, 0)])
def test_permute_swap_equals_three_cnots(a, b):
    n = 7
    psi = BF.random_state(n, rng(220 + a * 7 + b))
    perm = list(range(n))
    perm[a], perm[b] = b, a
    ref = O.apply_cu(psi.copy(), n, a, b, C.X_GATE)
    O.apply_cu(ref, n, b, a, C.X_GATE)
    O.apply_cu(ref, n, a, b, C.X_GATE)
    assert np.array_equal(O.permute_qubits(psi.copy(), n, perm), ref)


def test_permute_composes_and_inverts():
    n = 9
    r = rng(230)
    psi = BF.random_state(n, r)
    p1 = [int(x) for x in r.permutation(n)]
    p2 = [int(x) for x in r.permutation(n)]
    two = O.permute_qubits(O.permute_qubits(psi.copy(), n, p1), n, p2)
    assert np.array_equal(two, O.permute_qubits(psi.copy(), n, [p2[p1[q]] for q in range(n)]))
    inv = [0] * n
    for q in range(n):
        inv[p1[q]] = q
    assert np.array_equal(O.permute_qubits(O.permute_qubits(psi.copy(), n, p1), n, inv), psi)


def test_permute_rejects_non_permutations():
    psi = BF.random_state(4, rng(240))
    for p in ([0, 1, 2], [0, 1, 2, 2], [0, 1, 2, 4], [-1, 0, 1, 2]):
        with pytest.raises(ValueError):
            O.permute_qubits(psi.copy(), 4, p)
