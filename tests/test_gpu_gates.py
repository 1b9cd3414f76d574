"""GPU parity of the gate kernels (Eq. 2, Eq. 3) and state init against the
CPU oracle, element by element, through the C ABI.

Tolerance: complex128 max |amplitude error| <= 1e-12.  complex64 results are
compared with the oracle applied to the same (complex64-rounded) input; their
error is reported and bounded only loosely (1e-6), complex64 precision being
the point of that dtype."""
from __future__ import annotations

import math

import numpy as np
import pytest

import circuits as C
import oracle as O
from tests.gpu_util import Q, random_state, rounded_input, to_gpu_state  # noqa: F401

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
TOL64 = 1e-6
DTYPES = ["c128", "c64"]


def dt(Q, name):
    return Q.QS_C128 if name == "c128" else Q.QS_C64


def tol(name):
    return TOL128 if name == "c128" else TOL64


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n", [1, 2, 5, 13])
def test_init_basis_exact(Q, name, n):
    rng = np.random.default_rng(n)
    for index in {0, (1 << n) - 1, int(rng.integers(1 << n))}:
        st = Q.State(n, dt(Q, name), init=False)
        st.init_basis(index)
        got = st.numpy()
        ref = O.basis_state(n, index)
        assert np.array_equal(got, ref), index


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n", [1, 2, 3, 7, 11, 14])
def test_1q_every_target(Q, name, n):
    rng = np.random.default_rng(100 + n)
    psi = random_state(n, rng)
    st = to_gpu_state(Q, psi, dt(Q, name))
    ref = rounded_input(psi, name == "c64")
    for k in range(n):
        u = C.haar_unitary(rng)
        st.apply_1q(k, u)
        O.apply_1q(ref, n, k, u)
        got = st.numpy()
        err = np.abs(got - ref).max()
        assert err <= tol(name), (k, err)
        ref = rounded_input(got, name == "c64") if name == "c64" else ref


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("n", [2, 3, 5, 9])
def test_cu_every_pair(Q, name, n):
    rng = np.random.default_rng(200 + n)
    psi = random_state(n, rng)
    st = to_gpu_state(Q, psi, dt(Q, name))
    ref = rounded_input(psi, name == "c64")
    for c in range(n):
        for t in range(n):
            if c == t:
                continue
            u = C.haar_unitary(rng)
            st.apply_cu(c, t, u)
            O.apply_cu(ref, n, c, t, u)
            got = st.numpy()
            err = np.abs(got - ref).max()
            assert err <= tol(name), (c, t, err)
            if name == "c64":
                ref = rounded_input(got, True)


@pytest.mark.parametrize("name", DTYPES)
def test_cu_sampled_pairs_ragged_sizes(Q, name):
    rng = np.random.default_rng(300)
    for n in (12, 15):
        psi = random_state(n, rng)
        st = to_gpu_state(Q, psi, dt(Q, name))
        ref = rounded_input(psi, name == "c64")
        # (2, 12) / (2, 14) / (3, 13): 64-byte control runs with a target the
        # dispatch sends to the compact pass (complex128 / complex64 units)
        pairs = [(0, n - 1), (n - 1, 0), (1, 2), (2, 1), (0, 1), (1, 0)] + \
            ([(2, 12), (2, 14), (3, 13)] if n == 15 else []) + \
            [tuple(int(v) for v in rng.choice(n, 2, replace=False)) for _ in range(6)]
        for c, t in pairs:
            u = C.haar_unitary(rng)
            st.apply_cu(c, t, u)
            O.apply_cu(ref, n, c, t, u)
            got = st.numpy()
            assert np.abs(got - ref).max() <= tol(name), (n, c, t)
            if name == "c64":
                ref = rounded_input(got, True)


@pytest.mark.parametrize("name", DTYPES)
def test_cu_compact_below_the_line(Q, name, monkeypatch):
    """QS_CU_COMPACT_FROM=0 sends controls inside a 128-byte line to the
    compact enumeration too (the measurement of the line granularity uses
    it): every pair at n = 9 and sampled pairs at n = 13 against the oracle."""
    monkeypatch.setenv("QS_CU_COMPACT_FROM", "0")  # every control bit
    rng = np.random.default_rng(350)
    for n in (9, 13):
        psi = random_state(n, rng)
        st = to_gpu_state(Q, psi, dt(Q, name))
        ref = rounded_input(psi, name == "c64")
        pairs = [(c, t) for c in range(n) for t in range(n) if c != t] if n == 9 else \
            [(0, 12), (1, 12), (2, 12), (3, 9), (1, 0), (2, 5), (0, 1), (3, 2)]
        for c, t in pairs:
            u = C.haar_unitary(rng)
            st.apply_cu(c, t, u)
            O.apply_cu(ref, n, c, t, u)
            got = st.numpy()
            assert np.abs(got - ref).max() <= tol(name), (n, c, t)
            if name == "c64":
                ref = rounded_input(got, True)


@pytest.mark.parametrize("name", DTYPES)
@pytest.mark.parametrize("order", ["0", "1"])
def test_1q_block_orders(Q, name, order, monkeypatch):
    """QS_1Q_BLOCK_ORDER forces either block order of the paired-stream
    kernel (the dispatch table picks one per state size and target): every
    target of a 14-qubit state against the oracle."""
    monkeypatch.setenv("QS_1Q_BLOCK_ORDER", order)
    n = 14
    rng = np.random.default_rng(360 + int(order))
    psi = random_state(n, rng)
    st = to_gpu_state(Q, psi, dt(Q, name))
    ref = rounded_input(psi, name == "c64")
    for k in range(n):
        u = C.haar_unitary(rng)
        st.apply_1q(k, u)
        O.apply_1q(ref, n, k, u)
        got = st.numpy()
        assert np.abs(got - ref).max() <= tol(name), k
        if name == "c64":
            ref = rounded_input(got, True)


def test_cnot_exact_permutation_on_gpu(Q):
    n = 12
    psi = random_state(n, np.random.default_rng(7))
    idx = np.arange(1 << n)
    for c, t in [(0, 1), (5, 0), (11, 3), (3, 11)]:
        st = to_gpu_state(Q, psi, Q.QS_C128)
        st.apply_cu(c, t, C.X_GATE)
        perm = np.where((idx >> c) & 1, idx ^ (1 << t), idx)
        assert np.array_equal(st.numpy(), psi[perm])


def test_random_circuit_workload_n20(Q):
    """200-gate random 1q / controlled-U mix from |0...0> at n = 20: full
    state and per-qubit probabilities."""
    circ = C.workload_gates(20, 200)
    ref = O.run(circ.ops, 20)
    st = Q.State(20, Q.QS_C128)
    st.run(circ.ops, fuse=False)
    got = st.numpy()
    assert np.abs(got - ref).max() <= TOL128
    p1, nrm, _ = st.probabilities()
    rp1, rnrm, _ = O.probabilities(ref, 20)
    assert np.abs(p1 - rp1).max() <= TOL128
    assert abs(nrm - rnrm) <= TOL128


def _bitrev(z, n):
    return int(format(z, "0%db" % n)[::-1], 2)


def test_qft_basis_state_closed_form_gpu(Q):
    n = 12
    x = 0b101100111010
    st = Q.State(n, Q.QS_C128, init=False).init_basis(x)
    st.run(C.qft_circuit(n).ops, fuse=False)
    got = st.numpy()
    N = 1 << n
    rev = np.array([_bitrev(z, n) for z in range(N)])
    ref = np.exp(2j * np.pi * ((x * rev) % N) / N) / math.sqrt(N)
    assert np.abs(got - ref).max() <= TOL128


def test_u_then_udagger_on_gpu(Q):
    n = 16
    circ = C.random_circuit(n, 100, np.random.default_rng(9))
    inv = circ.ops[::-1].copy()
    for op in inv:
        op["mat"] = C.mat_to_row(C.row_to_mat(op["mat"]).conj().T)
    psi = random_state(n, np.random.default_rng(10))
    st = to_gpu_state(Q, psi, Q.QS_C128)
    st.run(circ.ops, fuse=False).run(inv, fuse=False)
    assert np.abs(st.numpy() - psi).max() <= TOL128


def test_argument_errors_queue_nothing(Q):
    n = 6
    psi = random_state(n, np.random.default_rng(11))
    st = to_gpu_state(Q, psi, Q.QS_C128)
    with pytest.raises(Q.QSError):
        st.apply_1q(n, C.H_GATE)
    with pytest.raises(Q.QSError):
        st.apply_cu(2, 2, C.X_GATE)
    bad = C.workload_gates(n, 5).ops.copy()
    bad[3]["target"] = 17
    with pytest.raises(Q.QSError):
        st.run(bad)
    assert np.array_equal(st.numpy(), psi)


@pytest.mark.parametrize("name,n", [("c128", 24), ("c64", 25)])
def test_dispatch_shapes_at_large_n(Q, name, n):
    """Every kernel shape the dispatcher picks (exchange by shuffle and by
    LDS, paired streams in both workgroup orders, compact / predicated /
    in-unit controls) at a size where the high-stride rules apply."""
    rng = np.random.default_rng(500 + n)
    psi = random_state(n, rng)
    st = to_gpu_state(Q, psi, dt(Q, name))
    ref = rounded_input(psi, name == "c64")
    gates = [("1q", k) for k in (0, 1, 5, 6, 7, 8, 9, 21, 22, 23, 24, n - 1)] + \
        [("cu", ct) for ct in ((0, n - 1), (n - 1, 0), (1, 2), (2, 9), (3, 22), (4, 23),
                               (7, 10), (8, 6), (10, 7), (23, 3), (9, 20), (20, 9), (5, 6),
                               (6, 5), (12, 1))]
    for kind, arg in gates:
        u = C.haar_unitary(rng)
        if kind == "1q":
            if arg >= n:
                continue
            st.apply_1q(arg, u)
            O.apply_1q(ref, n, arg, u)
        else:
            c, t = arg
            st.apply_cu(c, t, u)
            O.apply_cu(ref, n, c, t, u)
    got = st.numpy()
    bound = TOL128 if name == "c128" else 2e-6
    assert np.abs(got - ref).max() <= bound


# ------------------------------------------------------------ k-qubit gates

def _haar_dim(dim, rng):
    z = (rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


@pytest.mark.parametrize("name", ["c128", "c64"])
@pytest.mark.parametrize("n,k", [(8, 1), (8, 3), (13, 2), (13, 5), (17, 4), (17, 5), (6, 5)])
def test_apply_kq_vs_oracle(Q, name, n, k):
    """Dense k-qubit gates on random targets (always including qubit 0 or
    the top qubit) against the oracle's k-qubit gate."""
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    rng = np.random.default_rng(1000 + 10 * n + k)
    for trial in range(3):
        targets = [int(t) for t in rng.choice(n, k, replace=False)]
        if trial == 1 and 0 not in targets:
            targets[0] = 0
        if trial == 2 and n - 1 not in targets:
            targets[-1] = n - 1
        u = _haar_dim(1 << k, rng)
        psi = random_state(n, rng)
        st = to_gpu_state(Q, psi, dtype)
        held = st.numpy().astype(np.complex128)
        st.apply_kq(targets, u)
        ref = O.apply_kq(held.copy(), n, targets, u)
        tol = 1e-13 if name == "c128" else 2e-6
        assert np.abs(st.numpy() - ref).max() <= tol, (targets, trial)


@pytest.mark.parametrize("n", [9, 10, 14])
def test_apply_kq_five_qubits_matrix_core_path(Q, n):
    """complex128 five-qubit gates run on the FP64 matrix cores from n = 9
    (one batch of 16 groups) up: lowest, highest, reversed and random target
    orders against the oracle."""
    rng = np.random.default_rng(1100 + n)
    cases = [[0, 1, 2, 3, 4], list(range(n - 5, n)), [4, 3, 2, 1, 0], [n - 1, 0, n // 2 + 1, 2, 4]]
    cases.append([int(t) for t in rng.choice(n, 5, replace=False)])
    for targets in cases:
        u = _haar_dim(32, rng)
        psi = random_state(n, rng)
        st = to_gpu_state(Q, psi, Q.QS_C128)
        st.apply_kq(targets, u)
        ref = O.apply_kq(psi.copy(), n, targets, u)
        assert np.abs(st.numpy() - ref).max() <= 1e-13, targets


def test_apply_kq_equals_single_qubit_gates(Q):
    """A Kronecker product of 2x2 gates applied as one block equals the
    same gates applied one by one through qs_apply_1q."""
    rng = np.random.default_rng(1100)
    n = 16
    for k in (2, 3, 5):
        targets = [int(t) for t in rng.choice(n, k, replace=False)]
        qs = [_haar_dim(2, rng) for _ in range(k)]
        u = np.ones((1, 1), dtype=np.complex128)
        for q in reversed(qs):
            u = np.kron(u, q)
        psi = random_state(n, rng)
        a = to_gpu_state(Q, psi, Q.QS_C128).apply_kq(targets, u).numpy()
        b = to_gpu_state(Q, psi, Q.QS_C128)
        for t, q in zip(targets, qs):
            b.apply_1q(t, q)
        assert np.abs(a - b.numpy()).max() <= 1e-13, k


def test_apply_kq_then_inverse_at_n28(Q):
    """At a bandwidth-scale size: U on five qubits spread over the state,
    then U^dagger, returns the input; sampled amplitudes checked against the
    oracle's k-qubit gate one group at a time."""
    n, k = 28, 5
    rng = np.random.default_rng(1200)
    targets = [0, 7, 13, 21, 27]
    u = _haar_dim(1 << k, rng)
    st = Q.State(n, Q.QS_C128)
    for q in (0, 5, 13, 20, 27):
        st.apply_1q(q, C.H_GATE)
    before = st.numpy()
    st.apply_kq(targets, u)
    after = st.numpy()
    # one sampled group, recomputed from the definition
    tmask = sum(1 << t for t in targets)
    for base in (0, 1 << 3, (1 << 20) | (1 << 5)):
        assert base & tmask == 0
        idx = [base | sum(((r >> j) & 1) << t for j, t in enumerate(targets)) for r in range(1 << k)]
        assert np.abs(after[idx] - u @ before[idx]).max() <= 1e-14
    st.apply_kq(targets, u.conj().T)
    assert np.abs(st.numpy() - before).max() <= 1e-13


def test_apply_kq_rejects_bad_arguments(Q):
    st = Q.State(6, Q.QS_C128)
    for targets in ([0, 0], [6], [-1], [0, 1, 2, 3, 4, 5]):
        k = len(targets)
        u = np.eye(1 << k, dtype=np.complex128)
        with pytest.raises(Q.QSError) as ei:
            Q.qs_apply_kq(st.handle, targets, u)
        assert ei.value.code == Q.QS_EINVAL
    L = Q.lib()
    t = np.zeros(1, dtype=np.int32)
    m = np.zeros(8)
    assert L.qs_apply_kq(st.handle, 0, t.ctypes.data, m.ctypes.data) == Q.QS_EINVAL
    assert L.qs_apply_kq(None, 1, t.ctypes.data, m.ctypes.data) == Q.QS_EINVAL


@pytest.mark.parametrize("name", ["c128", "c64"])
def test_phase_gates_touch_only_their_quarter(Q, name):
    """diag(1, phi) single-qubit and controlled gates (the quarter-state
    phase kernel) against the oracle, for low, middle and top qubits."""
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    n = 14
    rng = np.random.default_rng(1300)
    psi = random_state(n, rng)
    st = to_gpu_state(Q, psi, dtype)
    ref = st.numpy().astype(np.complex128)
    tol = 1e-13 if name == "c128" else 3e-6
    for k in (0, 1, 2, 3, 7, n - 1):
        ph = np.diag([1.0, np.exp(1j * rng.uniform(0, 2 * np.pi))])
        st.apply_1q(k, ph)
        O.apply_1q(ref, n, k, ph)
    for c, t in ((0, 1), (1, 0), (2, 9), (9, 2), (0, n - 1), (n - 1, 5), (4, 3)):
        ph = np.diag([1.0, np.exp(1j * rng.uniform(0, 2 * np.pi))])
        st.apply_cu(c, t, ph)
        O.apply_cu(ref, n, c, t, ph)
    assert np.abs(st.numpy() - ref).max() <= tol
