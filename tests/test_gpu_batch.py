"""Batched persistent launch (qs_batch_*): every circuit's energy and
gradient against the oracle (parameter shift, FP64) and against the
unbatched qs_grad_adjoint of the same circuit, for states kept whole in LDS
and for states processed in LDS chunks through the workspace, under several
launch shapes."""
from __future__ import annotations

import numpy as np
import pytest

import circuits as C
import oracle as O
from tests.gpu_util import Q  # noqa: F401

pytestmark = pytest.mark.gpu


def ansatz_batch(count, nmin, nmax, lmin, lmax, nterms, seed):
    out = []
    for j in range(count):
        rng = np.random.default_rng(seed + j)
        n = int(rng.integers(nmin, nmax + 1))
        circ = C.ansatz_circuit(n, int(rng.integers(lmin, lmax + 1)), rng)
        ham = C.random_pauli_sum(n, nterms, rng)
        out.append((n, circ.ops, circ.theta, ham.codes, ham.coeff))
    return out


def unbatched(Q, item, dtype):
    n, ops, theta, codes, coeff = item
    st = Q.State(n, dtype)
    lam = Q.State(n, dtype, init=False)
    return Q.grad_adjoint(st, lam, ops, theta, codes, coeff)


def test_batch_in_lds_vs_oracle(Q):
    """n = 2..9: every state stays in LDS for the whole circuit."""
    items = ansatz_batch(24, 2, 9, 1, 4, 12, seed=5000)
    b = Q.Batch(items, Q.QS_C128)
    e, g = b.run()
    for c, (n, ops, theta, codes, coeff) in enumerate(items):
        assert abs(e[c] - O.energy(ops, n, theta, codes, coeff)) <= 1e-12, c
        rg = O.grad_param_shift(ops, n, theta, codes, coeff)
        assert np.abs(g[c] - rg).max() <= 1e-10, c


@pytest.mark.parametrize("lds_bits,khigh", [(10, 2), (10, 4), (11, 3), (12, 5)])
def test_batch_chunked_vs_unbatched(Q, lds_bits, khigh):
    """n above lds_bits: the state lives in the workspace and gate segments
    run on gathered LDS chunks."""
    items = ansatz_batch(10, 11, 14, 2, 5, 15, seed=6000 + lds_bits * 10 + khigh)
    b = Q.Batch(items, Q.QS_C128)
    e, g = b.run({"lds_bits": lds_bits, "khigh": khigh})
    for c, item in enumerate(items):
        re, rg = unbatched(Q, item, Q.QS_C128)
        assert abs(e[c] - re) <= 1e-12, c
        assert np.abs(g[c] - rg).max() <= 1e-11, c


def test_batch_chunked_vs_oracle(Q):
    items = ansatz_batch(3, 11, 12, 2, 2, 10, seed=6500)
    b = Q.Batch(items, Q.QS_C128)
    e, g = b.run({"lds_bits": 10, "khigh": 3})
    for c, (n, ops, theta, codes, coeff) in enumerate(items):
        assert abs(e[c] - O.energy(ops, n, theta, codes, coeff)) <= 1e-12
        sample = list(range(0, len(theta), 7))
        rg = O.grad_param_shift(ops, n, theta, codes, coeff, params=sample)
        assert np.abs(g[c][sample] - rg[sample]).max() <= 1e-10


def general_items(seed):
    """Fixed U / CU gates with controls and targets anywhere, RX / RY / RZ,
    parameters shared by several rotations, and uneven widths."""
    items = []
    for j, n in enumerate([3, 8, 11, 12, 13]):
        rng = np.random.default_rng(seed + j)
        parts = []
        npar = 2 * n
        for layer in range(3):
            for q in range(n):
                kind = [C.OP_RX, C.OP_RY, C.OP_RZ][(q + layer + j) % 3]
                parts.append(C.op_rot(kind, q, int(rng.integers(npar))))
            parts.append(C.random_circuit(n, 2 * n, rng).ops)
            parts.append(C.op_cu(n - 1, 0, C.haar_unitary(rng)))
            parts.append(C.op_cu(0, n - 1, np.diag([1, np.exp(0.3j)])))
        ops = np.concatenate(parts)
        theta = rng.uniform(0, 2 * np.pi, npar)
        ham = C.random_pauli_sum(n, 9, rng)
        items.append((n, ops, theta, ham.codes, ham.coeff))
    return items


@pytest.mark.parametrize("tuning", [None, {"lds_bits": 10, "khigh": 2, "threads": 512},
                                    {"lds_bits": 10, "khigh": 4, "wg_per_cu": 1, "order": 1}])
def test_batch_general_gates(Q, tuning):
    items = general_items(7100)
    b = Q.Batch(items, Q.QS_C128)
    e, g = b.run(tuning)
    for c, (n, ops, theta, codes, coeff) in enumerate(items):
        assert abs(e[c] - O.energy(ops, n, theta, codes, coeff)) <= 1e-12, c
        rg = O.grad_param_shift(ops, n, theta, codes, coeff)
        assert np.abs(g[c] - rg).max() <= 1e-10, c


def test_batch_c64_fp64_accumulation(Q):
    items = ansatz_batch(12, 6, 13, 2, 4, 12, seed=7300)
    b = Q.Batch(items, Q.QS_C64)
    e, g = b.run({"lds_bits": 11, "khigh": 3})
    for c, (n, ops, theta, codes, coeff) in enumerate(items):
        scale = max(1.0, np.abs(coeff).sum())
        assert abs(e[c] - O.energy(ops, n, theta, codes, coeff)) <= 1e-4 * scale, c
        sample = list(range(0, len(theta), 5))
        rg = O.grad_param_shift(ops, n, theta, codes, coeff, params=sample)
        assert np.abs(g[c][sample] - rg[sample]).max() <= 1e-4 * scale, c


def test_batch_tunings_agree_and_repeat_bitwise(Q):
    items = ansatz_batch(40, 8, 14, 2, 6, 10, seed=7400)
    b = Q.Batch(items, Q.QS_C128)
    e0, g0 = b.run_flat()
    e1, g1 = b.run_flat()
    assert np.array_equal(e0, e1) and np.array_equal(g0, g1)
    for t in ({"threads": 512}, {"lds_bits": 12, "khigh": 6}, {"wg_per_cu": 4, "order": 1},
              {"lds_bits": 10, "khigh": 3, "wg_per_cu": 1}):
        e, g = b.run_flat(t)
        assert np.abs(e - e0).max() <= 1e-12
        assert np.abs(g - g0).max() <= 1e-11


def test_batch_degenerate_circuits(Q):
    """No gates, no observable terms, one qubit, an identity observable."""
    rng = np.random.default_rng(3)
    one = C.op_rot(C.OP_RY, 0, 0)
    items = [
        (4, np.zeros(0, dtype=C.OP_DTYPE), np.zeros(0), np.zeros((1, 4), np.uint8), np.array([2.5])),
        (3, C.ansatz_circuit(3, 1, rng).ops, rng.uniform(0, 6, 6), np.zeros((0, 3), np.uint8),
         np.zeros(0)),
        (1, one, np.array([0.7]), np.array([[3]], np.uint8), np.array([1.0])),
        (12, np.zeros(0, dtype=C.OP_DTYPE), np.zeros(0), np.array([[3] * 12], np.uint8),
         np.array([-1.0])),
    ]
    b = Q.Batch(items, Q.QS_C128)
    e, g = b.run({"lds_bits": 10, "khigh": 2})
    assert e[0] == 2.5 and e[3] == -1.0 and e[1] == 0.0
    assert np.all(g[1] == 0.0)
    assert abs(e[2] - np.cos(0.7)) <= 1e-14
    assert abs(g[2][0] + np.sin(0.7)) <= 1e-14
    empty = Q.Batch([], Q.QS_C128)
    e, g = empty.run()
    assert e.size == 0


def test_batch_rejects_bad_tuning(Q):
    b = Q.Batch(ansatz_batch(2, 4, 5, 1, 2, 3, seed=1), Q.QS_C128)
    for t in ({"threads": 128}, {"lds_bits": 13}, {"lds_bits": 10, "khigh": 5},
              {"wg_per_cu": 9}, {"order": 2}, {"khigh": 1}):
        with pytest.raises(Q.QSError) as ei:
            b.run(t)
        assert ei.value.code == Q.QS_EINVAL
    b.run()  # still usable


def test_autotune_picks_a_valid_shape(Q):
    from paper_1601_07195_amd import autotune as A
    items = ansatz_batch(64, 8, 13, 2, 5, 8, seed=7600)
    b = Q.Batch(items, Q.QS_C128)
    t = A.tune(b, repeats=1)
    assert A.valid(t, Q.QS_C128)
    e0, g0 = b.run_flat()
    e, g = b.run_flat(A.fields(t))
    assert np.abs(e - e0).max() <= 1e-12 and np.abs(g - g0).max() <= 1e-11


def forms_items(seed, widths):
    """Every register-update form of the batch kernel: X (real), H (real),
    CNOT in both directions (controlled exchange), CZ and controlled phases
    (controlled diagonal, general path), fixed diagonal and real gates,
    controlled Haar gates, RX (general), RY (real) and RZ (diagonal)
    rotations, with qubits anywhere in the state."""
    items = []
    for j, n in enumerate(widths):
        rng = np.random.default_rng(seed + j)
        parts = []
        npar = 3 * n
        for _ in range(4 * n):
            q = int(rng.integers(n))
            c, t = (int(v) for v in rng.choice(n, 2, replace=False)) if n > 1 else (0, 0)
            r = int(rng.integers(10))
            if r == 0:
                parts.append(C.op_u(q, C.X_GATE))
            elif r == 1:
                parts.append(C.op_u(q, C.H_GATE))
            elif r == 2 and n > 1:
                parts.append(C.op_cu(c, t, C.X_GATE))
            elif r == 3 and n > 1:
                parts.append(C.op_cu(c, t, np.diag([1.0, -1.0])))
            elif r == 4 and n > 1:
                parts.append(C.op_cu(c, t, np.diag([1.0, np.exp(1j * rng.uniform(0, 6))])))
            elif r == 5:
                parts.append(C.op_u(q, np.diag(np.exp(1j * rng.uniform(0, 6, 2)))))
            elif r == 6 and n > 1:
                parts.append(C.op_cu(c, t, C.haar_unitary(rng)))
            else:
                kind = [C.OP_RX, C.OP_RY, C.OP_RZ][r % 3]
                parts.append(C.op_rot(kind, q, int(rng.integers(npar))))
        ops = np.concatenate(parts)
        theta = rng.uniform(0, 2 * np.pi, npar)
        ham = C.random_pauli_sum(n, 7, rng)
        items.append((n, ops, theta, ham.codes, ham.coeff))
    return items


@pytest.mark.parametrize("tuning", [None, {"lds_bits": 10, "khigh": 3, "threads": 512},
                                    {"lds_bits": 8, "khigh": 2}])
def test_batch_gate_forms_vs_oracle(Q, tuning):
    """States in LDS (n <= C, including 1 and 2 qubits padded to a 3-qubit
    register block) and chunked states (n > C)."""
    items = forms_items(7700, [1, 2, 3, 5, 8, 9, 11, 12])
    b = Q.Batch(items, Q.QS_C128)
    e, g = b.run(tuning)
    for c, (n, ops, theta, codes, coeff) in enumerate(items):
        assert abs(e[c] - O.energy(ops, n, theta, codes, coeff)) <= 1e-12, c
        rg = O.grad_param_shift(ops, n, theta, codes, coeff)
        assert np.abs(g[c] - rg).max() <= 1e-10, c


def test_batch_widest_states_vs_unbatched(Q):
    """The widest batched states (up to QS_BATCH_MAX_QUBITS) run chunked with
    the most chunks per segment; checked against the unbatched adjoint."""
    items = forms_items(7800, [20, Q.QS_BATCH_MAX_QUBITS])
    b = Q.Batch(items, Q.QS_C128)
    e, g = b.run()
    for c, item in enumerate(items):
        re, rg = unbatched(Q, item, Q.QS_C128)
        assert abs(e[c] - re) <= 1e-11 * max(1.0, abs(re)), c
        assert np.abs(g[c] - rg).max() <= 1e-10, c
