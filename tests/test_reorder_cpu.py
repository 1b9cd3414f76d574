"""CPU checks of the qubit-reordering planner (qs_plan_reorder, Sec. 6):
running its schedule -- the gates on their positions, the reorderings in
between and the final one -- on the CPU oracle gives the state the plain
gate list gives; inside the schedule every non-diagonal gate acts on a
local qubit; every reordering swaps upper with local positions; and the
counts follow from the schedule."""
from __future__ import annotations

import numpy as np
import pytest

import circuits as C
import oracle as O


@pytest.fixture(scope="module")
def Q():
    import paper_1601_07195_amd.qs as Q
    return Q


def _state(n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return (v / np.linalg.norm(v)).astype(np.complex128)


def _is_diagonal(op):
    if op["kind"] == C.OP_RZ:
        return True
    if op["kind"] in (C.OP_RX, C.OP_RY):
        return False
    m = op["mat"]
    return m[2] == 0 and m[3] == 0 and m[4] == 0 and m[5] == 0


def _circuit(kind, n):
    if kind == "random":
        return C.random_circuit(n, 250, np.random.default_rng(11)).ops, None
    if kind == "qft":
        return C.qft_circuit(n).ops, None
    if kind == "iqft":
        return C.iqft_circuit(n).ops, None
    circ, _ = C.workload_ansatz(n, 3, 4, seed=12)
    return circ.ops, circ.theta


def _run_schedule(n, ops, theta, at, perms, fin, psi):
    start = 0
    for r in range(len(at)):
        O.run(ops[start:at[r]], n, theta, psi=psi)
        O.permute_qubits(psi, n, perms[r])
        start = at[r]
    O.run(ops[start:], n, theta, psi=psi)
    return O.permute_qubits(psi, n, fin)


@pytest.mark.parametrize("kind", ["random", "qft", "iqft", "ansatz"])
@pytest.mark.parametrize("n,nlocal", [(10, 7), (11, 9), (12, 6), (9, 1), (8, 8)])
def test_reorder_schedule_gives_the_same_state(Q, kind, n, nlocal):
    ops, theta = _circuit(kind, n)
    info, pops, at, perms, fin = Q.qs_plan_reorder(n, nlocal, ops, theta)
    psi0 = _state(n, 13)
    ref = O.run(ops, n, theta, psi=psi0.copy())
    got = _run_schedule(n, pops, theta, at, perms, fin, psi0.copy())
    assert np.abs(got - ref).max() <= 1e-13
    # every non-diagonal gate of the schedule has a local target
    for op in pops:
        if not _is_diagonal(op):
            assert op["target"] < nlocal
    # gates keep their kind, parameter and matrix
    assert np.array_equal(pops["kind"], ops["kind"])
    assert np.array_equal(pops["mat"], ops["mat"])
    # reorderings: disjoint upper/local swaps, at least the needed one
    swaps = 0
    for r in range(len(at)):
        p = perms[r]
        assert sorted(p.tolist()) == list(range(n))
        moved = [x for x in range(n) if p[x] != x]
        for x in moved:
            assert p[p[x]] == x
            assert (x >= nlocal) != (p[x] >= nlocal)
        assert len(moved) >= 2
        swaps += len(moved) // 2
    assert info["remaps"] == len(at) and info["swaps"] == swaps
    assert sorted(fin.tolist()) == list(range(n))
    # the counts of Sec. 3.2's pairwise scheme, from the caller's order
    glob = [op for op in ops if not _is_diagonal(op) and op["target"] >= nlocal]
    assert info["global_gates"] == len(glob)
    pair = sum(1.0 if (op["kind"] == C.OP_CU and op["control"] < nlocal) else 2.0 for op in glob)
    assert info["traffic_pairwise"] == pytest.approx(pair)
    ks = [int(np.count_nonzero(perms[r] != np.arange(n))) // 2 for r in range(len(at))]
    if info["restore_swaps"]:
        ks.append(info["restore_swaps"])
    assert info["traffic_reordered"] == pytest.approx(sum(2 * (1 - 2.0 ** -k) for k in ks))
    if nlocal == n:
        assert info["remaps"] == 0 and info["global_gates"] == 0 and list(fin) == list(range(n))


def test_reorder_qft_needs_two_reorderings(Q):
    """The QFT's non-diagonal gates are its n Hadamards, one per qubit: with
    3 upper qubits the pairwise scheme exchanges 3 times.  Reordering swaps
    the 3 in at once; the 3 qubits they displace get theirs after one more
    reordering, which also sends every qubit home, so no final one is
    needed."""
    n, nlocal = 20, 17
    info, *_ = Q.qs_plan_reorder(n, nlocal, C.qft_circuit(n).ops)
    assert info["global_gates"] == 3
    assert info["remaps"] == 2 and info["swaps"] == 6 and info["restore_swaps"] == 0


def test_reorder_rejects_bad_arguments(Q):
    ops = C.qft_circuit(6).ops
    for nlocal in (0, 7, -1):
        with pytest.raises(Q.QSError):
            Q.qs_plan_reorder(6, nlocal, ops)
