"""CPU checks of the fusion planner (qs_plan): the execution order it picks
only moves gates past gates they commute with, so running the gates in that
order on the CPU oracle gives the same state; every gate is applied once;
and the pass counts behave as the cache-blocking argument predicts."""
from __future__ import annotations

import os

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


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("kind", ["random", "qft", "ansatz", "mixed"])
def test_plan_order_preserves_the_state(Q, dtype, kind):
    n = 15
    dt = Q.QS_C128 if dtype == "c128" else Q.QS_C64
    theta = None
    if kind == "random":
        ops = C.random_circuit(n, 300, np.random.default_rng(1)).ops
    elif kind == "qft":
        ops = C.qft_circuit(n).ops
    elif kind == "ansatz":
        circ, _ = C.workload_ansatz(n, 4, 5, seed=2)
        ops, theta = circ.ops, circ.theta
    else:
        rng = np.random.default_rng(3)
        parts = [C.random_circuit(n, 60, rng).ops, C.qft_circuit(n).ops,
                 C.iqft_circuit(n).ops, C.random_circuit(n, 60, rng).ops]
        ops = np.concatenate(parts)
    info, order, pass_of = Q.qs_plan(n, dt, ops, theta)
    assert sorted(order.tolist()) == list(range(len(ops)))
    assert info["passes"] == info["fused"] + info["single_1q"] + info["single_cu"]
    assert info["passes"] < len(ops)
    # passes are applied in order: pass_of is non-decreasing along `order`
    assert np.all(np.diff(pass_of[order]) >= 0)
    psi = _state(n, 4)
    a = O.run(ops, n, theta, psi=psi.copy())
    b = O.run(ops[order], n, theta, psi=psi.copy())
    assert np.abs(a - b).max() <= 1e-12


def test_plan_without_fusion_is_one_pass_per_gate(Q):
    n = 18
    ops = C.random_circuit(n, 50, np.random.default_rng(5)).ops
    info, order, _ = Q.qs_plan(n, Q.QS_C128, ops, flags=Q.QS_RUN_NO_FUSION)
    assert info["passes"] == 50 and info["fused"] == 0
    assert order.tolist() == list(range(50))
    S = (1 << n) * 16
    ncu = int((ops["kind"] == C.OP_CU).sum())
    assert info["hbm_bytes"] == (50 - ncu) * 2 * S + ncu * S  # Table 2 accounting


def test_small_states_are_not_fused(Q):
    info, _, _ = Q.qs_plan(8, Q.QS_C128, C.qft_circuit(8).ops)
    assert info["fused"] == 0 and info["passes"] == 36


def test_qft_fuses_into_few_passes(Q):
    # every QFT stage is one H plus controlled phases (diagonal): each pass
    # takes five high stages' targets, so ceil((n - L) / 5) + 1 passes suffice
    for n, dt, L in [(20, Q.QS_C128, 6), (30, Q.QS_C128, 6), (33, Q.QS_C128, 6), (34, Q.QS_C64, 7)]:
        info, _, _ = Q.qs_plan(n, dt, C.qft_circuit(n).ops)
        assert info["passes"] <= (n - L + 4) // 5 + 1, (n, info)


def test_plan_rejects_bad_ops(Q):
    ops = C.random_circuit(10, 5, np.random.default_rng(6)).ops.copy()
    ops[2]["target"] = 10
    with pytest.raises(Q.QSError):
        Q.qs_plan(10, Q.QS_C128, ops)


def _table2_rows():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table2_bounds.txt")
    rows = []
    with open(path) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            case, gate, cond, x, bw, sec = line.split()
            rows.append((int(case), gate, cond, int(x), bw, float(sec)))
    return rows


def test_table2_printed_bounds_follow_from_the_byte_model(Q):
    """Sec. 5.2, Table 2: every printed lower bound is 2^(m+x) bytes over the
    bandwidth the case is bound by, at m = 29, B_mem = 40 GB/s, B_net = 5.5 GB/s
    (printed to two decimals).  The byte counts are the library's own: a
    gate pass on one device (qs_plan, cases 1, 3 and the control-1 shard of
    case 4) and the pairwise exchanges of a state split by its top qubits
    (qs_plan_reorder's traffic_pairwise, cases 2, 5 and 6, in shard sizes)."""
    m = 29
    bandwidth = {"mem": 40e9, "net": 5.5e9}
    rows = _table2_rows()
    assert [r[0] for r in rows] == [1, 2, 3, 4, 5, 6]
    shard = (1 << m) * 16  # one shard of 2^m complex doubles = 2^(m+4) bytes
    u = C.haar_unitary(np.random.default_rng(7))
    p = 3  # 8 shards: the top three qubits are global
    n = m + p
    for case, gate, cond, x, bw, printed in rows:
        t = 2.0 ** (m + x) / bandwidth[bw]
        assert abs(t - printed) <= 0.005 + 1e-12, (case, t, printed)
        if case == 1:      # 1q gate on a local target
            ops = C.op_u(m - 1, u)
        elif case == 3:    # controlled gate, both qubits local
            ops = C.op_cu(3, m - 1, u)
        elif case == 4:    # control global: on a control-1 shard every pair changes
            ops = C.op_u(m - 1, u)
        if case in (1, 3, 4):
            info, _, _ = Q.qs_plan(m, Q.QS_C128, ops, flags=Q.QS_RUN_NO_FUSION)
            assert info["hbm_bytes"] == 2 ** (m + x), (case, info["hbm_bytes"])
            continue
        if case == 2:      # 1q gate on a global target
            ops = C.op_u(n - 1, u)
        elif case == 5:    # global target, local control
            ops = C.op_cu(3, n - 1, u)
        else:              # both global
            ops = C.op_cu(n - 2, n - 1, u)
        info, *_ = Q.qs_plan_reorder(n, m, ops)
        assert info["traffic_pairwise"] * shard == 2 ** (m + x), (case, info)


def test_wide_tiles_plan_fewer_passes():
    """Fixing fewer low qubits in each tile frees three tile qubits per pass:
    the 1000-gate random circuit at n = 30 needs fewer passes (and moves
    fewer bytes) at both amplitude types."""
    import numpy as np
    import circuits as C
    import paper_1601_07195_amd.qs as Q
    ops = C.random_circuit(30, 1000, np.random.default_rng(C.SEED_BASE + 1)).ops
    for dt in (Q.QS_C128, Q.QS_C64):
        narrow, _, _ = Q.qs_plan(30, dt, ops)
        wide, order, pass_of = Q.qs_plan(30, dt, ops, flags=Q.QS_RUN_WIDE_TILES)
        assert wide["passes"] < narrow["passes"] and wide["hbm_bytes"] < narrow["hbm_bytes"]
        assert sorted(order.tolist()) == list(range(len(ops)))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_plan_of_the_adjoint_reverse_sweep(Q, dtype):
    """QS_PLAN_ADJOINT_REVERSE plans the reversed, inverted list as the
    adjoint's reverse sweep does: every pass fused, 4S per pass (psi and
    lambda), and its order, applied to the inverted gates, undoes the
    circuit (so each gate keeps its place relative to the gates it does not
    commute with)."""
    n = 15
    dt = Q.QS_C128 if dtype == "c128" else Q.QS_C64
    S = (1 << n) * (16 if dtype == "c128" else 8)
    circ, _ = C.workload_ansatz(n, 4, 5, seed=6)
    for flags in (0, Q.QS_RUN_WIDE_TILES):
        info, order, pass_of = Q.qs_plan(n, dt, circ.ops, circ.theta, flags=flags | Q.QS_PLAN_ADJOINT_REVERSE)
        assert info["passes"] == info["fused"] > 0
        assert info["hbm_bytes"] == 4 * S * info["passes"]
        assert sorted(order.tolist()) == list(range(len(circ.ops)))
        assert np.all(np.diff(pass_of[order]) >= 0)
        # the reversed list with each gate inverted, in the planned order
        rev = circ.ops[::-1].copy()
        th = circ.theta.copy()
        for op in rev:
            if op["param"] >= 0:
                continue  # rotations: inverted below through theta
            op["mat"] = C.mat_to_row(C.row_to_mat(op["mat"]).conj().T)
        psi = _state(n, 7)
        fwd = O.run(circ.ops, n, circ.theta, psi=psi.copy())
        back = O.run(rev[order], n, -th, psi=fwd)
        assert np.abs(back - psi).max() <= 1e-12
    with pytest.raises(Q.QSError):
        Q.qs_plan(n, dt, circ.ops, circ.theta, flags=Q.QS_PLAN_ADJOINT_REVERSE | Q.QS_RUN_NO_FUSION)
