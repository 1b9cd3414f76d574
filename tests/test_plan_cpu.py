"""CPU checks of the fusion planner (qs_plan): the execution order it picks
only moves gates past gates they commute with, so running the gates in that
order on the CPU oracle gives the same state; every gate is applied once;
and the pass counts behave as the cache-blocking argument predicts."""
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
