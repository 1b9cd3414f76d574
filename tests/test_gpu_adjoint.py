"""GPU adjoint gradient vs the oracle's parameter-shift gradient (exact rule;
tolerance 1e-10 at FP64) and central finite differences (relative 1e-6),
plus the torch.autograd.Function wrapper."""
from __future__ import annotations

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


def adjoint(Q, circ, ham, dtype):
    st = Q.State(circ.n, dtype)
    lam = Q.State(circ.n, dtype, init=False)
    return Q.grad_adjoint(st, lam, circ.ops, circ.theta, ham.codes, ham.coeff)


@pytest.mark.parametrize("n,layers,nterms", [(1, 2, 3), (2, 2, 5), (5, 3, 30), (8, 2, 40)])
def test_adjoint_vs_parameter_shift(Q, n, layers, nterms):
    circ, ham = C.workload_ansatz(n, layers, nterms, seed=1000 + n)
    e, g = adjoint(Q, circ, ham, Q.QS_C128)
    re = O.energy(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    rg = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    assert abs(e - re) <= 1e-12
    assert np.abs(g - rg).max() <= 1e-10


def test_adjoint_vs_central_fd(Q):
    n = 6
    circ, ham = C.workload_ansatz(n, 3, 20, seed=77)
    _, g = adjoint(Q, circ, ham, Q.QS_C128)
    fd = O.grad_central_fd(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())


def test_adjoint_mixed_gates_and_shared_parameters(Q):
    """Fixed U / CU gates between rotations, RX too, and a parameter used by
    two rotations (its gradient is the sum over both)."""
    n = 5
    rng = np.random.default_rng(3)
    ops = np.concatenate([
        C.op_rot(C.OP_RX, 0, 0), C.op_u(1, C.haar_unitary(rng)), C.op_rot(C.OP_RY, 1, 1),
        C.op_cu(1, 3, C.haar_unitary(rng)), C.op_rot(C.OP_RZ, 3, 2), C.op_rot(C.OP_RX, 4, 0),
        C.op_cu(4, 0, C.X_GATE), C.op_rot(C.OP_RY, 2, 3), C.op_u(2, C.H_GATE),
    ])
    theta = rng.uniform(0, 2 * np.pi, 4)
    ham = C.random_pauli_sum(n, 15, rng)
    st = Q.State(n, Q.QS_C128)
    lam = Q.State(n, Q.QS_C128, init=False)
    e, g = Q.grad_adjoint(st, lam, ops, theta, ham.codes, ham.coeff)
    rg = O.grad_param_shift(ops, n, theta, ham.codes, ham.coeff)
    assert abs(e - O.energy(ops, n, theta, ham.codes, ham.coeff)) <= 1e-12
    assert np.abs(g - rg).max() <= 1e-10


def test_adjoint_restores_initial_state(Q):
    n = 7
    circ, ham = C.workload_ansatz(n, 2, 10, seed=4)
    st = Q.State(n, Q.QS_C128)
    lam = Q.State(n, Q.QS_C128, init=False)
    Q.grad_adjoint(st, lam, circ.ops, circ.theta, ham.codes, ham.coeff)
    ref = O.basis_state(n)
    assert np.abs(st.numpy() - ref).max() <= 1e-12


def test_adjoint_c64_fp64_accumulation(Q):
    n = 8
    circ, ham = C.workload_ansatz(n, 3, 20, seed=8)
    e, g = adjoint(Q, circ, ham, Q.QS_C64)
    rg = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    re = O.energy(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    # complex64 state: error reported against the FP64 oracle, loosely bounded
    assert abs(e - re) <= 1e-4 * max(1.0, np.abs(ham.coeff).sum())
    assert np.abs(g - rg).max() <= 1e-4 * max(1.0, np.abs(ham.coeff).sum())


def test_autograd_function(Q):
    import torch
    n = 5
    circ, ham = C.workload_ansatz(n, 2, 12, seed=21)
    theta = torch.tensor(circ.theta, dtype=torch.float64, requires_grad=True)
    e = Q.AdjointEnergy.apply(theta, circ.ops, n, ham.codes, ham.coeff, Q.QS_C128)
    e.backward()
    rg = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    assert abs(e.item() - O.energy(circ.ops, n, circ.theta, ham.codes, ham.coeff)) <= 1e-12
    assert np.abs(theta.grad.numpy() - rg).max() <= 1e-10


def test_state_is_final_flag(Q):
    n = 6
    circ, ham = C.workload_ansatz(n, 2, 10, seed=31)
    st = Q.State(n, Q.QS_C128)
    st.run(circ.ops, circ.theta)
    lam = Q.State(n, Q.QS_C128, init=False)
    e, g = Q.grad_adjoint(st, lam, circ.ops, circ.theta, ham.codes, ham.coeff, state_is_final=True)
    rg = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    assert np.abs(g - rg).max() <= 1e-10


@pytest.mark.parametrize("name,n", [("c128", 11), ("c128", 14), ("c64", 12), ("c64", 15)])
def test_fused_adjoint_vs_parameter_shift(Q, name, n):
    """States at least one fused tile wide take the fused reverse sweep
    (psi and lambda in registers, gradients folded per workgroup)."""
    circ, ham = C.workload_ansatz(n, 2, 25, seed=2000 + n)
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    e, g = adjoint(Q, circ, ham, dtype)
    re = O.energy(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    sample = list(range(0, circ.nparams, 5))
    rg = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff, params=sample)
    scale = max(1.0, np.abs(ham.coeff).sum())
    if name == "c128":
        assert abs(e - re) <= 1e-12
        assert np.abs(g[sample] - rg[sample]).max() <= 1e-10
    else:
        assert abs(e - re) <= 1e-4 * scale
        assert np.abs(g[sample] - rg[sample]).max() <= 1e-4 * scale


def test_fused_adjoint_general_circuit(Q):
    """Fixed U / CU gates (including diagonal ones and controls on every kind
    of tile bit) between rotations, RX / RY / RZ, and a shared parameter."""
    n = 13
    rng = np.random.default_rng(77)
    parts = []
    p = 0
    for layer in range(3):
        for q in range(n):
            kind = [C.OP_RX, C.OP_RY, C.OP_RZ][(q + layer) % 3]
            parts.append(C.op_rot(kind, q, p % 17))
            p += 1
        parts.append(C.random_circuit(n, 12, rng).ops)
        parts.append(C.op_cu(int(rng.integers(n)), (layer * 5 + 3) % n, np.diag([1, 1j])))
    ops = np.concatenate(parts)
    theta = rng.uniform(0, 2 * np.pi, 17)
    ham = C.random_pauli_sum(n, 20, rng)
    st = Q.State(n, Q.QS_C128)
    lam = Q.State(n, Q.QS_C128, init=False)
    e, g = Q.grad_adjoint(st, lam, ops, theta, ham.codes, ham.coeff)
    rg = O.grad_param_shift(ops, n, theta, ham.codes, ham.coeff)
    assert abs(e - O.energy(ops, n, theta, ham.codes, ham.coeff)) <= 1e-12
    assert np.abs(g - rg).max() <= 1e-10
    assert np.abs(st.numpy() - O.basis_state(n)).max() <= 1e-12


def test_fused_adjoint_reproducible(Q):
    n = 14
    circ, ham = C.workload_ansatz(n, 2, 10, seed=9)
    a = adjoint(Q, circ, ham, Q.QS_C128)
    b = adjoint(Q, circ, ham, Q.QS_C128)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("name,n", [("c128", 13), ("c128", 16), ("c64", 14)])
def test_fused_adjoint_wide_tiles(Q, name, n):
    """QS_ADJ_WIDE_TILES plans the forward and reverse sweeps on wide tiles:
    the same energy and gradient (parameter shift on the oracle)."""
    circ, ham = C.workload_ansatz(n, 3, 25, seed=2100 + n)
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    st = Q.State(n, dtype)
    lam = Q.State(n, dtype, init=False)
    e, g = Q.grad_adjoint(st, lam, circ.ops, circ.theta, ham.codes, ham.coeff, wide=True)
    re = O.energy(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    sample = list(range(0, circ.nparams, 4))
    rg = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff, params=sample)
    scale = max(1.0, np.abs(ham.coeff).sum())
    if name == "c128":
        assert abs(e - re) <= 1e-12 and np.abs(g[sample] - rg[sample]).max() <= 1e-10
    else:
        assert abs(e - re) <= 1e-4 * scale and np.abs(g[sample] - rg[sample]).max() <= 1e-4 * scale
