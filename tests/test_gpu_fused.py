"""GPU parity of the fused executor (qs_run with gate fusion) against the
CPU oracle, element by element: random circuits, QFT closed form, the
parameterised ansatz and diagonal-heavy circuits whose diagonal gates act on
qubits outside the tile."""
from __future__ import annotations

import math

import numpy as np
import pytest

import circuits as C
import oracle as O
from tests.gpu_util import Q, random_state, rounded_input, to_gpu_state  # noqa: F401

pytestmark = pytest.mark.gpu


@pytest.fixture(params=["interpreted", "compiled"], autouse=True)
def fused_exec(request, monkeypatch):
    """Every test here runs twice: fused passes on the interpreter kernels and
    on kernels compiled per pass shape (QS_FUSED_EXEC drives states left in
    QS_EXEC_AUTO)."""
    monkeypatch.setenv("QS_FUSED_EXEC", request.param)
    return request.param


def dt(Q, name):
    return Q.QS_C128 if name == "c128" else Q.QS_C64


def bound(name, ngates):
    return 1e-12 if name == "c128" else 2e-7 * math.sqrt(ngates) + 1e-6


def diag_heavy(n, ngates, rng):
    ops = C.empty_ops(ngates)
    for g in range(ngates):
        r = rng.random()
        if r < 0.35:
            c, t = (int(v) for v in rng.choice(n, 2, replace=False))
            ph = np.exp(2j * np.pi * rng.random())
            ops[g] = C.op_cu(c, t, np.diag([1.0, ph]))[0]
        elif r < 0.6:
            ops[g] = C.op_u(int(rng.integers(n)), np.diag(np.exp(2j * np.pi * rng.random(2))))[0]
        elif r < 0.8:
            ops[g] = C.op_u(int(rng.integers(n)), C.haar_unitary(rng))[0]
        else:
            c, t = (int(v) for v in rng.choice(n, 2, replace=False))
            ops[g] = C.op_cu(c, t, C.haar_unitary(rng))[0]
    return ops


@pytest.mark.parametrize("name,n", [("c128", 12), ("c128", 13), ("c128", 16), ("c128", 20),
                                    ("c64", 13), ("c64", 14), ("c64", 18)])
def test_fused_random_circuit(Q, name, n):
    rng = np.random.default_rng(600 + n)
    ops = C.random_circuit(n, 300, rng).ops
    psi = random_state(n, rng)
    st = to_gpu_state(Q, psi, dt(Q, name))
    st.run(ops)
    ref = O.run(ops, n, psi=rounded_input(psi, name == "c64"))
    assert np.abs(st.numpy() - ref).max() <= bound(name, 300)
    info, _, _ = Q.qs_plan(n, dt(Q, name), ops)
    assert info["fused"] > 0


@pytest.mark.parametrize("name,n", [("c128", 14), ("c128", 17), ("c64", 15)])
def test_fused_diagonal_heavy(Q, name, n):
    rng = np.random.default_rng(700 + n)
    ops = diag_heavy(n, 400, rng)
    psi = random_state(n, rng)
    st = to_gpu_state(Q, psi, dt(Q, name))
    st.run(ops)
    ref = O.run(ops, n, psi=rounded_input(psi, name == "c64"))
    assert np.abs(st.numpy() - ref).max() <= bound(name, 400)


def phase_blocks(n, nblocks, rng):
    """Blocks of consecutive phase gates diag(1, e^{i phi}) that share a
    target: uncontrolled, or controlled by random qubits (in registers, on
    thread bits or outside the tile, depending on the pass's map), with a
    Haar-random gate between blocks.  Block sizes 1-12 give runs with no,
    one and several per-lane entries and with tile-index entries."""
    ops = []
    for _ in range(nblocks):
        t = int(rng.integers(n))
        for _ in range(int(rng.integers(1, 13))):
            ph = np.diag([1.0, np.exp(2j * np.pi * rng.random())])
            if rng.random() < 0.25:
                ops.append(C.op_u(t, ph))
            else:
                c = int(rng.choice([q for q in range(n) if q != t]))
                ops.append(C.op_cu(c, t, ph))
        ops.append(C.op_u(int(rng.integers(n)), C.haar_unitary(rng)))
    return np.concatenate(ops)


@pytest.mark.parametrize("name,n", [("c128", 13), ("c128", 17), ("c64", 15), ("c64", 18)])
def test_fused_phase_blocks(Q, name, n):
    rng = np.random.default_rng(750 + n)
    ops = phase_blocks(n, 60, rng)
    psi = random_state(n, rng)
    st = to_gpu_state(Q, psi, dt(Q, name))
    st.run(ops)
    ref = O.run(ops, n, psi=rounded_input(psi, name == "c64"))
    assert np.abs(st.numpy() - ref).max() <= bound(name, len(ops))


def _bitrev(z, n):
    return int(format(z, "0%db" % n)[::-1], 2)


@pytest.mark.parametrize("n", [14, 20])
def test_fused_qft_closed_form(Q, n):
    rng = np.random.default_rng(n)
    x = int(rng.integers(1 << n))
    st = Q.State(n, Q.QS_C128, init=False).init_basis(x)
    st.run(C.qft_circuit(n).ops)
    N = 1 << n
    rev = np.array([_bitrev(z, n) for z in range(N)], dtype=np.int64)
    ref = np.exp(2j * np.pi * ((x * rev) % N) / N) / math.sqrt(N)
    assert np.abs(st.numpy() - ref).max() <= 1e-12


@pytest.mark.parametrize("name", ["c128", "c64"])
def test_fused_ansatz(Q, name):
    n = 16
    circ, _ = C.workload_ansatz(n, 5, 1, seed=44)
    st = Q.State(n, dt(Q, name))
    st.run(circ.ops, circ.theta)
    ref = O.run(circ.ops, n, circ.theta)
    assert np.abs(st.numpy() - ref).max() <= bound(name, len(circ))


def test_fused_matches_unfused_workload_n20(Q):
    circ = C.workload_gates(20, 200)
    ref = O.run(circ.ops, 20)
    st = Q.State(20, Q.QS_C128)
    st.run(circ.ops)  # fused
    assert np.abs(st.numpy() - ref).max() <= 1e-12
    p1, nrm, _ = st.probabilities()
    rp1, rnrm, _ = O.probabilities(ref, 20)
    assert np.abs(p1 - rp1).max() <= 1e-12 and abs(nrm - rnrm) <= 1e-12


def test_fused_u_then_udagger(Q):
    n = 18
    circ = C.random_circuit(n, 400, np.random.default_rng(9))
    inv = circ.ops[::-1].copy()
    for op in inv:
        op["mat"] = C.mat_to_row(C.row_to_mat(op["mat"]).conj().T)
    psi = random_state(n, np.random.default_rng(10))
    st = to_gpu_state(Q, psi, Q.QS_C128)
    st.run(circ.ops).run(inv)
    assert np.abs(st.numpy() - psi).max() <= 1e-12


@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("name,n", [("c128", 13), ("c128", 18), ("c64", 15)])
def test_qft_iqft_fused_and_unfused(Q, name, n, fused):
    """The QFT/IQFT pair of the fused-vs-unfused sweep: QFT of a random state
    against the oracle, then the IQFT returns the input; both with fusion and
    with one streaming pass per gate."""
    flags = 0 if fused else Q.QS_RUN_NO_FUSION
    psi = random_state(n, np.random.default_rng(900 + n))
    st = to_gpu_state(Q, psi, dt(Q, name))
    held = st.numpy()
    qft = C.qft_circuit(n).ops
    st.run(qft, fuse=fused)
    ref = O.run(qft, n, psi=held.astype(np.complex128))
    ngates = len(qft)
    assert np.abs(st.numpy() - ref).max() <= bound(name, ngates)
    st.run(C.iqft_circuit(n).ops, fuse=fused)
    assert np.abs(st.numpy() - held).max() <= bound(name, 2 * ngates)
    info, _, _ = Q.qs_plan(n, dt(Q, name), qft, flags=flags)
    if fused:
        assert info["passes"] < ngates
    else:
        assert info["passes"] == ngates and info["fused"] == 0


@pytest.mark.parametrize("name,n", [("c128", 12), ("c128", 17), ("c64", 13), ("c64", 18)])
def test_wide_tiles(Q, name, n):
    """QS_RUN_WIDE_TILES: tiles fix fewer low qubits (lanes also hold free
    tile qubits), so loads and stores use shorter contiguous runs and the
    plan has fewer passes; random gates, phase blocks and a QFT against the
    oracle."""
    rng = np.random.default_rng(950 + n)
    ops = np.concatenate([C.random_circuit(n, 250, rng).ops, phase_blocks(n, 20, rng), C.qft_circuit(n).ops])
    psi = random_state(n, rng)
    st = to_gpu_state(Q, psi, dt(Q, name))
    st.run(ops, wide=True)
    ref = O.run(ops, n, psi=rounded_input(psi, name == "c64"))
    assert np.abs(st.numpy() - ref).max() <= bound(name, len(ops))
    narrow, _, _ = Q.qs_plan(n, dt(Q, name), ops)
    wide, _, _ = Q.qs_plan(n, dt(Q, name), ops, flags=Q.QS_RUN_WIDE_TILES)
    assert wide["passes"] <= narrow["passes"]


@pytest.mark.parametrize("name,n,wide", [("c128", 14, False), ("c128", 16, True), ("c64", 15, False),
                                         ("c64", 17, True)])
def test_verify_mode(Q, name, n, wide):
    """QS_RUN_VERIFY runs the list as asked and, on a scratch copy, gate by
    gate: a unitary list passes with per-gate agreement and no norm drift;
    a non-unitary gate fails the check with QS_EVERIFY."""
    rng = np.random.default_rng(980 + n)
    ops = np.concatenate([C.random_circuit(n, 200, rng).ops, C.qft_circuit(n).ops])
    psi = random_state(n, rng)
    st = to_gpu_state(Q, psi, dt(Q, name))
    st.run(ops, wide=wide, verify=True)
    diff, drift = Q.qs_get_verify(st.handle)
    ref = O.run(ops, n, psi=rounded_input(psi, name == "c64"))
    assert np.abs(st.numpy() - ref).max() <= bound(name, len(ops))
    lim = 1e-13 if name == "c128" else 1e-5
    assert 0.0 <= diff <= lim and 0.0 <= drift <= lim
    bad = C.random_circuit(n, 40, rng).ops
    bad[7]["mat"] = C.mat_to_row(1.5 * np.eye(2))
    with pytest.raises(Q.QSError) as err:
        st.run(bad, wide=wide, verify=True)
    assert err.value.code == Q.QS_EVERIFY
    assert Q.qs_get_verify(st.handle)[1] > 0.1
