"""CPU-only checks of the batch entry points: qs_batch_create validates the
whole description on the host (naming the bad circuit) before any device
call, and the autotuner's search space only proposes launch shapes the
library accepts.  No compute calls."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import circuits as C


@pytest.fixture(scope="module")
def Q():
    import paper_1601_07195_amd.qs as Q
    return Q


def _pack(circs):
    n = np.array([c[0] for c in circs], dtype=np.int32)
    ops = [c[1] for c in circs]
    th = [np.asarray(c[2], dtype=np.float64) for c in circs]
    xs = [np.asarray(c[3], dtype=np.uint64) for c in circs]
    zs = [np.asarray(c[4], dtype=np.uint64) for c in circs]
    cf = [np.asarray(c[5], dtype=np.float64) for c in circs]

    def off(parts):
        o = np.zeros(len(parts) + 1, dtype=np.int64)
        o[1:] = np.cumsum([len(p) for p in parts])
        return o

    cat = lambda parts, dt: np.ascontiguousarray(np.concatenate(parts) if parts else np.zeros(0, dt))
    return dict(n=n, op_off=off(ops), ops=cat(ops, C.OP_DTYPE), par_off=off(th),
                theta=cat(th, np.float64), term_off=off(cf), x=cat(xs, np.uint64),
                z=cat(zs, np.uint64), coeff=cat(cf, np.float64))


def _create(Q, dtype, p, ncirc=None):
    h = ctypes.c_void_p()
    nc = len(p["n"]) if ncirc is None else ncirc
    ptr = lambda a: a.ctypes.data
    rc = Q.lib().qs_batch_create(dtype, nc, ptr(p["n"]), ptr(p["op_off"]), ptr(p["ops"]),
                                 ptr(p["par_off"]), ptr(p["theta"]), ptr(p["term_off"]),
                                 ptr(p["x"]), ptr(p["z"]), ptr(p["coeff"]), None,
                                 ctypes.byref(h))
    return rc, h


def _good(n=4):
    c = C.ansatz_circuit(n, 2, np.random.default_rng(1))
    return (n, c.ops, c.theta, [0b11], [0b01], [0.5])


def test_batch_create_rejects_bad_descriptions(Q):
    assert _create(Q, 7, _pack([_good()]))[0] == Q.QS_EINVAL
    p = _pack([_good(), _good(3)])
    p["op_off"][0] = 1
    assert _create(Q, Q.QS_C128, p)[0] == Q.QS_EINVAL
    p = _pack([_good(), _good(3)])
    p["par_off"][1], p["par_off"][2] = p["par_off"][2], p["par_off"][1]
    assert _create(Q, Q.QS_C128, p)[0] == Q.QS_EINVAL
    assert "offsets" in Q.qs_last_error()
    bad_n = list(_good(4))
    bad_n[0] = Q.QS_BATCH_MAX_QUBITS + 1
    assert _create(Q, Q.QS_C64, _pack([_good(), tuple(bad_n)]))[0] == Q.QS_ERANGE
    assert "circuit 1" in Q.qs_last_error()
    ctl = C.op_cu(2, 2, C.X_GATE)  # control == target
    assert _create(Q, Q.QS_C128, _pack([_good(), (3, ctl, [], [], [], [])]))[0] == Q.QS_EINVAL
    assert "circuit 1" in Q.qs_last_error()
    rot = C.op_rot(C.OP_RY, 0, 5)  # parameter 5 of a circuit with 1 parameter
    assert _create(Q, Q.QS_C128, _pack([(2, rot, [0.1], [], [], [])]))[0] == Q.QS_EINVAL
    mask = (2, C.op_rot(C.OP_RY, 0, 0), [0.1], [0b100], [0], [1.0])  # X on qubit 2 of 2
    assert _create(Q, Q.QS_C128, _pack([mask]))[0] == Q.QS_EINVAL
    assert Q.lib().qs_batch_create(Q.QS_C128, 1, None, None, None, None, None, None, None, None,
                                   None, None, None) == Q.QS_EINVAL


def test_batch_null_handles(Q):
    L = Q.lib()
    assert L.qs_batch_run(None, None, None, None) == Q.QS_EINVAL
    assert L.qs_batch_destroy(None) == Q.QS_OK


def test_batch_create_without_device_reports_enodev(Q):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _create(Q, Q.QS_C128, _pack([_good(), _good(6)]))[0] == Q.QS_ENODEV


def test_tuning_layout(Q):
    assert ctypes.sizeof(Q.QSBatchTuning) == 20
    assert [f for f, _ in Q.QSBatchTuning._fields_] == \
        ["threads", "lds_bits", "khigh", "wg_per_cu", "order"]


def test_autotune_space_is_valid(Q):
    from paper_1601_07195_amd import autotune as A
    for dt, amp in ((Q.QS_C128, 16), (Q.QS_C64, 8)):
        assert A.valid(A.DEFAULT, dt)
        for C_ in A.SPACE["lds_bits"]:
            for K in A.SPACE["khigh"]:
                t = dict(A.DEFAULT, lds_bits=C_, khigh=K)
                ok = A.valid(t, dt)
                assert ok == (2 * (1 << C_) * amp <= 128 * 1024 and 2 <= K <= min(8, C_ - 6))
