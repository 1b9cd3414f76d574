"""CPU-only checks of the C ABI: libqs.so loads, exports every entry point
declared in include/qs.h, validates arguments before touching a GPU, and the
Python marshalling agrees with the header's layouts.  No compute calls."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import circuits as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qs.h")


@pytest.fixture(scope="module")
def Q():
    import paper_1601_07195_amd.qs as Q
    return Q


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qs_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_expected_api():
    names = declared_functions()
    for must in ("qs_create", "qs_apply_1q", "qs_apply_cu", "qs_probabilities",
                 "qs_expect_pauli", "qs_grad_adjoint", "qs_permute_qubits",
                 "qs_plan_reorder", "qs_run_reordered"):
        assert must in names


def test_library_exports_every_declared_symbol(Q):
    lib = Q.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) <= set(Q.EXPORTED)


def test_header_constants_match_binding(Q):
    src = open(HEADER).read()
    consts = dict(re.findall(r"#define\s+(QS_[A-Z0-9_]+)\s+\(?(-?\d+)\)?", src))
    for k, v in consts.items():
        assert getattr(Q, k) == int(v), k


def test_op_record_layout(Q):
    assert Q.QS_OP_DTYPE.itemsize == 80
    assert Q.QS_OP_DTYPE == C.OP_DTYPE
    assert [Q.QS_OP_U, Q.QS_OP_CU, Q.QS_OP_RX, Q.QS_OP_RY, Q.QS_OP_RZ] == \
        [C.OP_U, C.OP_CU, C.OP_RX, C.OP_RY, C.OP_RZ]
    ops = C.ansatz_circuit(3, 1).ops
    assert Q.ops_array(ops).dtype == Q.QS_OP_DTYPE


def test_pauli_masks_marshalling(Q):
    codes = np.array([[0, 1, 2, 3], [3, 3, 0, 2], [0, 0, 0, 0]], dtype=np.uint8)
    x, z = Q.pauli_masks(codes)
    assert list(x) == [0b0110, 0b1000, 0]
    assert list(z) == [0b1100, 0b1011, 0]


def _create(Q, n, dtype, ptr, nbytes):
    h = ctypes.c_void_p()
    return Q.lib().qs_create(n, dtype, ctypes.c_void_p(ptr), nbytes, None, ctypes.byref(h)), h


def test_create_validates_before_any_gpu_call(Q):
    assert _create(Q, 0, Q.QS_C128, 256, 1 << 20)[0] == Q.QS_ERANGE
    assert _create(Q, 34, Q.QS_C128, 256, 1 << 40)[0] == Q.QS_ERANGE
    assert _create(Q, 35, Q.QS_C64, 256, 1 << 40)[0] == Q.QS_ERANGE
    assert _create(Q, 10, 7, 256, 1 << 20)[0] == Q.QS_EINVAL
    assert _create(Q, 10, Q.QS_C128, 0, 1 << 20)[0] == Q.QS_EINVAL
    assert _create(Q, 10, Q.QS_C128, 256 + 8, 1 << 20)[0] == Q.QS_EINVAL
    assert _create(Q, 10, Q.QS_C128, 256, (1 << 14) - 1)[0] == Q.QS_ERANGE
    assert "buffer" in Q.qs_last_error()
    assert Q.lib().qs_create(10, Q.QS_C128, ctypes.c_void_p(256), 1 << 20, None, None) == Q.QS_EINVAL


def test_null_handles_rejected(Q):
    L = Q.lib()
    q = np.eye(2, dtype=np.complex128)
    m = np.stack([q.real, q.imag], -1).reshape(8).copy()
    assert L.qs_apply_1q(None, 0, m.ctypes.data) == Q.QS_EINVAL
    assert L.qs_apply_cu(None, 0, 1, m.ctypes.data) == Q.QS_EINVAL
    t = np.zeros(1, dtype=np.int32)
    assert L.qs_apply_kq(None, 1, t.ctypes.data, m.ctypes.data) == Q.QS_EINVAL
    assert L.qs_permute_qubits(None, t.ctypes.data) == Q.QS_EINVAL
    assert L.qs_run_reordered(None, 1, None, 0, None, 0, 0, None) == Q.QS_EINVAL
    assert L.qs_init_basis(None, 0) == Q.QS_EINVAL
    assert L.qs_run(None, None, 0, None, 0, 0) == Q.QS_EINVAL
    assert L.qs_probabilities(None, None, None, None, 0) == Q.QS_EINVAL
    assert L.qs_destroy(None) == Q.QS_OK
    assert Q.qs_strerror(Q.QS_ERANGE) == "size out of range"


def test_create_without_device_reports_enodev(Q):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _create(Q, 10, Q.QS_C128, 256, 1 << 20)[0] == Q.QS_ENODEV
