"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow complex128 simulator (oracle.c, built into liboracle.so) plus
the Python orchestration of the quantities built on top of it: circuit runs,
Pauli-sum energies and the parameter-shift gradient.  Only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import this package;
the GPU library never does, and the two share no code.

Everything is float64 / complex128.  Conventions (qHiPSTER Sec. 2): qubit q
is bit q of the amplitude index, gates are 2x2 row-major matrices acting on
(alpha_{..0_k..}, alpha_{..1_k..}) (Eq. 2), controlled gates act where the
control bit is 1 (Eq. 3).  Rotations are R_P(theta) = exp(-i theta P / 2).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_lib = None

OP_U, OP_CU, OP_RX, OP_RY, OP_RZ = 0, 1, 2, 3, 4

_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    """Load liboracle.so, building it with gcc first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        vp, i, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64
        L.oracle_set_threads.argtypes = [i]
        L.oracle_get_threads.restype = i
        L.oracle_init_basis.argtypes = [vp, i, u64]
        L.oracle_apply_1q.argtypes = [vp, i, i, vp]
        L.oracle_apply_cu.argtypes = [vp, i, i, i, vp]
        L.oracle_apply_kq.argtypes = [vp, i, i, vp, vp]
        L.oracle_permute_qubits.argtypes = [vp, i, vp]
        L.oracle_permute_qubits.restype = i
        L.oracle_probabilities.argtypes = [vp, i, vp, vp, vp]
        L.oracle_inner.argtypes = [vp, vp, i, _dp, _dp]
        L.oracle_apply_pauli_string.argtypes = [vp, i, vp, vp]
        L.oracle_expect_pauli.argtypes = [vp, i, i, vp, vp, _dp]
        L.oracle_expect_pauli.restype = i
        L.oracle_apply_pauli_sum.argtypes = [vp, i, i, vp, vp, vp]
        L.oracle_apply_pauli_sum.restype = i
        L.oracle_rotation_matrix.argtypes = [i, ctypes.c_double, vp]
        L.oracle_run.argtypes = [vp, i, vp, i, vp]
        L.oracle_run.restype = i
        _lib = L
    return _lib


def set_threads(t: int) -> None:
    lib().oracle_set_threads(int(t))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _state(psi: np.ndarray, n: int) -> np.ndarray:
    if psi.dtype != np.complex128 or not psi.flags.c_contiguous or psi.shape != (1 << n,):
        raise ValueError("oracle state must be a contiguous complex128 vector of 2^n")
    return psi


def _mat8(q) -> np.ndarray:
    q = np.ascontiguousarray(q)
    if q.dtype == np.complex128 or q.shape == (2, 2):
        q = np.asarray(q, dtype=np.complex128).reshape(2, 2)
        q = np.stack([q.real, q.imag], axis=-1).reshape(8)
    return np.ascontiguousarray(q, dtype=np.float64)


def basis_state(n: int, index: int = 0) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().oracle_init_basis(_ptr(psi), n, index)
    return psi


def apply_1q(psi: np.ndarray, n: int, k: int, q) -> np.ndarray:
    """In place: Eq. 2 on qubit k."""
    if not 0 <= k < n:
        raise ValueError("target out of range")
    m = _mat8(q)
    lib().oracle_apply_1q(_ptr(_state(psi, n)), n, k, _ptr(m))
    return psi


def apply_cu(psi: np.ndarray, n: int, c: int, t: int, q) -> np.ndarray:
    """In place: Eq. 3 with control c and target t."""
    if not (0 <= c < n and 0 <= t < n) or c == t:
        raise ValueError("bad control/target")
    m = _mat8(q)
    lib().oracle_apply_cu(_ptr(_state(psi, n)), n, c, t, _ptr(m))
    return psi


KQ_MAX = 5  # largest k the oracle's k-qubit gate takes (groups of 32 amplitudes)


def apply_kq(psi: np.ndarray, n: int, targets, u) -> np.ndarray:
    """In place: the 2^k x 2^k matrix u on the qubits `targets` (bit j of u's
    index is qubit targets[j])."""
    t = np.ascontiguousarray(targets, dtype=np.int32)
    k = len(t)
    if not 1 <= k <= KQ_MAX or len(set(t.tolist())) != k or t.min() < 0 or t.max() >= n:
        raise ValueError("bad targets")
    m = np.asarray(u, dtype=np.complex128)
    if m.shape != (1 << k, 1 << k):
        raise ValueError("u must be 2^k x 2^k")
    flat = np.ascontiguousarray(m).view(np.float64).copy()
    lib().oracle_apply_kq(_ptr(_state(psi, n)), n, k, _ptr(t), _ptr(flat))
    return psi


def permute_qubits(psi: np.ndarray, n: int, perm) -> np.ndarray:
    """In place: relabel qubit q as qubit perm[q] (state reordering, Sec. 6):
    the amplitude of index i moves to the index whose bit perm[q] is bit q
    of i."""
    p = np.ascontiguousarray(perm, dtype=np.int32)
    if p.shape != (n,) or sorted(p.tolist()) != list(range(n)):
        raise ValueError("perm must be a permutation of 0..n-1")
    if lib().oracle_permute_qubits(_ptr(_state(psi, n)), n, _ptr(p)) != 0:
        raise MemoryError("oracle_permute_qubits: no memory for the copy")
    return psi


def rotation_matrix(kind: int, theta: float) -> np.ndarray:
    """2x2 complex matrix of RX/RY/RZ(theta) = exp(-i theta P / 2)."""
    q = np.empty(8, dtype=np.float64)
    lib().oracle_rotation_matrix(int(kind), float(theta), _ptr(q))
    return q.reshape(2, 2, 2)[..., 0] + 1j * q.reshape(2, 2, 2)[..., 1]


def run(ops: np.ndarray, n: int, theta=None, psi: np.ndarray | None = None) -> np.ndarray:
    """Apply a gate list (circuit records) in order; starts from |0...0>
    unless psi is given (then it is updated in place)."""
    if psi is None:
        psi = basis_state(n, 0)
    ops = np.ascontiguousarray(ops)
    if ops.dtype.itemsize != 80:
        raise ValueError("ops must be 80-byte gate records")
    for name in ("target", "control"):
        v = ops[name]
        if len(v) and (v.max() >= n):
            raise ValueError(f"{name} out of range")
    if len(ops) and ((ops["target"] < 0).any()):
        raise ValueError("negative target")
    cu = ops["kind"] == OP_CU
    if cu.any() and ((ops["control"][cu] < 0).any() or (ops["control"][cu] == ops["target"][cu]).any()):
        raise ValueError("controlled gate needs a control distinct from its target")
    th = np.ascontiguousarray(theta if theta is not None else np.zeros(1), dtype=np.float64)
    rot = ops["kind"] >= OP_RX
    if rot.any() and (ops["param"][rot].max() >= len(th) or ops["param"][rot].min() < 0):
        raise ValueError("parameter index out of range")
    rc = lib().oracle_run(_ptr(_state(psi, n)), n, _ptr(ops), len(ops), _ptr(th))
    if rc != 0:
        raise ValueError("unknown gate kind")
    return psi


def probabilities(psi: np.ndarray, n: int, full: bool = False):
    """Returns (p1, norm2, full_or_None): p1[k] = P(qubit k reads 1)."""
    p1 = np.zeros(n, dtype=np.float64)
    nrm = np.zeros(1, dtype=np.float64)
    fp = np.empty(1 << n, dtype=np.float64) if full else None
    lib().oracle_probabilities(_ptr(_state(psi, n)), n, _ptr(p1), _ptr(nrm),
                               _ptr(fp) if full else None)
    return p1, float(nrm[0]), fp


def inner(a: np.ndarray, b: np.ndarray, n: int) -> complex:
    re, im = ctypes.c_double(), ctypes.c_double()
    lib().oracle_inner(_ptr(_state(a, n)), _ptr(_state(b, n)), n, ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def _codes(codes: np.ndarray, n: int) -> np.ndarray:
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    if codes.ndim != 2 or codes.shape[1] != n or (codes > 3).any():
        raise ValueError("codes must be (nterms, n) with values 0..3")
    return codes


def apply_pauli_string(psi: np.ndarray, n: int, codes_row) -> np.ndarray:
    out = np.empty_like(psi)
    row = _codes(np.asarray(codes_row).reshape(1, n), n)
    lib().oracle_apply_pauli_string(_ptr(_state(psi, n)), n, _ptr(row), _ptr(out))
    return out


def expect_pauli(psi: np.ndarray, n: int, codes: np.ndarray, coeff) -> float:
    """<psi|H|psi> for H = sum_j coeff[j] P_j (codes row j = P_j)."""
    codes = _codes(codes, n)
    c = np.ascontiguousarray(coeff, dtype=np.float64)
    out = ctypes.c_double()
    rc = lib().oracle_expect_pauli(_ptr(_state(psi, n)), n, len(c), _ptr(codes), _ptr(c), ctypes.byref(out))
    if rc != 0:
        raise MemoryError("oracle scratch allocation failed")
    return out.value


def apply_pauli_sum(psi: np.ndarray, n: int, codes: np.ndarray, coeff) -> np.ndarray:
    """H psi for H = sum_j coeff[j] P_j."""
    codes = _codes(codes, n)
    c = np.ascontiguousarray(coeff, dtype=np.float64)
    out = np.empty_like(psi)
    rc = lib().oracle_apply_pauli_sum(_ptr(_state(psi, n)), n, len(c), _ptr(codes), _ptr(c), _ptr(out))
    if rc != 0:
        raise MemoryError("oracle scratch allocation failed")
    return out


def energy(ops: np.ndarray, n: int, theta, codes: np.ndarray, coeff) -> float:
    """E(theta) = <0|U(theta)^dagger H U(theta)|0>."""
    psi = run(ops, n, theta)
    return expect_pauli(psi, n, codes, coeff)


def grad_param_shift(ops: np.ndarray, n: int, theta, codes: np.ndarray, coeff,
                     params=None) -> np.ndarray:
    """dE/dtheta by the parameter-shift rule (Mitarai et al. 2018; Schuld et
    al. 2019): for one gate exp(-i theta P / 2),
    dE/dtheta = [E(theta + pi/2) - E(theta - pi/2)] / 2 exactly.  Each gate
    occurrence is shifted on its own (its angle only) and the results are
    added to its parameter, so shared parameters are handled too.
    `params` restricts the computation to a subset of parameter indices."""
    theta = np.asarray(theta, dtype=np.float64)
    ops = np.ascontiguousarray(ops)
    grad = np.zeros(len(theta), dtype=np.float64)
    want = None if params is None else set(int(p) for p in params)
    rot_idx = np.nonzero(ops["kind"] >= OP_RX)[0]
    nparams = len(theta)
    for g in rot_idx:
        p = int(ops["param"][g])
        if want is not None and p not in want:
            continue
        # Give this one gate its own private parameter slot, then shift it.
        ops_s = ops.copy()
        ops_s["param"][g] = nparams
        vals = []
        for s in (+0.5 * math.pi, -0.5 * math.pi):
            th = np.concatenate([theta, [theta[p] + s]])
            vals.append(energy(ops_s, n, th, codes, coeff))
        grad[p] += 0.5 * (vals[0] - vals[1])
    return grad


def grad_central_fd(ops: np.ndarray, n: int, theta, codes: np.ndarray, coeff,
                    h: float = 1e-5, params=None) -> np.ndarray:
    """Central finite differences [E(theta + h e_j) - E(theta - h e_j)] / 2h."""
    theta = np.asarray(theta, dtype=np.float64)
    grad = np.zeros(len(theta), dtype=np.float64)
    idx = range(len(theta)) if params is None else params
    for j in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        grad[j] = (energy(ops, n, tp, codes, coeff) - energy(ops, n, tm, codes, coeff)) / (2 * h)
    return grad
