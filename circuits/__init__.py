"""Seeded synthetic inputs: gate matrices, circuits, observables, workloads.

This module only *describes* work -- gate lists, 2x2 matrices, parameter
vectors and Pauli strings.  It applies nothing to a state and computes no
probability, expectation or gradient, so both the CPU oracle and the GPU
library can take their inputs from it without sharing any of the method's
arithmetic.

Representation
--------------
A circuit is a numpy structured array of ``OP_DTYPE`` records whose layout is
the C struct ``qs_op`` of the library's public header (80 bytes):

    kind     int32   OP_U, OP_CU, OP_RX, OP_RY or OP_RZ
    target   int32   qubit the 2x2 acts on (k in Eq. 2, t in Eq. 3)
    control  int32   control qubit c of Eq. 3 (CU only, -1 otherwise)
    param    int32   index into the parameter vector (rotations only, else -1)
    mat      8 x f64 row-major q11, q12, q21, q22 as (re, im) pairs (U, CU)

Qubit q is bit q of the amplitude index (qHiPSTER, Sec. 2).  Rotations are
R_P(theta) = exp(-i theta P / 2); their matrices are built by whoever applies
them, from theta.

A Pauli sum is ``PauliSum(codes, coeff)`` with ``codes`` an (nterms, n) uint8
array, one code per qubit (0 = I, 1 = X, 2 = Y, 3 = Z).

Seeds: workload i of the benchmark suite uses ``numpy.random.default_rng``
with seed 1601 + i; circuit j of the batch workload uses 1601 * 10**4 + j.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

OP_U, OP_CU, OP_RX, OP_RY, OP_RZ = 0, 1, 2, 3, 4
OP_NAMES = {OP_U: "U", OP_CU: "CU", OP_RX: "RX", OP_RY: "RY", OP_RZ: "RZ"}

OP_DTYPE = np.dtype(
    [
        ("kind", "<i4"),
        ("target", "<i4"),
        ("control", "<i4"),
        ("param", "<i4"),
        ("mat", "<f8", (8,)),
    ],
    align=False,
)
assert OP_DTYPE.itemsize == 80

SEED_BASE = 1601
BATCH_SEED_BASE = 1601 * 10**4

# Gate matrices as complex 2x2 arrays (inputs, not arithmetic on a state).
H_GATE = np.array([[1.0, 1.0], [1.0, -1.0]], dtype=np.complex128) / math.sqrt(2.0)
X_GATE = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
Y_GATE = np.array([[0.0, -1.0j], [1.0j, 0.0]], dtype=np.complex128)
Z_GATE = np.array([[1.0, 0.0], [0.0, -1.0]], dtype=np.complex128)
I_GATE = np.eye(2, dtype=np.complex128)


def mat_to_row(q: np.ndarray) -> np.ndarray:
    """2x2 complex -> 8 doubles, row-major (q11, q12, q21, q22) as (re, im)."""
    q = np.asarray(q, dtype=np.complex128).reshape(2, 2)
    return np.stack([q.real, q.imag], axis=-1).reshape(8).astype(np.float64)


def row_to_mat(row) -> np.ndarray:
    """Inverse of mat_to_row."""
    r = np.asarray(row, dtype=np.float64).reshape(2, 2, 2)
    return r[..., 0] + 1j * r[..., 1]


def haar_unitary(rng: np.random.Generator) -> np.ndarray:
    """Haar-random 2x2 unitary (Mezzadri 2007): QR of a complex Ginibre
    matrix with the phases of R's diagonal divided out."""
    z = (rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    return q * (d / np.abs(d))


def empty_ops(count: int) -> np.ndarray:
    ops = np.zeros(count, dtype=OP_DTYPE)
    ops["control"] = -1
    ops["param"] = -1
    return ops


def op_u(k: int, q: np.ndarray) -> np.ndarray:
    op = empty_ops(1)
    op["kind"], op["target"], op["mat"][0] = OP_U, k, mat_to_row(q)
    return op


def op_cu(c: int, t: int, q: np.ndarray) -> np.ndarray:
    op = empty_ops(1)
    op["kind"], op["target"], op["control"], op["mat"][0] = OP_CU, t, c, mat_to_row(q)
    return op


def op_rot(kind: int, k: int, param: int) -> np.ndarray:
    op = empty_ops(1)
    op["kind"], op["target"], op["param"] = kind, k, param
    return op


@dataclass
class Circuit:
    n: int
    ops: np.ndarray                 # OP_DTYPE records
    nparams: int = 0
    theta: np.ndarray | None = None  # float64[nparams] (parameterised circuits)

    def __len__(self) -> int:
        return len(self.ops)


@dataclass
class PauliSum:
    codes: np.ndarray   # uint8 (nterms, n): 0 = I, 1 = X, 2 = Y, 3 = Z
    coeff: np.ndarray   # float64 (nterms,)

    @property
    def nterms(self) -> int:
        return int(self.coeff.shape[0])

    @property
    def n(self) -> int:
        return int(self.codes.shape[1])


def random_circuit(n: int, ngates: int, rng: np.random.Generator) -> Circuit:
    """The random mix of the gate workloads: each gate is, with probability
    1/2, a Haar-random 1-qubit gate on a uniform random qubit, otherwise a
    controlled Haar-random U on a uniform ordered pair of distinct qubits."""
    if n < 2:
        raise ValueError("random_circuit needs n >= 2")
    ops = empty_ops(ngates)
    for g in range(ngates):
        if rng.random() < 0.5:
            k = int(rng.integers(n))
            ops[g] = op_u(k, haar_unitary(rng))[0]
        else:
            c, t = (int(v) for v in rng.choice(n, size=2, replace=False))
            ops[g] = op_cu(c, t, haar_unitary(rng))[0]
    return Circuit(n, ops)


def qft_circuit(n: int) -> Circuit:
    """QFT without the final qubit-order reversal (qHiPSTER Sec. 5.5 / Table 3
    counts n(n+1)/2 gates, i.e. no swaps): for q = n-1 down to 0, H on q,
    then for p = q-1 down to 0 a controlled phase diag(1, exp(2 pi i /
    2^(q-p+1))) with control p and target q."""
    ops = []
    for q in range(n - 1, -1, -1):
        ops.append(op_u(q, H_GATE))
        for p in range(q - 1, -1, -1):
            phase = np.exp(2j * math.pi / 2.0 ** (q - p + 1))
            ops.append(op_cu(p, q, np.diag([1.0, phase])))
    return Circuit(n, np.concatenate(ops) if ops else empty_ops(0))


def iqft_circuit(n: int) -> Circuit:
    """Inverse QFT (qHiPSTER Fig. 6): n stages; stage i applies the inverse
    controlled phases controlled by the higher qubits i+1 .. n-1 and then H on
    qubit i.  It is the gate-by-gate inverse of qft_circuit (reversed order,
    conjugated phases; H is its own inverse)."""
    fwd = qft_circuit(n).ops[::-1].copy()
    for op in fwd:
        q = row_to_mat(op["mat"])
        op["mat"] = mat_to_row(q.conj().T)
    return Circuit(n, fwd)


def ansatz_circuit(n: int, layers: int, rng: np.random.Generator | None = None) -> Circuit:
    """Hardware-efficient ansatz: every layer applies RY(theta) to each qubit,
    then RZ(theta) to each qubit, then a CNOT ladder i -> i+1 for i = 0..n-2.
    Every rotation has its own parameter (P = 2 n L); theta ~ U[0, 2 pi)."""
    per_layer = 3 * n - 1
    ops = empty_ops(layers * per_layer)
    q = np.arange(n, dtype=np.int32)
    x_row = mat_to_row(X_GATE)
    p = 0
    for layer in range(layers):
        base = layer * per_layer
        ry = ops[base:base + n]
        ry["kind"], ry["target"], ry["param"] = OP_RY, q, p + q
        p += n
        rz = ops[base + n:base + 2 * n]
        rz["kind"], rz["target"], rz["param"] = OP_RZ, q, p + q
        p += n
        cx = ops[base + 2 * n:base + per_layer]
        cx["kind"], cx["control"], cx["target"] = OP_CU, q[:-1], q[:-1] + 1
        cx["mat"] = x_row
    theta = None
    if rng is not None:
        theta = rng.uniform(0.0, 2.0 * math.pi, size=p)
    return Circuit(n, ops, nparams=p, theta=theta)


def random_pauli_sum(n: int, nterms: int, rng: np.random.Generator,
                     max_weight: int = 4) -> PauliSum:
    """nterms random Pauli strings: weight w uniform in 1..min(max_weight, n),
    w distinct uniform qubits, each factor uniform over X, Y, Z; N(0, 1)
    coefficients."""
    codes = np.zeros((nterms, n), dtype=np.uint8)
    for j in range(nterms):
        w = int(rng.integers(1, min(max_weight, n) + 1))
        qs = rng.choice(n, size=w, replace=False)
        codes[j, qs] = rng.integers(1, 4, size=w).astype(np.uint8)
    coeff = rng.standard_normal(nterms)
    return PauliSum(codes, coeff)


# ---------------------------------------------------------------- workloads

def workload_gates(n: int = 20, ngates: int = 200, seed: int = SEED_BASE) -> Circuit:
    """Random 1q / controlled-U mix on |0...0> (n = 20, 200 gates)."""
    return random_circuit(n, ngates, np.random.default_rng(seed))


def workload_sweep(n: int = 30, ncu: int = 64, seed: int = SEED_BASE + 1):
    """Per-gate sweep at n qubits: H and one Haar U on every target, CU(U) on
    ncu random ordered (c, t) pairs.  Returns (u, pairs)."""
    rng = np.random.default_rng(seed)
    u = haar_unitary(rng)
    pairs = [tuple(int(v) for v in rng.choice(n, size=2, replace=False)) for _ in range(ncu)]
    return u, pairs


def workload_circuit_qft(n: int, ngates: int = 500, seed: int = SEED_BASE + 2) -> Circuit:
    """A random circuit of the gate mix followed by a QFT on all qubits."""
    rc = random_circuit(n, ngates, np.random.default_rng(seed))
    q = qft_circuit(n)
    return Circuit(n, np.concatenate([rc.ops, q.ops]))


def workload_ansatz(n: int, layers: int = 20, nterms: int = 100,
                    seed: int = SEED_BASE + 3):
    """Parameterised ansatz with theta ~ U[0, 2 pi) and a random Pauli sum."""
    rng = np.random.default_rng(seed)
    circ = ansatz_circuit(n, layers, rng)
    ham = random_pauli_sum(n, nterms, rng)
    return circ, ham


def workload_batch(ncircuits: int = 4096, nmin: int = 10, nmax: int = 18,
                   lmin: int = 5, lmax: int = 30, nterms: int = 20,
                   seed_base: int = BATCH_SEED_BASE):
    """Independent ansatz circuits of uneven width and depth, each with its
    own theta and its own Pauli sum.  Returns a list of (Circuit, PauliSum)."""
    out = []
    for j in range(ncircuits):
        rng = np.random.default_rng(seed_base + j)
        n = int(rng.integers(nmin, nmax + 1))
        layers = int(rng.integers(lmin, lmax + 1))
        circ = ansatz_circuit(n, layers, rng)
        ham = random_pauli_sum(n, nterms, rng)
        out.append((circ, ham))
    return out


def basis_index_of(bits: dict) -> int:
    """Amplitude index of the computational basis state with the given qubit
    values (qubit q is bit q)."""
    return sum(1 << q for q, b in bits.items() if b)
