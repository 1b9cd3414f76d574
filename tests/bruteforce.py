"""Brute-force dense operators for tiny n: the full 2^n x 2^n matrices that the
simulator deliberately never builds (qHiPSTER Eq. 1).  Used to pin the CPU
oracle from outside; independent of both the oracle and the GPU library.

Kronecker order: qubit k is bit k of the index, so the factor acting on qubit
k sits at position n-1-k from the left:
    U_k = I^(n-1-k) (x) Q (x) I^(k).
"""
from __future__ import annotations

import numpy as np

P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
I2 = np.eye(2, dtype=np.complex128)
PAULI = {
    0: I2,
    1: np.array([[0, 1], [1, 0]], dtype=np.complex128),
    2: np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    3: np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def kron_chain(factors_by_qubit: dict, n: int) -> np.ndarray:
    """Tensor product with factors_by_qubit[q] on qubit q (identity elsewhere)."""
    out = np.ones((1, 1), dtype=np.complex128)
    for q in range(n - 1, -1, -1):
        out = np.kron(out, factors_by_qubit.get(q, I2))
    return out


def kron_1q(n: int, k: int, q: np.ndarray) -> np.ndarray:
    return kron_chain({k: np.asarray(q, dtype=np.complex128)}, n)


def kron_cu(n: int, c: int, t: int, q: np.ndarray) -> np.ndarray:
    """|0><0|_c (x) I_t + |1><1|_c (x) Q_t."""
    return kron_chain({c: P0}, n) + kron_chain({c: P1, t: np.asarray(q, dtype=np.complex128)}, n)


def kron_pauli(codes_row) -> np.ndarray:
    n = len(codes_row)
    return kron_chain({q: PAULI[int(c)] for q, c in enumerate(codes_row)}, n)


def kron_hamiltonian(codes: np.ndarray, coeff) -> np.ndarray:
    n = codes.shape[1]
    h = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for row, c in zip(codes, coeff):
        h += c * kron_pauli(row)
    return h


def random_state(n: int, rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return (v / np.linalg.norm(v)).astype(np.complex128)
