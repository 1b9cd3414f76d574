"""Helpers shared by the GPU parity tests (no simulation arithmetic)."""
from __future__ import annotations

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("this test needs an MI355X GPU (run with -m 'not gpu' on a CPU host)")
    import paper_1601_07195_amd.qs as Q  # raises ImportError when libqs.so is missing
    return Q


@pytest.fixture(scope="module")
def Q():
    return require_gpu()


def to_gpu_state(Q, psi: np.ndarray, dtype: int):
    import torch
    tdt = torch.complex128 if dtype == Q.QS_C128 else torch.complex64
    n = int(np.log2(psi.size))
    t = torch.from_numpy(np.ascontiguousarray(psi)).to(device="cuda", dtype=tdt)
    return Q.State(n, dtype, tensor=t, init=False)


def rounded_input(psi: np.ndarray, dtype_is_c64: bool) -> np.ndarray:
    """The input as the GPU holds it (complex64 rounding), back in complex128."""
    if dtype_is_c64:
        return psi.astype(np.complex64).astype(np.complex128)
    return psi.copy()


def random_state(n: int, rng: np.random.Generator) -> np.ndarray:
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    return (v / np.linalg.norm(v)).astype(np.complex128)
