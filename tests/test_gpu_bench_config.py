"""The benchmark's step at its full size and launch configuration (n = 30
complex128, also n = 31 complex64), where the oracle cannot run whole:
after the per-gate sweep (H then the Haar U on every target) sampled
amplitudes must equal the product-state closed form (one-qubit factors from
the oracle); the controlled-U pairs and the 1000-gate fused circuit follow,
the norm must hold, and the inverse of everything, applied in reverse
order, must return |0...0>."""
from __future__ import annotations

import numpy as np
import pytest

import circuits as C
import oracle as O
from tests.gpu_util import Q  # noqa: F401

pytestmark = pytest.mark.gpu


def _dagger_ops(ops):
    inv = ops[::-1].copy()
    for g in range(len(inv)):
        inv[g]["mat"] = C.mat_to_row(C.row_to_mat(inv[g]["mat"]).conj().T)
    return inv


@pytest.mark.parametrize("name,n", [("c128", 30), ("c64", 31)])
def test_bench_step_full_size(Q, name, n):
    import torch
    dt = Q.QS_C128 if name == "c128" else Q.QS_C64
    seed = C.SEED_BASE + 1
    u, pairs = C.workload_sweep(n, 64, seed)
    circ = C.random_circuit(n, 1000, np.random.default_rng(seed))
    st = Q.State(n, dt)
    for k in range(n):
        st.apply_1q(k, C.H_GATE)
        st.apply_1q(k, u)
    # product form: every qubit in u H |0>
    f = O.apply_1q(O.apply_1q(O.basis_state(1, 0), 1, 0, C.H_GATE), 1, 0, u)
    rng = np.random.default_rng(1900 + n)
    idx = rng.integers(0, 1 << n, 4096, dtype=np.int64)
    ones = np.array([bin(int(i)).count("1") for i in idx])
    ref = f[0] ** (n - ones) * f[1] ** ones
    got = st.tensor[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
    tol = 1e-14 if name == "c128" else 1e-9
    assert np.abs(got - ref).max() <= tol
    for c, t in pairs:
        st.apply_cu(c, t, u)
    info, _, _ = Q.qs_plan(n, dt, circ.ops)
    assert info["fused"] == info["passes"] and info["passes"] > 40
    st.run(circ.ops)
    _, nrm, _ = st.probabilities()
    assert abs(nrm - 1.0) <= (1e-12 if name == "c128" else 1e-4)
    # back to |0...0>
    st.run(_dagger_ops(circ.ops))
    ud = u.conj().T
    for c, t in reversed(pairs):
        st.apply_cu(c, t, ud)
    for k in reversed(range(n)):
        st.apply_1q(k, ud)
        st.apply_1q(k, C.H_GATE)
    p1, nrm, _ = st.probabilities()
    a0 = complex(st.tensor[0].item())
    if name == "c128":
        assert abs(a0 - 1.0) <= 1e-11 and p1.max() <= 1e-20
    else:
        assert abs(a0 - 1.0) <= 1e-3 and p1.max() <= 1e-6
    del st
    torch.cuda.empty_cache()
