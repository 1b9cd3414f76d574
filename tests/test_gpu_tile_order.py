"""Tile order of compiled passes: every order (2^k regions of tiles walked
side by side) and the tuner that times them and keeps the fastest must give
bit-identical states and gradients (the order only decides which workgroup
takes which tile), and those must match the oracle within the usual
bounds."""
from __future__ import annotations

import math

import numpy as np
import pytest

import circuits as C
import oracle as O
from tests.gpu_util import Q, random_state, rounded_input, to_gpu_state  # noqa: F401

pytestmark = pytest.mark.gpu

# forced orders k = 0..4, then "" (the tuner): each run times the next
# order (each run ends with a host copy, so the last timing has completed),
# until every order the tile count allows (at most five at 32 tiles) is
# timed; the runs after that take the fastest
ORDERS = ("0", "1", "2", "3", "4") + ("",) * 7


def dt(Q, name):
    return Q.QS_C128 if name == "c128" else Q.QS_C64


# 16 and 32 tiles of 2^11 (complex128) or 2^12 (complex64) amplitudes:
# four and five distinct orders
@pytest.mark.parametrize("name,n", [("c128", 15), ("c128", 16), ("c64", 16), ("c64", 17)])
def test_tile_orders_forward(Q, name, n, monkeypatch):
    monkeypatch.setenv("QS_FUSED_EXEC", "compiled")
    rng = np.random.default_rng(900 + n)
    ops = np.concatenate([C.random_circuit(n, 300, rng).ops, C.qft_circuit(n).ops])
    psi = random_state(n, rng)
    outs = []
    for order in ORDERS:
        monkeypatch.setenv("QS_TILE_ORDER", order)
        st = to_gpu_state(Q, psi, dt(Q, name))
        st.run(ops)
        outs.append(st.numpy())
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    ref = O.run(ops, n, psi=rounded_input(psi, name == "c64"))
    bound = 1e-12 if name == "c128" else 2e-7 * math.sqrt(len(ops)) + 1e-6
    assert np.abs(outs[0] - ref).max() <= bound


@pytest.mark.parametrize("name,n", [("c128", 16), ("c64", 17)])
def test_tile_orders_adjoint(Q, name, n, monkeypatch):
    """Gradient partials are kept per tile, so the sum over them, and the
    gradient, are the same in either order."""
    monkeypatch.setenv("QS_FUSED_EXEC", "compiled")
    circ, ham = C.workload_ansatz(n, 2, 20, seed=950 + n)
    res = []
    for order in ORDERS:
        monkeypatch.setenv("QS_TILE_ORDER", order)
        st = Q.State(n, dt(Q, name))
        lam = Q.State(n, dt(Q, name), init=False)
        res.append(Q.grad_adjoint(st, lam, circ.ops, circ.theta, ham.codes, ham.coeff))
    for e, g in res[1:]:
        assert e == res[0][0] and np.array_equal(g, res[0][1])
    e, g = res[0]
    sample = [0, 7, circ.nparams // 2, circ.nparams - 1]
    rg = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff, params=sample)
    re = O.energy(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    if name == "c128":
        assert abs(e - re) <= 1e-12 and np.abs(g[sample] - rg[sample]).max() <= 1e-10
    else:
        scale = max(1.0, np.abs(ham.coeff).sum())
        assert abs(e - re) <= 1e-4 * scale and np.abs(g[sample] - rg[sample]).max() <= 1e-4 * scale
