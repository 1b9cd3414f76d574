"""Oracle parity at the workloads' own sizes.

- The differentiation workload: the hardware-efficient ansatz with L = 20
  layers and 100 Pauli strings (seed 1604) at n = 20, checked against the
  oracle's energy, its parameter-shift gradient on sampled parameters from
  the first, middle and last layers, and central finite differences of
  oracle energies; at n = 24 (the largest the host oracle finishes within a
  test's budget) the energy and one parameter-shift entry; at n = 28 the
  properties that hold at any size (adjoint against parameter shift on the
  same GPU, the state returned to |0...0>).
- The batching workload: the full 4096-circuit batch in one persistent
  launch, eight of its circuits (among them the widest and the deepest)
  checked against the oracle, complex128 and complex64.
- A reverse sweep whose passes would hold more than the per-pass gradient
  slots, and the persistent-grid branches (forced with a grid limit at small
  n, and reached by size at n = 31 / 32 with closed-form gradients).

Tolerances: complex128 energies 1e-12, gradients 1e-10 against parameter
shift, 1e-6 relative against central differences.  complex64 states carry
their own rounding (about 1e-7 relative per gate); their energy and gradient
errors against the FP64 oracle are printed and bounded loosely by
1e-4 * sum |c_j|.
"""
from __future__ import annotations

import os

import numpy as np
import pytest

import circuits as C
import oracle as O
from tests.gpu_util import Q  # noqa: F401

pytestmark = pytest.mark.gpu

L_LAYERS, NTERMS = 20, 100


def _oracle_threads():
    O.set_threads(max(1, min(16, os.cpu_count() or 1)))


def _adjoint(Q, circ, ham, dtype, grid_limit=0):
    st = Q.State(circ.n, dtype)
    lam = Q.State(circ.n, dtype, init=False)
    if grid_limit:
        st.set_grid_limit(grid_limit)
    e, g = Q.grad_adjoint(st, lam, circ.ops, circ.theta, ham.codes, ham.coeff)
    return e, g, st


def _sample_params(n, layers):
    per = 2 * n
    first = [0, n // 3, n - 1, n, n + n // 2, 2 * n - 1]
    mid = [(layers // 2) * per + j for j in (1, n // 2, n + 3)]
    last = [(layers - 1) * per + j for j in (0, n // 2 + 1, n - 1, n, n + n // 3, 2 * n - 1)]
    return sorted(set(first + mid + last + [per + 2]))


_cache = {}


def _config3(n):
    if n not in _cache:
        _cache[n] = C.workload_ansatz(n, L_LAYERS, NTERMS, seed=C.SEED_BASE + 3)
    return _cache[n]


def _oracle_ps(n, params):
    key = ("ps", n, tuple(params))
    if key not in _cache:
        circ, ham = _config3(n)
        _oracle_threads()
        _cache[key] = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff, params=params)
    return _cache[key]


def _oracle_energy(n):
    key = ("e", n)
    if key not in _cache:
        circ, ham = _config3(n)
        _oracle_threads()
        _cache[key] = O.energy(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    return _cache[key]


def test_config3_n20_energy_and_parameter_shift(Q):
    n = 20
    circ, ham = _config3(n)
    assert circ.nparams == 800 and len(circ.ops) == 1180 and len(ham.coeff) == 100
    params = _sample_params(n, L_LAYERS)
    assert len(params) >= 16 and params[0] == 0 and params[-1] == circ.nparams - 1
    e, g, st = _adjoint(Q, circ, ham, Q.QS_C128)
    re = _oracle_energy(n)
    rg = _oracle_ps(n, params)
    err_e, err_g = abs(e - re), float(np.abs(g[params] - rg[params]).max())
    print(f"config3 n=20 c128: |dE| {err_e:.2e}, max |dg| {err_g:.2e} over {len(params)} params")
    assert err_e <= 1e-12
    assert err_g <= 1e-10
    # the reverse sweep takes the state back to |0...0>
    psi = st.numpy()
    assert abs(psi[0] - 1.0) <= 1e-10 and np.abs(psi[1:]).max() <= 1e-10


def test_config3_n20_central_differences(Q):
    n = 20
    circ, ham = _config3(n)
    params = [0, 2 * n - 1, 10 * 2 * n + 5, circ.nparams - 1]
    _, g, _ = _adjoint(Q, circ, ham, Q.QS_C128)
    _oracle_threads()
    fd = O.grad_central_fd(circ.ops, n, circ.theta, ham.codes, ham.coeff, h=1e-5, params=params)
    err = float(np.abs(g[params] - fd[params]).max())
    print(f"config3 n=20 c128 vs central FD: {err:.2e}")
    assert err <= 1e-6 * max(1.0, float(np.abs(fd[params]).max()))


def test_config3_n20_complex64_error_against_fp64_oracle(Q):
    n = 20
    circ, ham = _config3(n)
    params = _sample_params(n, L_LAYERS)
    e, g, _ = _adjoint(Q, circ, ham, Q.QS_C64)
    re = _oracle_energy(n)
    rg = _oracle_ps(n, params)
    err_e, err_g = abs(e - re), float(np.abs(g[params] - rg[params]).max())
    scale = max(1.0, float(np.abs(ham.coeff).sum()))
    print(f"config3 n=20 c64 vs FP64 oracle: |dE| {err_e:.2e}, max |dg| {err_g:.2e} (sum|c| {scale:.1f})")
    assert err_e <= 1e-4 * scale and err_g <= 1e-4 * scale


def test_config3_n24_energy_and_parameter_shift(Q):
    """The ansatz form at n = 24: L = 20, 1420 gates, 960 parameters."""
    n = 24
    circ, ham = _config3(n)
    e, g, _ = _adjoint(Q, circ, ham, Q.QS_C128)
    params = [circ.nparams - 2 * n + 3]  # an RY of the last layer
    re = _oracle_energy(n)
    rg = _oracle_ps(n, params)
    print(f"config3 n=24 c128: |dE| {abs(e - re):.2e}, |dg| {abs(g[params[0]] - rg[params[0]]):.2e}")
    assert abs(e - re) <= 1e-12
    assert abs(g[params[0]] - rg[params[0]]) <= 1e-10


def test_config3_n28_adjoint_against_parameter_shift_on_the_gpu(Q):
    """n = 28, L = 20, 1660 gates, 1120 parameters: beyond the host oracle's
    test budget, so the checks are identities that hold at any size --
    the adjoint gradient equals the parameter-shift rule evaluated with the
    GPU's own forward sweeps (a different method on the same kernels), the
    adjoint energy equals qs_run + qs_expect_pauli, and the reverse sweep
    returns the state to |0...0>."""
    n = 28
    circ, ham = _config3(n)
    assert circ.nparams == 1120 and len(circ.ops) == 1660
    e, g, st = _adjoint(Q, circ, ham, Q.QS_C128)
    psi0 = st.tensor
    assert abs(complex(psi0[0].item()) - 1.0) <= 1e-10
    del st, psi0

    def energy(theta):
        s = Q.State(n, Q.QS_C128)
        s.run(circ.ops, theta)
        return s.expect(ham.codes, ham.coeff)

    e_run = energy(circ.theta)
    assert abs(e - e_run) <= 1e-12
    for p in (0, circ.nparams - 1):
        tp, tm = circ.theta.copy(), circ.theta.copy()
        tp[p] += np.pi / 2
        tm[p] -= np.pi / 2
        ps = 0.5 * (energy(tp) - energy(tm))
        print(f"config3 n=28 param {p}: adjoint {g[p]:.15f} shift {ps:.15f}")
        assert abs(g[p] - ps) <= 1e-10


def _batch_sample(items):
    ns = np.array([it[0] for it in items])
    depth = np.array([len(it[1]) for it in items])
    widest_deepest = int(np.argmax(depth + (ns == ns.max()) * 10 ** 6))
    deepest = int(np.argmax(depth))
    smallest = int(np.argmin(depth))
    rng = np.random.default_rng(4096)
    pick = [widest_deepest, deepest, smallest] + [int(i) for i in rng.choice(len(items), 8, replace=False)]
    out = []
    for i in pick:
        if i not in out:
            out.append(i)
    return out[:8]


@pytest.fixture(scope="module")
def batch_workload():
    wl = C.workload_batch()
    items = [(c.n, c.ops, c.theta, h.codes, h.coeff) for c, h in wl]
    return items


@pytest.mark.parametrize("name", ["c128", "c64"])
def test_config4_full_batch_against_oracle(Q, batch_workload, name):
    items = batch_workload
    assert len(items) == 4096
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    b = Q.Batch(items, dtype)
    e, g = b.run()
    b.close()
    sample = _batch_sample(items)
    ns = [items[i][0] for i in sample]
    assert max(ns) == 18
    _oracle_threads()
    worst_e = worst_g = 0.0
    for i in sample:
        n, ops, th, codes, coeff = items[i]
        nparams = len(th)
        params = sorted({0, 1, n, nparams // 2, nparams - n - 1, nparams - 1})
        re = O.energy(ops, n, th, codes, coeff)
        rg = O.grad_param_shift(ops, n, th, codes, coeff, params=params)
        de, dg = abs(e[i] - re), float(np.abs(g[i][params] - rg[params]).max())
        worst_e, worst_g = max(worst_e, de), max(worst_g, dg)
        if name == "c128":
            assert de <= 1e-12, (i, n, de)
            assert dg <= 1e-10, (i, n, dg)
        else:
            scale = max(1.0, float(np.abs(coeff).sum()))
            assert de <= 1e-4 * scale and dg <= 1e-4 * scale, (i, n, de, dg)
    print(f"config4 {name}: circuits {sample} (n {ns}); max |dE| {worst_e:.2e}, max |dg| {worst_g:.2e}")


@pytest.mark.parametrize("mode", ["interpreted", "compiled"])
@pytest.mark.parametrize("name,n,layers", [("c128", 12, 6), ("c64", 13, 6)])
def test_adjoint_passes_split_at_the_gradient_slot_limit(Q, name, n, layers, mode, monkeypatch):
    monkeypatch.setenv("QS_FUSED_EXEC", mode)
    """Every rotation of these circuits fits one fused pass by its qubits,
    but a pass carries at most 64 gradient slots, so the sweep splits; all
    2nL parameters are checked."""
    circ, ham = C.workload_ansatz(n, layers, 30, seed=3100 + n)
    assert circ.nparams > 64
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    e, g, _ = _adjoint(Q, circ, ham, dtype)
    rg = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    re = O.energy(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    if name == "c128":
        assert abs(e - re) <= 1e-12 and np.abs(g - rg).max() <= 1e-10
    else:
        scale = max(1.0, float(np.abs(ham.coeff).sum()))
        assert abs(e - re) <= 1e-4 * scale and np.abs(g - rg).max() <= 1e-4 * scale


@pytest.mark.parametrize("mode", ["interpreted", "compiled"])
@pytest.mark.parametrize("name,n,limit", [("c128", 14, 3), ("c128", 15, 5), ("c64", 14, 1),
                                          ("c64", 15, 3)])
def test_persistent_grid_forced_by_a_grid_limit(Q, name, n, limit, mode, monkeypatch):
    monkeypatch.setenv("QS_FUSED_EXEC", mode)
    """A grid limit below the tile count makes each workgroup loop over
    several tiles (the branch large states take), in the forward passes and
    in the reverse sweep, whose gradient partials then accumulate across
    tiles before one sum over all slots."""
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    circ, ham = C.workload_ansatz(n, 3, 30, seed=3200 + n)
    e, g, st = _adjoint(Q, circ, ham, dtype, grid_limit=limit)
    e0, g0, _ = _adjoint(Q, circ, ham, dtype)
    sample = list(range(0, circ.nparams, 3))
    rg = O.grad_param_shift(circ.ops, n, circ.theta, ham.codes, ham.coeff, params=sample)
    re = O.energy(circ.ops, n, circ.theta, ham.codes, ham.coeff)
    assert e == e0  # the forward sweep and energy do not depend on the grid
    if name == "c128":
        assert abs(e - re) <= 1e-12
        assert np.abs(g[sample] - rg[sample]).max() <= 1e-10
        assert np.abs(g - g0).max() <= 1e-12
    else:
        scale = max(1.0, float(np.abs(ham.coeff).sum()))
        assert abs(e - re) <= 1e-4 * scale
        assert np.abs(g[sample] - rg[sample]).max() <= 1e-4 * scale
    # a forward fused run under the limit: bit for bit the unlimited run
    ops = C.random_circuit(n, 150, np.random.default_rng(3300 + n)).ops
    a = Q.State(n, dtype).set_grid_limit(limit).run(ops).numpy()
    b = Q.State(n, dtype).run(ops).numpy()
    assert np.array_equal(a, b)
    if name == "c128":
        assert np.abs(a - O.run(ops, n)).max() <= 1e-12


def _product_ansatz(n):
    """RY(a_q) then RZ(b_q) on every qubit, parameters a_q = q, b_q = n + q."""
    ops = np.concatenate([C.op_rot(C.OP_RY, q, q) for q in range(n)] +
                         [C.op_rot(C.OP_RZ, q, n + q) for q in range(n)])
    return ops


@pytest.mark.parametrize("name,n", [("c128", 31), ("c64", 32)])
def test_large_state_adjoint_closed_form(Q, name, n):
    """At n = 31 (complex128) / 32 (complex64) the reverse sweep has 2^20
    tiles and takes its persistent grid by size.  On the product state
    RY(a) RZ(b) |0>, <Z> = cos a, <X> = sin a cos b, <Y> = sin a sin b per
    qubit, so E = sum_q cz cos a + cx sin a cos b + cy sin a sin b and its
    derivatives are closed forms."""
    import torch
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    rng = np.random.default_rng(3400 + n)
    a = rng.uniform(0, 2 * np.pi, n)
    b = rng.uniform(0, 2 * np.pi, n)
    theta = np.concatenate([a, b])
    cz, cx, cy = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
    codes = np.zeros((3 * n, n), dtype=np.uint8)
    for q in range(n):
        codes[3 * q, q], codes[3 * q + 1, q], codes[3 * q + 2, q] = 3, 1, 2
    coeff = np.stack([cz, cx, cy], 1).reshape(-1)
    st = Q.State(n, dtype)
    lam = Q.State(n, dtype, init=False)
    e, g = Q.grad_adjoint(st, lam, _product_ansatz(n), theta, codes, coeff)
    e_ref = float(np.sum(cz * np.cos(a) + cx * np.sin(a) * np.cos(b) + cy * np.sin(a) * np.sin(b)))
    ga = -cz * np.sin(a) + cx * np.cos(a) * np.cos(b) + cy * np.cos(a) * np.sin(b)
    gb = -cx * np.sin(a) * np.sin(b) + cy * np.sin(a) * np.cos(b)
    g_ref = np.concatenate([ga, gb])
    err_e, err_g = abs(e - e_ref), float(np.abs(g - g_ref).max())
    print(f"n={n} {name}: |dE| {err_e:.2e}, max |dg| {err_g:.2e}")
    del st, lam
    torch.cuda.empty_cache()
    if name == "c128":
        assert err_e <= 1e-10 and err_g <= 1e-10
    else:
        scale = float(np.abs(coeff).sum())
        assert err_e <= 1e-4 * scale and err_g <= 1e-4 * scale
