"""GPU parity of qubit reordering (Sec. 6) through the C ABI: the in-place
permutation kernels against the oracle's qubit relabelling, bit for bit
(pure data movement), at sizes that span single tiles, several tiles and a
ragged number of upper qubits, and at the bandwidth-scale sizes the
benchmark times (sampled amplitudes, and a round trip through the inverse);
and the reordered runner against the oracle and against the plain run."""
from __future__ import annotations

import math

import numpy as np
import pytest

import circuits as C
import oracle as O
from tests.gpu_util import Q, random_state, rounded_input, to_gpu_state  # noqa: F401

pytestmark = pytest.mark.gpu


def dt(Q, name):
    return Q.QS_C128 if name == "c128" else Q.QS_C64


def bound(name, ngates):
    return 1e-12 if name == "c128" else 2e-7 * math.sqrt(ngates) + 1e-6


def _swap(n, a, b):
    p = list(range(n))
    p[a], p[b] = b, a
    return p


def perm_cases(n, rng):
    """Permutations of n qubits that reach every launch form: the identity,
    swaps inside the low block bits, between a block bit and an upper qubit
    and between two upper qubits, cycles, the reversal, more than four swaps
    that touch the block bits, and random permutations."""
    cases = {"identity": list(range(n)), "reverse": list(range(n))[::-1],
             "cycle": [(q + 1) % n for q in range(n)]}
    for a, b in ((0, 1), (0, n - 1), (2, 5), (5, 6), (3, 9), (6, 13), (7, n - 1), (8, 12)):
        if a < n and b < n and a != b:
            cases[f"swap{a}_{b}"] = _swap(n, a, b)
    if n >= 3:
        p = list(range(n))
        p[0], p[1], p[2] = 1, 2, 0
        cases["3cycle_low"] = p
    if n >= 14:
        p = list(range(n))
        for q in range(7):
            p[q], p[q + 7] = q + 7, q
        cases["seven_block_swaps"] = p
    for s in range(3):
        cases[f"random{s}"] = [int(x) for x in rng.permutation(n)]
    return cases


@pytest.mark.parametrize("name", ["c128", "c64"])
@pytest.mark.parametrize("n", [1, 2, 5, 6, 7, 8, 11, 14, 17])
def test_permute_vs_oracle_bitwise(Q, name, n):
    rng = np.random.default_rng(1500 + n)
    psi = rounded_input(random_state(n, rng), name == "c64")
    for label, perm in perm_cases(n, rng).items():
        st = to_gpu_state(Q, psi, dt(Q, name))
        st.permute_qubits(perm)
        ref = O.permute_qubits(psi.copy(), n, perm)
        assert np.array_equal(st.numpy(), ref), (label, perm)


def _moved_index(i, perm):
    j = np.zeros_like(i)
    for q, p in enumerate(perm):
        j |= ((i >> q) & 1) << p
    return j


@pytest.mark.parametrize("name,n", [("c128", 28), ("c64", 29), ("c128", 30)])
def test_permute_large_sampled_and_round_trip(Q, name, n):
    """Sampled amplitudes land where the relabelling sends them, and the
    inverse relabelling restores the state bit for bit.  The 3-swap case is
    the shape of one reordering of a state split by its top 3 qubits (the
    benchmark's launch)."""
    import torch
    rng = np.random.default_rng(1600 + n)
    st = Q.State(n, dt(Q, name), init=False)
    gen = torch.Generator(device="cuda").manual_seed(1600 + n)
    st.tensor.real.copy_(torch.randn(1 << n, device="cuda", generator=gen))
    st.tensor.imag.copy_(torch.randn(1 << n, device="cuda", generator=gen))
    before = st.tensor.clone()
    samples = torch.from_numpy(rng.integers(0, 1 << n, 4096, dtype=np.int64)).cuda()
    cases = {"three_upper_swaps": list(range(n)), "low_and_upper": _swap(n, 0, n - 1),
             "random": [int(x) for x in rng.permutation(n)]}
    for a, b in ((n - 1, 9), (n - 2, 8), (n - 3, 7)):
        cases["three_upper_swaps"][a], cases["three_upper_swaps"][b] = b, a
    for label, perm in cases.items():
        st.permute_qubits(perm)
        dst = torch.from_numpy(_moved_index(samples.cpu().numpy(), perm)).cuda()
        assert torch.equal(st.tensor[dst], before[samples]), label
        inv = [0] * n
        for q in range(n):
            inv[perm[q]] = q
        st.permute_qubits(inv)
        assert torch.equal(st.tensor, before), label
    del before, st
    torch.cuda.empty_cache()


def test_permute_rejects_bad_arguments(Q):
    st = Q.State(5, Q.QS_C128)
    for perm in ([0, 1, 2, 3, 3], [0, 1, 2, 3, 5], [-1, 0, 1, 2, 3]):
        with pytest.raises(Q.QSError) as ei:
            Q.qs_permute_qubits(st.handle, perm)
        assert ei.value.code == Q.QS_EINVAL


def _circuit(kind, n, seed):
    if kind == "random":
        return C.random_circuit(n, 300, np.random.default_rng(seed)).ops, None
    if kind == "qft":
        return C.qft_circuit(n).ops, None
    circ, _ = C.workload_ansatz(n, 3, 4, seed=seed)
    return circ.ops, circ.theta


@pytest.mark.parametrize("name,n", [("c128", 12), ("c128", 15), ("c64", 14)])
@pytest.mark.parametrize("kind", ["random", "qft", "ansatz"])
@pytest.mark.parametrize("upper", [1, 3, 5])
def test_run_reordered_vs_oracle(Q, name, n, kind, upper):
    rng = np.random.default_rng(1700 + n + upper)
    ops, theta = _circuit(kind, n, 1701 + n)
    psi = random_state(n, rng)
    st = to_gpu_state(Q, psi, dt(Q, name))
    info = st.run_reordered(ops, n - upper, theta)
    ref = O.run(ops, n, theta, psi=rounded_input(psi, name == "c64"))
    assert np.abs(st.numpy() - ref).max() <= bound(name, len(ops))
    plan, *_ = Q.qs_plan_reorder(n, n - upper, ops, theta)
    assert info == plan


@pytest.mark.parametrize("name,n", [("c128", 24), ("c64", 25)])
def test_run_reordered_equals_plain_run(Q, name, n):
    ops = C.workload_circuit_qft(n, 500).ops
    a = Q.State(n, dt(Q, name))
    a.run(ops)
    b = Q.State(n, dt(Q, name))
    info = b.run_reordered(ops, n - 3)
    assert info["remaps"] > 0
    err = float((a.tensor - b.tensor).abs().max())
    assert err <= (1e-12 if name == "c128" else 1e-5), err
