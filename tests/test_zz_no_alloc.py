"""The allocation-free probabilities entry point, called through the C ABI:
its outputs equal those of qs_probabilities (same kernels, same fixed-order
sums, so bit for bit) and the oracle's, on two calls in a row, the second on
a smaller state, for both amplitude types; and it refuses host outputs."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import Q, random_state, to_gpu_state  # noqa: F401

pytestmark = pytest.mark.gpu


def _noalloc(Q, st, full=True):
    import torch
    p1 = torch.full((st.n,), -1.0, dtype=torch.float64, device="cuda")
    nrm = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    ft = torch.full((1 << st.n,), -1.0, dtype=torch.float64, device="cuda") if full else None
    rc = Q.lib().qs_probabilities_noalloc(
        ctypes.c_void_p(st.handle), ctypes.c_void_p(p1.data_ptr()), ctypes.c_void_p(nrm.data_ptr()),
        ctypes.c_void_p(ft.data_ptr() if full else 0), (1 << st.n) * 8 if full else 0)
    assert rc == Q.QS_OK, Q.qs_last_error()
    st.stream.synchronize()
    return p1.cpu().numpy(), float(nrm.item()), (ft.cpu().numpy() if full else None)


@pytest.mark.parametrize("name", ["c128", "c64"])
def test_noalloc_matches_probabilities_on_two_calls(Q, name):
    dtype = Q.QS_C128 if name == "c128" else Q.QS_C64
    rng = np.random.default_rng(7070)
    for n in (22, 13):  # the second call on a smaller state
        psi = random_state(n, rng)
        st = to_gpu_state(Q, psi, dtype)
        p1, nrm, full = _noalloc(Q, st)
        rp1, rnrm, rfull = st.probabilities(full=True)
        rfull = rfull.cpu().numpy()
        assert np.array_equal(p1, rp1) and nrm == rnrm and np.array_equal(full, rfull)
        held = st.numpy()  # the amplitudes the GPU holds (complex64 rounding)
        op1, onrm, ofull = O.probabilities(held, n, full=True)
        assert np.abs(p1 - op1).max() <= 1e-12 and abs(nrm - onrm) <= 1e-12
        assert np.abs(full - ofull).max() <= 1e-15
        # sums only (no full vector) give the same values
        p1b, nrmb, _ = _noalloc(Q, st, full=False)
        assert np.array_equal(p1b, p1) and nrmb == nrm
        st.close()


def test_noalloc_rejects_host_outputs(Q):
    import torch
    st = Q.State(12, Q.QS_C128)
    host = np.zeros(12, dtype=np.float64)
    rc = Q.lib().qs_probabilities_noalloc(ctypes.c_void_p(st.handle), ctypes.c_void_p(host.ctypes.data),
                                          None, None, 0)
    assert rc == Q.QS_EINVAL and "not device memory" in Q.qs_last_error()
    small = torch.zeros(10, dtype=torch.float64, device="cuda")
    rc = Q.lib().qs_probabilities_noalloc(ctypes.c_void_p(st.handle), None, None,
                                          ctypes.c_void_p(small.data_ptr()), 10 * 8)
    assert rc == Q.QS_ERANGE
