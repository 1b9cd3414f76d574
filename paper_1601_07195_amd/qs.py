"""Python binding of libqs, the MI355X state-vector simulator.

Thin ctypes marshalling over the C ABI declared in include/qs.h: the
module-level functions carry the C names (qs_create, qs_apply_1q, ...) and
only convert arguments; every step of the computation runs in the HIP
kernels of libqs.so.  PyTorch supplies device memory (tensors) and the
stream (torch.cuda.current_stream()).

The library must be built (python -m paper_1601_07195_amd.build); importing
this module without libqs.so raises ImportError -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loaded first: libqs binds to the HIP runtime torch already loaded

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqs.so")

QS_OK, QS_EINVAL, QS_ENOMEM, QS_EHIP, QS_ENODEV, QS_ERANGE, QS_EVERIFY = 0, -1, -2, -3, -4, -5, -6
QS_C64, QS_C128 = 1, 2
QS_MAX_QUBITS_C128, QS_MAX_QUBITS_C64 = 33, 34
QS_OP_U, QS_OP_CU, QS_OP_RX, QS_OP_RY, QS_OP_RZ = 0, 1, 2, 3, 4
QS_RUN_NO_FUSION = 1
QS_RUN_WIDE_TILES = 2
QS_RUN_VERIFY = 4
QS_PLAN_ADJOINT_REVERSE = 16
QS_ADJ_STATE_IS_FINAL = 1
QS_ADJ_WIDE_TILES = 2
QS_BATCH_MAX_QUBITS = 24
QS_KQ_MAX = 5
QS_NOALLOC_SCRATCH_BYTES = 2048 * 35 * 8 + 35 * 8
QS_EXEC_AUTO, QS_EXEC_INTERPRETED, QS_EXEC_COMPILED = 0, 1, 2
QS_PRECOMPILE_ADJOINT = 1

# Mirror of `struct qs_op` (80 bytes).
QS_OP_DTYPE = np.dtype([("kind", "<i4"), ("target", "<i4"), ("control", "<i4"),
                        ("param", "<i4"), ("mat", "<f8", (8,))])

EXPORTED = ("qs_version", "qs_strerror", "qs_last_error", "qs_create", "qs_destroy",
            "qs_set_stream", "qs_init_basis", "qs_apply_1q", "qs_apply_cu", "qs_run",
            "qs_probabilities", "qs_expect_pauli", "qs_apply_pauli_sum", "qs_grad_adjoint",
            "qs_stream_copy", "qs_plan", "qs_batch_create", "qs_batch_run",
            "qs_batch_destroy", "qs_apply_kq", "qs_permute_qubits", "qs_plan_reorder",
            "qs_run_reordered", "qs_set_grid_limit", "qs_probabilities_noalloc",
            "qs_set_fused_exec", "qs_precompile", "qs_get_jit_stats", "qs_get_verify")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1601_07195_amd.build`")

_L = ctypes.CDLL(LIB_PATH)
_vp, _i, _sz, _u64, _dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_void_p

_L.qs_version.restype = _i
_L.qs_strerror.argtypes = [_i]
_L.qs_strerror.restype = ctypes.c_char_p
_L.qs_last_error.restype = ctypes.c_char_p
_L.qs_create.argtypes = [_i, _i, _vp, _sz, _vp, ctypes.POINTER(_vp)]
_L.qs_destroy.argtypes = [_vp]
_L.qs_set_stream.argtypes = [_vp, _vp]
_L.qs_set_grid_limit.argtypes = [_vp, _i]
_L.qs_set_fused_exec.argtypes = [_vp, _i]
_L.qs_get_verify.argtypes = [_vp, _dp, _dp]
_L.qs_precompile.argtypes = [_i, _i, _vp, _i, _dp, _i, _i, _vp]


class QSJitStats(ctypes.Structure):
    _fields_ = [("kernels_compiled", ctypes.c_int64), ("kernels_cached", ctypes.c_int64),
                ("modules_loaded", ctypes.c_int64), ("compile_seconds", ctypes.c_double),
                ("kernels_from_disk", ctypes.c_int64), ("programs_clang", ctypes.c_int64),
                ("programs_hiprtc", ctypes.c_int64)]


_L.qs_get_jit_stats.argtypes = [ctypes.POINTER(QSJitStats)]
_L.qs_init_basis.argtypes = [_vp, _u64]
_L.qs_apply_1q.argtypes = [_vp, _i, _dp]
_L.qs_apply_cu.argtypes = [_vp, _i, _i, _dp]
_L.qs_apply_kq.argtypes = [_vp, _i, _vp, _dp]
_L.qs_run.argtypes = [_vp, _vp, _i, _dp, _i, _i]
_L.qs_probabilities.argtypes = [_vp, _dp, _dp, _vp, _sz]
_L.qs_probabilities_noalloc.argtypes = [_vp, _vp, _vp, _vp, _sz]
_L.qs_expect_pauli.argtypes = [_vp, _i, _vp, _vp, _dp, _dp]
_L.qs_apply_pauli_sum.argtypes = [_vp, _vp, _i, _vp, _vp, _dp]
_L.qs_grad_adjoint.argtypes = [_vp, _vp, _i, _dp, _i, _i, _vp, _vp, _dp, _vp, _i, _dp, _dp]
_L.qs_stream_copy.argtypes = [_vp, _vp, _sz, _vp]


class QSPlanInfo(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_int32), ("fused", ctypes.c_int32),
                ("single_1q", ctypes.c_int32), ("single_cu", ctypes.c_int32),
                ("remaps", ctypes.c_int32), ("fused_ops", ctypes.c_int32),
                ("hbm_bytes", ctypes.c_double)]


_L.qs_plan.argtypes = [_i, _i, _vp, _i, _dp, _i, _i, ctypes.POINTER(QSPlanInfo), _vp, _vp]


class QSReorderInfo(ctypes.Structure):
    _fields_ = [("remaps", ctypes.c_int32), ("swaps", ctypes.c_int32),
                ("restore_swaps", ctypes.c_int32), ("global_gates", ctypes.c_int32),
                ("traffic_reordered", ctypes.c_double), ("traffic_pairwise", ctypes.c_double)]


_L.qs_permute_qubits.argtypes = [_vp, _vp]
_L.qs_plan_reorder.argtypes = [_i, _i, _vp, _i, _dp, _i, ctypes.POINTER(QSReorderInfo), _vp, _vp,
                               _vp, _i, _vp]
_L.qs_run_reordered.argtypes = [_vp, _i, _vp, _i, _dp, _i, _i, ctypes.POINTER(QSReorderInfo)]


class QSBatchTuning(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("lds_bits", ctypes.c_int32),
                ("khigh", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("order", ctypes.c_int32)]


_L.qs_batch_create.argtypes = [_i, _i, _vp, _vp, _vp, _vp, _dp, _vp, _vp, _vp, _dp, _vp,
                               ctypes.POINTER(_vp)]
_L.qs_batch_run.argtypes = [_vp, ctypes.POINTER(QSBatchTuning), _dp, _dp]
_L.qs_batch_destroy.argtypes = [_vp]
for _name in EXPORTED:
    if _name not in ("qs_strerror", "qs_last_error"):
        getattr(_L, _name).restype = _i


class QSError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _L.qs_last_error().decode() or _L.qs_strerror(code).decode()
        super().__init__(f"{where}: {_L.qs_strerror(code).decode()} ({code}): {msg}")


def _check(rc: int, where: str) -> None:
    if rc != QS_OK:
        raise QSError(rc, where)


def lib() -> ctypes.CDLL:
    return _L


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _mat8(q) -> np.ndarray:
    q = np.asarray(q)
    if np.iscomplexobj(q) or q.shape == (2, 2):
        q = np.asarray(q, dtype=np.complex128).reshape(2, 2)
        q = np.stack([q.real, q.imag], axis=-1).reshape(8)
    q = _f64(q)
    if q.shape != (8,):
        raise ValueError("a gate is a 2x2 complex matrix or 8 doubles")
    return q


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


def _stream_handle(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def ops_array(ops) -> np.ndarray:
    """Gate records as a contiguous qs_op array (any 80-byte structured
    array with the same fields is accepted)."""
    a = np.ascontiguousarray(ops)
    if a.dtype.itemsize != QS_OP_DTYPE.itemsize or a.dtype.names != QS_OP_DTYPE.names:
        raise ValueError("ops must be qs_op records")
    return a.view(QS_OP_DTYPE)


def pauli_masks(codes: np.ndarray):
    """Pauli strings (nterms, n) with codes 0 = I, 1 = X, 2 = Y, 3 = Z ->
    (x, z) uint64 bit masks as the C ABI takes them."""
    codes = np.asarray(codes, dtype=np.uint8)
    if codes.ndim != 2:
        raise ValueError("codes must be (nterms, n)")
    n = codes.shape[1]
    w = (np.uint64(1) << np.arange(n, dtype=np.uint64))
    x = (((codes == 1) | (codes == 2)).astype(np.uint64) * w).sum(axis=1, dtype=np.uint64)
    z = (((codes == 3) | (codes == 2)).astype(np.uint64) * w).sum(axis=1, dtype=np.uint64)
    return np.ascontiguousarray(x, dtype=np.uint64), np.ascontiguousarray(z, dtype=np.uint64)


# ------------------------------------------------------ C-named functions

def qs_version() -> int:
    return _L.qs_version()


def qs_strerror(code: int) -> str:
    return _L.qs_strerror(code).decode()


def qs_last_error() -> str:
    return _L.qs_last_error().decode()


def qs_create(n: int, dtype: int, dev_ptr: int, nbytes: int, stream: int | None) -> int:
    h = _vp()
    _check(_L.qs_create(n, dtype, dev_ptr, nbytes, stream, ctypes.byref(h)), "qs_create")
    return h.value


def qs_destroy(h: int) -> None:
    _check(_L.qs_destroy(h), "qs_destroy")


def qs_set_stream(h: int, stream: int | None) -> None:
    _check(_L.qs_set_stream(h, stream), "qs_set_stream")


def qs_set_grid_limit(h: int, max_workgroups: int) -> None:
    _check(_L.qs_set_grid_limit(h, max_workgroups), "qs_set_grid_limit")


def qs_init_basis(h: int, index: int = 0) -> None:
    _check(_L.qs_init_basis(h, index), "qs_init_basis")


def qs_apply_1q(h: int, k: int, q) -> None:
    m = _mat8(q)
    _check(_L.qs_apply_1q(h, k, _ptr(m)), "qs_apply_1q")


def qs_apply_cu(h: int, c: int, t: int, q) -> None:
    m = _mat8(q)
    _check(_L.qs_apply_cu(h, c, t, _ptr(m)), "qs_apply_cu")


def qs_apply_kq(h: int, targets, u) -> None:
    """Dense 2^k x 2^k gate u on `targets` (bit j of u's index is qubit
    targets[j])."""
    t = np.ascontiguousarray(targets, dtype=np.int32)
    m = np.ascontiguousarray(np.asarray(u, dtype=np.complex128))
    k = len(t)
    if m.shape != (1 << k, 1 << k):
        raise ValueError("u must be 2^k x 2^k for k targets")
    flat = m.view(np.float64).copy()
    _check(_L.qs_apply_kq(h, k, _ptr(t), _ptr(flat)), "qs_apply_kq")


def qs_run(h: int, ops, theta=None, flags: int = 0) -> None:
    a = ops_array(ops)
    th = _f64(theta) if theta is not None else None
    _check(_L.qs_run(h, _ptr(a), len(a), _ptr(th), 0 if th is None else len(th), flags), "qs_run")


def qs_probabilities(h: int, n: int, full_tensor: torch.Tensor | None = None, want_p1: bool = True):
    p1 = np.zeros(n, dtype=np.float64) if want_p1 else None
    nrm = np.zeros(1, dtype=np.float64)
    fptr, fbytes = None, 0
    if full_tensor is not None:
        if full_tensor.dtype != torch.float64 or not full_tensor.is_contiguous():
            raise ValueError("full probabilities go to a contiguous float64 device tensor")
        fptr, fbytes = full_tensor.data_ptr(), full_tensor.numel() * 8
    _check(_L.qs_probabilities(h, _ptr(p1), _ptr(nrm), fptr, fbytes), "qs_probabilities")
    return p1, float(nrm[0])


def qs_probabilities_noalloc(h: int, p1: torch.Tensor | None, norm2: torch.Tensor | None,
                             full: torch.Tensor | None = None) -> None:
    """Allocation-free probabilities into float64 GPU tensors (asynchronous)."""
    def dev(t):
        if t is None:
            return None
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("outputs must be contiguous float64 GPU tensors")
        return t.data_ptr()
    fb = 0 if full is None else full.numel() * 8
    _check(_L.qs_probabilities_noalloc(h, dev(p1), dev(norm2), dev(full), fb),
           "qs_probabilities_noalloc")


def qs_expect_pauli(h: int, x, z, coeff) -> float:
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    c = _f64(coeff)
    out = np.zeros(1, dtype=np.float64)
    _check(_L.qs_expect_pauli(h, len(c), _ptr(x), _ptr(z), _ptr(c), _ptr(out)), "qs_expect_pauli")
    return float(out[0])


def qs_apply_pauli_sum(src: int, dst: int, x, z, coeff) -> None:
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    c = _f64(coeff)
    _check(_L.qs_apply_pauli_sum(src, dst, len(c), _ptr(x), _ptr(z), _ptr(c)), "qs_apply_pauli_sum")


def qs_grad_adjoint(h: int, ops, theta, x, z, coeff, lam: int, flags: int = 0):
    a = ops_array(ops)
    th = _f64(theta)
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    c = _f64(coeff)
    e = np.zeros(1, dtype=np.float64)
    g = np.zeros(len(th), dtype=np.float64)
    _check(_L.qs_grad_adjoint(h, _ptr(a), len(a), _ptr(th), len(th), len(c), _ptr(x), _ptr(z),
                              _ptr(c), lam, flags, _ptr(e), _ptr(g)), "qs_grad_adjoint")
    return float(e[0]), g


def qs_plan(n: int, dtype: int, ops, theta=None, flags: int = 0):
    """Host-only planning: returns (info dict, order, pass_of)."""
    a = ops_array(ops)
    th = _f64(theta) if theta is not None else None
    info = QSPlanInfo()
    order = np.zeros(len(a), dtype=np.int32)
    pass_of = np.zeros(len(a), dtype=np.int32)
    _check(_L.qs_plan(n, dtype, _ptr(a), len(a), _ptr(th), 0 if th is None else len(th), flags,
                      ctypes.byref(info), _ptr(order), _ptr(pass_of)), "qs_plan")
    d = {f: getattr(info, f) for f, _ in QSPlanInfo._fields_}
    return d, order, pass_of


def qs_get_verify(h: int):
    """(max |fused - per-gate|, norm^2 drift) of the state's last verified run."""
    d = np.zeros(2, dtype=np.float64)
    _check(_L.qs_get_verify(h, _ptr(d[:1]), _ptr(d[1:])), "qs_get_verify")
    return float(d[0]), float(d[1])


def qs_set_fused_exec(h: int, mode: int) -> None:
    _check(_L.qs_set_fused_exec(h, mode), "qs_set_fused_exec")


def qs_precompile(n: int, dtype: int, ops, theta=None, flags: int = 0) -> int:
    """Host-only: compile the pass kernels a run of `ops` needs; returns their count."""
    a = ops_array(ops)
    th = _f64(theta) if theta is not None else None
    nk = np.zeros(1, dtype=np.int32)
    _check(_L.qs_precompile(n, dtype, _ptr(a), len(a), _ptr(th), 0 if th is None else len(th), flags,
                            _ptr(nk)), "qs_precompile")
    return int(nk[0])


def qs_get_jit_stats() -> dict:
    st = QSJitStats()
    _check(_L.qs_get_jit_stats(ctypes.byref(st)), "qs_get_jit_stats")
    return {f: getattr(st, f) for f, _ in QSJitStats._fields_}


def qs_permute_qubits(h: int, perm) -> None:
    """Relabel qubit q as perm[q] in place (state reordering, Sec. 6)."""
    p = np.ascontiguousarray(perm, dtype=np.int32)
    _check(_L.qs_permute_qubits(h, _ptr(p)), "qs_permute_qubits")


def _reorder_dict(info):
    return {f: getattr(info, f) for f, _ in QSReorderInfo._fields_}


def qs_plan_reorder(n: int, nlocal: int, ops, theta=None):
    """Host-only reordering plan for a state split by its top n - nlocal
    qubits: returns (info dict, ops on positions, remap_at, remap_perm
    [R x n], final_perm)."""
    a = ops_array(ops)
    th = _f64(theta) if theta is not None else None
    nth = 0 if th is None else len(th)
    info = QSReorderInfo()
    _check(_L.qs_plan_reorder(n, nlocal, _ptr(a), len(a), _ptr(th), nth, ctypes.byref(info),
                              None, None, None, 0, None), "qs_plan_reorder")
    R = info.remaps
    out = np.zeros(len(a), dtype=QS_OP_DTYPE)
    at = np.zeros(max(R, 1), dtype=np.int32)
    perm = np.zeros((max(R, 1), n), dtype=np.int32)
    fin = np.zeros(n, dtype=np.int32)
    _check(_L.qs_plan_reorder(n, nlocal, _ptr(a), len(a), _ptr(th), nth, ctypes.byref(info),
                              _ptr(out), _ptr(at), _ptr(perm), R, _ptr(fin)), "qs_plan_reorder")
    return _reorder_dict(info), out, at[:R].copy(), perm[:R].copy(), fin


def qs_run_reordered(h: int, nlocal: int, ops, theta=None, flags: int = 0):
    a = ops_array(ops)
    th = _f64(theta) if theta is not None else None
    info = QSReorderInfo()
    _check(_L.qs_run_reordered(h, nlocal, _ptr(a), len(a), _ptr(th), 0 if th is None else len(th),
                               flags, ctypes.byref(info)), "qs_run_reordered")
    return _reorder_dict(info)


def qs_stream_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst smaller than src")
    _check(_L.qs_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, _stream_handle(stream)),
           "qs_stream_copy")


def qs_batch_create(dtype: int, n, op_off, ops, par_off, theta, term_off, x, z, coeff,
                    stream=None) -> int:
    """Arrays as the C ABI takes them (offsets int64 of ncircuits + 1)."""
    n = np.ascontiguousarray(n, dtype=np.int32)
    op_off = np.ascontiguousarray(op_off, dtype=np.int64)
    par_off = np.ascontiguousarray(par_off, dtype=np.int64)
    term_off = np.ascontiguousarray(term_off, dtype=np.int64)
    a = ops_array(ops) if len(ops) else np.zeros(0, dtype=QS_OP_DTYPE)
    th = _f64(theta)
    x = np.ascontiguousarray(x, dtype=np.uint64)
    z = np.ascontiguousarray(z, dtype=np.uint64)
    c = _f64(coeff)
    if not (len(op_off) == len(par_off) == len(term_off) == len(n) + 1):
        raise ValueError("offset arrays need ncircuits + 1 entries")
    h = _vp()
    _check(_L.qs_batch_create(dtype, len(n), _ptr(n), _ptr(op_off), _ptr(a), _ptr(par_off),
                              _ptr(th), _ptr(term_off), _ptr(x), _ptr(z), _ptr(c),
                              _stream_handle(stream), ctypes.byref(h)), "qs_batch_create")
    return h.value


def _tuning(t) -> QSBatchTuning | None:
    if t is None:
        return None
    if isinstance(t, QSBatchTuning):
        return t
    return QSBatchTuning(**{k: int(v) for k, v in dict(t).items() if not k.startswith("_")})


def qs_batch_run(h: int, ncircuits: int, nparams: int, tuning=None):
    """Returns (energy[ncircuits], grad[nparams]) as float64 arrays; tuning
    is None, a QSBatchTuning or a dict of its fields."""
    e = np.zeros(ncircuits, dtype=np.float64)
    g = np.zeros(nparams, dtype=np.float64)
    t = _tuning(tuning)
    _check(_L.qs_batch_run(h, None if t is None else ctypes.byref(t), _ptr(e), _ptr(g)),
           "qs_batch_run")
    return e, g


def qs_batch_destroy(h: int) -> None:
    _check(_L.qs_batch_destroy(h), "qs_batch_destroy")


# ------------------------------------------------------------ conveniences

_TORCH_DTYPE = {QS_C128: torch.complex128, QS_C64: torch.complex64}


class State:
    """An n-qubit state in a torch tensor on the current GPU, bound to a
    libqs handle.  Work is queued on `stream` (default: torch's current
    stream at construction)."""

    def __init__(self, n: int, dtype: int = QS_C128, device: str | torch.device = "cuda",
                 stream=None, tensor: torch.Tensor | None = None, init: bool = True):
        self.n = n
        self.dtype = dtype
        if tensor is None:
            tensor = torch.empty(1 << n, dtype=_TORCH_DTYPE[dtype], device=device)
        if tensor.dtype != _TORCH_DTYPE[dtype] or not tensor.is_contiguous() or not tensor.is_cuda:
            raise ValueError("state tensor must be a contiguous GPU tensor of the state dtype")
        self.tensor = tensor
        self.stream = stream if stream is not None else torch.cuda.current_stream(tensor.device)
        self.handle = qs_create(n, dtype, tensor.data_ptr(), tensor.numel() * tensor.element_size(),
                                self.stream.cuda_stream)
        if init:
            qs_init_basis(self.handle, 0)

    def close(self) -> None:
        if getattr(self, "handle", None):
            qs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_grid_limit(self, max_workgroups: int) -> "State":
        qs_set_grid_limit(self.handle, max_workgroups)
        return self

    def set_fused_exec(self, mode: int) -> "State":
        qs_set_fused_exec(self.handle, mode)
        return self

    def init_basis(self, index: int = 0) -> "State":
        qs_init_basis(self.handle, index)
        return self

    def apply_1q(self, k: int, q) -> "State":
        qs_apply_1q(self.handle, k, q)
        return self

    def apply_cu(self, c: int, t: int, q) -> "State":
        qs_apply_cu(self.handle, c, t, q)
        return self

    def apply_kq(self, targets, u) -> "State":
        qs_apply_kq(self.handle, targets, u)
        return self

    def run(self, ops, theta=None, fuse: bool = True, wide: bool = False, verify: bool = False) -> "State":
        qs_run(self.handle, ops, theta, (0 if fuse else QS_RUN_NO_FUSION) | (QS_RUN_WIDE_TILES if wide else 0)
               | (QS_RUN_VERIFY if verify else 0))
        return self

    def permute_qubits(self, perm) -> "State":
        qs_permute_qubits(self.handle, perm)
        return self

    def run_reordered(self, ops, nlocal: int, theta=None, fuse: bool = True) -> dict:
        return qs_run_reordered(self.handle, nlocal, ops, theta, 0 if fuse else QS_RUN_NO_FUSION)

    def probabilities(self, full: bool = False):
        ft = torch.empty(1 << self.n, dtype=torch.float64, device=self.tensor.device) if full else None
        p1, nrm = qs_probabilities(self.handle, self.n, ft)
        return p1, nrm, ft

    def expect(self, codes, coeff) -> float:
        x, z = pauli_masks(codes)
        return qs_expect_pauli(self.handle, x, z, coeff)

    def numpy(self) -> np.ndarray:
        self.stream.synchronize()
        return self.tensor.detach().cpu().numpy().astype(np.complex128)


def grad_adjoint(state: State, lam: State, ops, theta, codes, coeff, state_is_final: bool = False,
                 wide: bool = False):
    """Energy and adjoint gradient; see qs_grad_adjoint."""
    x, z = pauli_masks(codes)
    flags = (QS_ADJ_STATE_IS_FINAL if state_is_final else 0) | (QS_ADJ_WIDE_TILES if wide else 0)
    return qs_grad_adjoint(state.handle, ops, theta, x, z, coeff, lam.handle, flags)


class AdjointEnergy(torch.autograd.Function):
    """E(theta) = <0|U(theta)^dagger H U(theta)|0> with d E / d theta from
    one adjoint reverse sweep.

    forward(theta, ops, n, codes, coeff, dtype) runs the circuit (qs_run) and
    the expectation (qs_expect_pauli); backward runs qs_grad_adjoint on the
    state the forward left behind, so the forward sweep is not repeated.
    theta is a float64 CPU or GPU tensor; E is returned as a 0-d float64
    tensor on theta's device."""

    @staticmethod
    def forward(ctx, theta, ops, n, codes, coeff, dtype=QS_C128):
        th = theta.detach().to("cpu", torch.float64).numpy()
        st = State(n, dtype)
        st.run(ops, th)
        x, z = pauli_masks(codes)
        e = qs_expect_pauli(st.handle, x, z, coeff)
        ctx.saved = (st, ops, th, codes, coeff, dtype, n)
        return torch.tensor(e, dtype=torch.float64, device=theta.device)

    @staticmethod
    def backward(ctx, grad_out):
        st, ops, th, codes, coeff, dtype, n = ctx.saved
        lam = State(n, dtype, init=False)
        _, g = grad_adjoint(st, lam, ops, th, codes, coeff, state_is_final=True)
        ctx.saved = None
        gt = torch.from_numpy(g).to(grad_out.device) * grad_out
        return gt, None, None, None, None, None


class Batch:
    """Many independent circuits, each with its own parameters and Pauli-sum
    observable, run as one persistent launch (qs_batch_*).

    circuits: sequence of (n, ops, theta, codes, coeff); codes (nterms, n)
    with 0 = I, 1 = X, 2 = Y, 3 = Z.  run() returns (energy[c], [grad_c])."""

    def __init__(self, circuits, dtype: int = QS_C128, stream=None):
        circuits = list(circuits)
        self.dtype = dtype
        self.ncircuits = len(circuits)
        n = np.array([c[0] for c in circuits], dtype=np.int32)
        ops = [ops_array(c[1]) for c in circuits]
        theta = [_f64(c[2]) for c in circuits]
        masks = [pauli_masks(c[3]) for c in circuits]
        coeff = [_f64(c[4]) for c in circuits]

        def offsets(parts):
            o = np.zeros(len(parts) + 1, dtype=np.int64)
            o[1:] = np.cumsum([len(p) for p in parts])
            return o

        self.n = n
        self.op_off, self.par_off, self.term_off = offsets(ops), offsets(theta), offsets(coeff)
        cat = lambda parts, dt: np.concatenate(parts) if parts else np.zeros(0, dtype=dt)
        self.handle = qs_batch_create(
            dtype, n, self.op_off, cat(ops, QS_OP_DTYPE), self.par_off, cat(theta, np.float64),
            self.term_off, cat([m[0] for m in masks], np.uint64),
            cat([m[1] for m in masks], np.uint64), cat(coeff, np.float64), stream)

    def run_flat(self, tuning=None):
        """(energy[ncircuits], concatenated gradient) from one launch."""
        return qs_batch_run(self.handle, self.ncircuits, int(self.par_off[-1]), tuning)

    def run(self, tuning=None):
        e, g = self.run_flat(tuning)
        return e, [g[self.par_off[c]:self.par_off[c + 1]] for c in range(self.ncircuits)]

    def close(self) -> None:
        if getattr(self, "handle", None):
            qs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
