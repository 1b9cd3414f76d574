// qs_api.cpp -- the C ABI of libqs: argument validation, state handles,
// small-buffer management and dispatch to the kernel launchers.
//
// Every entry point validates all of its arguments on the host before the
// first HIP call, so a rejected call queues nothing.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <cmath>
#include <string.h>

#include <new>
#include <string>

#include "qs_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int done(const qs::Status& s) {
  if (s.good()) return QS_OK;
  return fail(s.code, s.msg);
}

int max_qubits(int dtype) { return dtype == QS_C128 ? QS_MAX_QUBITS_C128 : QS_MAX_QUBITS_C64; }

bool valid_state(const qs_state* s) { return s && s->impl.ptr && s->impl.n > 0; }

}  // namespace

namespace qs {

Status ensure_dev(StateImpl* s, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes) return Status::ok();
  if (b.ptr) {
    // Earlier queued kernels may still read the old buffer.
    Status st = hip_status(hipStreamSynchronize(s->stream), "sync before regrow");
    if (!st.good()) return st;
    (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
  }
  size_t want = 4096;
  while (want < bytes) want <<= 1;
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    Status st;
    st.code = QS_ENOMEM;
    st.msg = "device scratch allocation of " + std::to_string(want) + " bytes failed";
    return st;
  }
  b.ptr = p;
  b.bytes = want;
  return Status::ok();
}

Status ensure_result_host(StateImpl* s, size_t bytes) {
  if (s->result_bytes >= bytes) return Status::ok();
  if (s->result_host) (void)hipHostFree(s->result_host);
  s->result_host = nullptr;
  s->result_bytes = 0;
  size_t want = 4096;
  while (want < bytes) want <<= 1;
  void* p = nullptr;
  if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    Status st;
    st.code = QS_ENOMEM;
    st.msg = "pinned host allocation failed";
    return st;
  }
  s->result_host = (double*)p;
  s->result_bytes = want;
  return Status::ok();
}

Status upload_table(StateImpl* s, const void* src, size_t bytes) {
  if (bytes == 0) bytes = 16;
  Status st;
  if (s->stage.pending) {
    st = hip_status(hipEventSynchronize(s->stage.done), "staging wait");
    if (!st.good()) return st;
    s->stage.pending = false;
  }
  if (s->stage.bytes < bytes) {
    if (s->stage.host) (void)hipHostFree(s->stage.host);
    s->stage.host = nullptr;
    s->stage.bytes = 0;
    size_t want = 4096;
    while (want < bytes) want <<= 1;
    if (hipHostMalloc(&s->stage.host, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      st.code = QS_ENOMEM;
      st.msg = "pinned staging allocation failed";
      return st;
    }
    s->stage.bytes = want;
  }
  if (!s->stage.done) {
    st = hip_status(hipEventCreateWithFlags(&s->stage.done, hipEventDisableTiming), "event");
    if (!st.good()) return st;
  }
  st = ensure_dev(s, s->table, bytes);
  if (!st.good()) return st;
  if (src) memcpy(s->stage.host, src, bytes);
  st = hip_status(hipMemcpyAsync(s->table.ptr, s->stage.host, bytes, hipMemcpyHostToDevice,
                                 s->stream), "table upload");
  if (!st.good()) return st;
  st = hip_status(hipEventRecord(s->stage.done, s->stream), "event record");
  if (!st.good()) return st;
  s->stage.pending = true;
  return Status::ok();
}

// Matrix of a rotation R_P(theta) = exp(-i theta P / 2), 8-double layout.
static void rotation(int kind, double theta, double* m) {
  const double c = cos(0.5 * theta), sn = sin(0.5 * theta);
  for (int e = 0; e < 8; ++e) m[e] = 0.0;
  if (kind == QS_OP_RX) {  // [[c, -i s], [-i s, c]]
    m[0] = c; m[3] = -sn; m[5] = -sn; m[6] = c;
  } else if (kind == QS_OP_RY) {  // [[c, -s], [s, c]]
    m[0] = c; m[2] = -sn; m[4] = sn; m[6] = c;
  } else {  // RZ: diag(e^{-i theta/2}, e^{i theta/2})
    m[0] = c; m[1] = -sn; m[6] = c; m[7] = sn;
  }
}

Status normalize_ops(int n, const qs_op* ops, int nops, const double* theta, int nparams,
                     std::vector<XGate>* out) {
  out->clear();
  out->reserve(nops);
  Status bad;
  bad.code = QS_EINVAL;
  for (int g = 0; g < nops; ++g) {
    const qs_op& op = ops[g];
    XGate x;
    x.kind = op.kind;
    x.target = op.target;
    x.control = -1;
    x.param = -1;
    if (op.target < 0 || op.target >= n) {
      bad.msg = "op " + std::to_string(g) + ": target " + std::to_string(op.target) + " out of range";
      return bad;
    }
    switch (op.kind) {
      case QS_OP_U:
        memcpy(x.m, op.mat, sizeof(x.m));
        break;
      case QS_OP_CU:
        if (op.control < 0 || op.control >= n || op.control == op.target) {
          bad.msg = "op " + std::to_string(g) + ": bad control " + std::to_string(op.control);
          return bad;
        }
        x.control = op.control;
        memcpy(x.m, op.mat, sizeof(x.m));
        break;
      case QS_OP_RX:
      case QS_OP_RY:
      case QS_OP_RZ:
        if (!theta || op.param < 0 || op.param >= nparams) {
          bad.msg = "op " + std::to_string(g) + ": parameter index " + std::to_string(op.param) +
                    " out of range";
          return bad;
        }
        x.param = op.param;
        rotation(op.kind, theta[op.param], x.m);
        break;
      default:
        bad.msg = "op " + std::to_string(g) + ": unknown kind " + std::to_string(op.kind);
        return bad;
    }
    out->push_back(x);
  }
  return Status::ok();
}

}  // namespace qs

using qs::Status;

extern "C" {

int qs_version(void) { return 10000; }

const char* qs_strerror(int code) {
  switch (code) {
    case QS_OK: return "success";
    case QS_EINVAL: return "invalid argument";
    case QS_ENOMEM: return "out of memory";
    case QS_EHIP: return "HIP runtime error";
    case QS_ENODEV: return "no usable GPU device";
    case QS_ERANGE: return "size out of range";
    case QS_EVERIFY: return "verification failed";
    default: return "unknown status";
  }
}

const char* qs_last_error(void) { return g_last_error.c_str(); }

// The device must be a gfx950 (the only target the kernels are built for).
static int check_device(int dev, const char* who) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QS_ENODEV, std::string(who) + ": cannot query device " + std::to_string(dev));
  }
  if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(QS_ENODEV, std::string(who) + ": device " + std::to_string(dev) + " is " +
                               prop.gcnArchName + ", not gfx950");
  return QS_OK;
}

// `ptr` must be device (or managed) memory of device `dev` with at least
// `need` bytes from ptr to the end of its allocation.  A host pointer would
// otherwise pass validation and fault on the first kernel.
static int check_device_buffer(const void* ptr, size_t need, int dev, const std::string& what) {
  hipPointerAttribute_t at;
  memset(&at, 0, sizeof(at));
  if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QS_EINVAL, what + " is not device memory");
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
    return fail(QS_EINVAL, what + " is not device memory");
  if (at.device != dev)
    return fail(QS_EINVAL, what + " belongs to device " + std::to_string(at.device) +
                               ", not the current device " + std::to_string(dev));
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)ptr) == hipSuccess && base && size) {
    const size_t avail = size - (size_t)((const char*)ptr - (const char*)base);
    if (avail < need)
      return fail(QS_ERANGE, what + ": the allocation holds " + std::to_string(avail) +
                                 " bytes from the pointer, fewer than " + std::to_string(need));
  } else {
    (void)hipGetLastError();
  }
  return QS_OK;
}

int qs_create(int n, int dtype, void* dev_ptr, size_t bytes, void* stream, qs_state** out) {
  if (!out) return fail(QS_EINVAL, "qs_create: out is NULL");
  *out = nullptr;
  if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_EINVAL, "qs_create: bad dtype");
  if (n < 1 || n > max_qubits(dtype))
    return fail(QS_ERANGE, "qs_create: n=" + std::to_string(n) + " outside 1.." +
                               std::to_string(max_qubits(dtype)));
  if (!dev_ptr) return fail(QS_EINVAL, "qs_create: dev_ptr is NULL");
  if (((uintptr_t)dev_ptr) & 255) return fail(QS_EINVAL, "qs_create: dev_ptr not 256-byte aligned");
  const size_t need = ((size_t)1 << n) * qs::amp_bytes(dtype);
  if (bytes < need)
    return fail(QS_ERANGE, "qs_create: buffer of " + std::to_string(bytes) + " bytes < " +
                               std::to_string(need));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QS_ENODEV, "qs_create: no HIP device");
  }
  {
    int rc = check_device(dev, "qs_create");
    if (rc) return rc;
    rc = check_device_buffer(dev_ptr, need, dev, "qs_create: dev_ptr");
    if (rc) return rc;
  }
  qs_state* s = new (std::nothrow) qs_state();
  if (!s) return fail(QS_ENOMEM, "qs_create: handle allocation failed");
  s->impl.n = n;
  s->impl.dtype = dtype;
  s->impl.ptr = dev_ptr;
  s->impl.bytes = bytes;
  s->impl.stream = (hipStream_t)stream;
  s->impl.device = dev;
  *out = s;
  return QS_OK;
}

int qs_destroy(qs_state* s) {
  if (!s) return QS_OK;
  qs::StateImpl& m = s->impl;
  int rc = QS_OK;
  if (hipStreamSynchronize(m.stream) != hipSuccess) {
    (void)hipGetLastError();
    rc = fail(QS_EHIP, "qs_destroy: stream synchronisation failed");
  }
  if (m.red.ptr) (void)hipFree(m.red.ptr);
  if (m.scal.ptr) (void)hipFree(m.scal.ptr);
  if (m.table.ptr) (void)hipFree(m.table.ptr);
  if (m.stage.host) (void)hipHostFree(m.stage.host);
  if (m.stage.done) (void)hipEventDestroy(m.stage.done);
  if (m.result_host) (void)hipHostFree(m.result_host);
  delete s;
  return rc;
}

int qs_set_stream(qs_state* s, void* stream) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_set_stream: bad state");
  // Work queued on the old stream must finish before the new stream reuses
  // the handle's scratch buffers.
  Status st = qs::hip_status(hipStreamSynchronize(s->impl.stream), "qs_set_stream sync");
  if (!st.good()) return done(st);
  s->impl.stream = (hipStream_t)stream;
  return QS_OK;
}

int qs_set_grid_limit(qs_state* s, int max_workgroups) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_set_grid_limit: bad state");
  if (max_workgroups < 0) return fail(QS_EINVAL, "qs_set_grid_limit: negative limit");
  s->impl.grid_limit = max_workgroups;
  return QS_OK;
}

int qs_set_fused_exec(qs_state* s, int mode) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_set_fused_exec: bad state");
  if (mode != QS_EXEC_AUTO && mode != QS_EXEC_INTERPRETED && mode != QS_EXEC_COMPILED)
    return fail(QS_EINVAL, "qs_set_fused_exec: unknown mode");
  s->impl.exec = mode;
  return QS_OK;
}

int qs_precompile(int n, int dtype, const qs_op* ops, int nops, const double* theta, int nparams,
                  int flags, int32_t* nkernels) {
  if (nkernels) *nkernels = 0;
  if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_EINVAL, "qs_precompile: bad dtype");
  if (n < 1 || n > max_qubits(dtype)) return fail(QS_ERANGE, "qs_precompile: n out of range");
  if (nops < 0 || (nops > 0 && !ops)) return fail(QS_EINVAL, "qs_precompile: bad op list");
  if (nparams < 0) return fail(QS_EINVAL, "qs_precompile: nparams < 0");
  if (flags & ~(QS_PRECOMPILE_ADJOINT | QS_RUN_WIDE_TILES)) return fail(QS_EINVAL, "qs_precompile: unknown flags");
  std::vector<qs::XGate> gates;
  Status st = qs::normalize_ops(n, ops, nops, theta, nparams, &gates);
  if (!st.good()) return done(st);
  int nk = 0;
  st = qs::precompile_passes(n, dtype, gates, (flags & QS_PRECOMPILE_ADJOINT) != 0,
                             (flags & QS_RUN_WIDE_TILES) != 0, &nk);
  if (!st.good()) return done(st);
  if (nkernels) *nkernels = nk;
  return QS_OK;
}

int qs_get_jit_stats(qs_jit_stats* out) {
  if (!out) return fail(QS_EINVAL, "qs_get_jit_stats: out is NULL");
  const qs::JitStats j = qs::jit_stats();
  out->kernels_compiled = j.kernels;
  out->kernels_cached = j.cached;
  out->modules_loaded = j.modules_loaded;
  out->compile_seconds = j.compile_seconds;
  out->kernels_from_disk = j.loaded_from_disk;
  out->programs_clang = j.programs_clang;
  out->programs_hiprtc = j.programs_hiprtc;
  return QS_OK;
}

int qs_init_basis(qs_state* s, uint64_t index) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_init_basis: bad state");
  if (index >= (1ull << s->impl.n)) return fail(QS_EINVAL, "qs_init_basis: index >= 2^n");
  return done(qs::launch_init_basis(&s->impl, index));
}

int qs_apply_1q(qs_state* s, int k, const double* q) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_apply_1q: bad state");
  if (!q) return fail(QS_EINVAL, "qs_apply_1q: q is NULL");
  if (k < 0 || k >= s->impl.n) return fail(QS_EINVAL, "qs_apply_1q: target out of range");
  return done(qs::launch_apply_1q(&s->impl, k, q));
}

int qs_apply_cu(qs_state* s, int c, int t, const double* q) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_apply_cu: bad state");
  if (!q) return fail(QS_EINVAL, "qs_apply_cu: q is NULL");
  const int n = s->impl.n;
  if (c < 0 || c >= n || t < 0 || t >= n) return fail(QS_EINVAL, "qs_apply_cu: qubit out of range");
  if (c == t) return fail(QS_EINVAL, "qs_apply_cu: control equals target");
  return done(qs::launch_apply_cu(&s->impl, c, t, q));
}

int qs_apply_kq(qs_state* s, int k, const int32_t* targets, const double* u) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_apply_kq: bad state");
  if (!targets || !u) return fail(QS_EINVAL, "qs_apply_kq: targets or u is NULL");
  const int n = s->impl.n;
  if (k < 1 || k > QS_KQ_MAX || k > n) return fail(QS_EINVAL, "qs_apply_kq: k out of range");
  uint64_t seen = 0;
  for (int j = 0; j < k; ++j) {
    if (targets[j] < 0 || targets[j] >= n) return fail(QS_EINVAL, "qs_apply_kq: target out of range");
    if ((seen >> targets[j]) & 1) return fail(QS_EINVAL, "qs_apply_kq: repeated target");
    seen |= 1ull << targets[j];
  }
  return done(qs::launch_apply_kq(&s->impl, k, targets, u));
}

int qs_permute_qubits(qs_state* s, const int32_t* perm) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_permute_qubits: bad state");
  if (!perm) return fail(QS_EINVAL, "qs_permute_qubits: perm is NULL");
  const int n = s->impl.n;
  uint64_t seen = 0;
  for (int q = 0; q < n; ++q) {
    if (perm[q] < 0 || perm[q] >= n) return fail(QS_EINVAL, "qs_permute_qubits: entry out of range");
    if ((seen >> perm[q]) & 1) return fail(QS_EINVAL, "qs_permute_qubits: not a permutation");
    seen |= 1ull << perm[q];
  }
  return done(qs::launch_permute(&s->impl, perm));
}

// QS_RUN_VERIFY: the list runs as asked on the state and, on a scratch copy
// of the input, as one streaming kernel per gate; the two results and the
// norm before and after are compared.
static Status run_verified(qs::StateImpl* s, const std::vector<qs::XGate>& gates, int flags) {
  using qs::Status;
  double norm0 = 0.0, norm1 = 0.0;
  Status st = qs::launch_probabilities(s, nullptr, &norm0, nullptr);
  if (!st.good()) return st;
  const size_t bytes = ((size_t)1 << s->n) * qs::amp_bytes(s->dtype);
  void* copy = nullptr;
  st = qs::hip_status(hipMalloc(&copy, bytes), "verify: scratch state");
  if (!st.good()) return st;
  qs::StateImpl twin;
  twin.n = s->n;
  twin.dtype = s->dtype;
  twin.ptr = copy;
  twin.bytes = bytes;
  twin.stream = s->stream;
  twin.device = s->device;
  twin.exec = QS_EXEC_INTERPRETED;
  st = qs::hip_status(hipMemcpyAsync(copy, s->ptr, bytes, hipMemcpyDeviceToDevice, s->stream), "verify: copy");
  if (st.good()) st = qs::run_gates(s, gates, flags);
  if (st.good()) st = qs::run_gates(&twin, gates, QS_RUN_NO_FUSION);
  double diff = 0.0;
  if (st.good()) st = qs::max_abs_diff(s, copy, &diff);
  if (st.good()) st = qs::launch_probabilities(s, nullptr, &norm1, nullptr);
  (void)hipStreamSynchronize(s->stream);
  (void)hipFree(copy);
  if (twin.red.ptr) (void)hipFree(twin.red.ptr);
  if (twin.scal.ptr) (void)hipFree(twin.scal.ptr);
  if (twin.table.ptr) (void)hipFree(twin.table.ptr);
  if (twin.stage.host) (void)hipHostFree(twin.stage.host);
  if (twin.stage.done) (void)hipEventDestroy(twin.stage.done);
  if (twin.result_host) (void)hipHostFree(twin.result_host);
  if (!st.good()) return st;
  const double drift = std::fabs(norm1 - norm0);
  s->verify_diff = diff;
  s->verify_drift = drift;
  // rounding of a unitary gate list: about one unit in the last place of
  // the amplitude type per gate on the way, grown like sqrt(gates)
  const double eps = s->dtype == QS_C128 ? 1.1e-16 : 6e-8;
  const double tol = 64.0 * eps * std::sqrt((double)gates.size() + 1.0) * std::max(1.0, std::sqrt(norm0));
  if (diff > tol || drift > tol * std::max(1.0, norm0)) {
    Status bad;
    bad.code = QS_EVERIFY;
    bad.msg = "qs_run verify: fused and per-gate results differ by " + std::to_string(diff) +
              ", norm^2 drifted by " + std::to_string(drift) + " (tolerance " + std::to_string(tol) +
              "); a non-unitary gate also fails this check";
    return bad;
  }
  return Status::ok();
}

int qs_run(qs_state* s, const qs_op* ops, int nops, const double* theta, int nparams, int flags) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_run: bad state");
  if (nops < 0 || (nops > 0 && !ops)) return fail(QS_EINVAL, "qs_run: bad op list");
  if (nparams < 0) return fail(QS_EINVAL, "qs_run: nparams < 0");
  if (flags & ~(QS_RUN_NO_FUSION | QS_RUN_WIDE_TILES | QS_RUN_VERIFY))
    return fail(QS_EINVAL, "qs_run: unknown flags");
  std::vector<qs::XGate> gates;
  Status st = qs::normalize_ops(s->impl.n, ops, nops, theta, nparams, &gates);
  if (!st.good()) return done(st);
  if (!(flags & QS_RUN_VERIFY)) return done(qs::run_gates(&s->impl, gates, flags));
  return done(run_verified(&s->impl, gates, flags & ~QS_RUN_VERIFY));
}

int qs_get_verify(qs_state* s, double* max_abs_diff, double* norm_drift) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_get_verify: bad state");
  if (max_abs_diff) *max_abs_diff = s->impl.verify_diff;
  if (norm_drift) *norm_drift = s->impl.verify_drift;
  return QS_OK;
}

static int check_terms(const char* who, int nterms, const uint64_t* x, const uint64_t* z,
                       const double* coeff) {
  if (nterms < 0) return fail(QS_EINVAL, std::string(who) + ": nterms < 0");
  if (nterms > 0 && (!x || !z || !coeff)) return fail(QS_EINVAL, std::string(who) + ": NULL term array");
  return QS_OK;
}

int qs_probabilities(qs_state* s, double* p1, double* norm2, void* full, size_t full_bytes) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_probabilities: bad state");
  if (full) {
    if (((uintptr_t)full) & 7) return fail(QS_EINVAL, "qs_probabilities: full not 8-byte aligned");
    if (full_bytes < (((size_t)1) << s->impl.n) * sizeof(double))
      return fail(QS_ERANGE, "qs_probabilities: full buffer too small");
    int rc = check_device_buffer(full, (((size_t)1) << s->impl.n) * sizeof(double), s->impl.device,
                                 "qs_probabilities: full");
    if (rc) return rc;
  }
  if (!p1 && !norm2 && !full) return QS_OK;
  return done(qs::launch_probabilities(&s->impl, p1, norm2, (double*)full));
}

int qs_probabilities_noalloc(qs_state* s, double* p1_dev, double* norm2_dev, void* full,
                             size_t full_bytes) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_probabilities_noalloc: bad state");
  const int n = s->impl.n;
  if (full) {
    if (((uintptr_t)full) & 7) return fail(QS_EINVAL, "qs_probabilities_noalloc: full not 8-byte aligned");
    if (full_bytes < (((size_t)1) << n) * sizeof(double))
      return fail(QS_ERANGE, "qs_probabilities_noalloc: full buffer too small");
    int rc = check_device_buffer(full, (((size_t)1) << n) * sizeof(double), s->impl.device,
                                 "qs_probabilities_noalloc: full");
    if (rc) return rc;
  }
  if (p1_dev) {
    if (((uintptr_t)p1_dev) & 7) return fail(QS_EINVAL, "qs_probabilities_noalloc: p1 not 8-byte aligned");
    int rc = check_device_buffer(p1_dev, (size_t)n * sizeof(double), s->impl.device,
                                 "qs_probabilities_noalloc: p1");
    if (rc) return rc;
  }
  if (norm2_dev) {
    if (((uintptr_t)norm2_dev) & 7)
      return fail(QS_EINVAL, "qs_probabilities_noalloc: norm2 not 8-byte aligned");
    int rc = check_device_buffer(norm2_dev, sizeof(double), s->impl.device,
                                 "qs_probabilities_noalloc: norm2");
    if (rc) return rc;
  }
  if (!p1_dev && !norm2_dev && !full) return QS_OK;
  return done(qs::launch_probabilities_noalloc(&s->impl, p1_dev, norm2_dev, (double*)full));
}

int qs_expect_pauli(qs_state* s, int nterms, const uint64_t* x, const uint64_t* z,
                    const double* coeff, double* out) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_expect_pauli: bad state");
  if (!out) return fail(QS_EINVAL, "qs_expect_pauli: out is NULL");
  int rc = check_terms("qs_expect_pauli", nterms, x, z, coeff);
  if (rc) return rc;
  qs::PauliTable t;
  Status st = qs::build_pauli_table(s->impl.n, nterms, x, z, coeff, &t);
  if (!st.good()) return done(st);
  return done(qs::launch_expect(&s->impl, t, out));
}

int qs_apply_pauli_sum(qs_state* src, qs_state* dst, int nterms, const uint64_t* x,
                       const uint64_t* z, const double* coeff) {
  if (!valid_state(src) || !valid_state(dst)) return fail(QS_EINVAL, "qs_apply_pauli_sum: bad state");
  if (src->impl.n != dst->impl.n || src->impl.dtype != dst->impl.dtype)
    return fail(QS_EINVAL, "qs_apply_pauli_sum: states differ in n or dtype");
  if (src->impl.ptr == dst->impl.ptr) return fail(QS_EINVAL, "qs_apply_pauli_sum: src and dst alias");
  int rc = check_terms("qs_apply_pauli_sum", nterms, x, z, coeff);
  if (rc) return rc;
  qs::PauliTable t;
  Status st = qs::build_pauli_table(src->impl.n, nterms, x, z, coeff, &t);
  if (!st.good()) return done(st);
  return done(qs::launch_apply_pauli_sum(&src->impl, &dst->impl, t));
}

int qs_grad_adjoint(qs_state* s, const qs_op* ops, int nops, const double* theta, int nparams,
                    int nterms, const uint64_t* x, const uint64_t* z, const double* coeff,
                    qs_state* lambda, int flags, double* energy, double* grad) {
  if (!valid_state(s) || !valid_state(lambda)) return fail(QS_EINVAL, "qs_grad_adjoint: bad state");
  if (s->impl.n != lambda->impl.n || s->impl.dtype != lambda->impl.dtype)
    return fail(QS_EINVAL, "qs_grad_adjoint: lambda differs in n or dtype");
  if (s->impl.ptr == lambda->impl.ptr) return fail(QS_EINVAL, "qs_grad_adjoint: lambda aliases the state");
  if (nops < 0 || (nops > 0 && !ops)) return fail(QS_EINVAL, "qs_grad_adjoint: bad op list");
  if (nparams < 0 || (nparams > 0 && !grad)) return fail(QS_EINVAL, "qs_grad_adjoint: bad gradient buffer");
  if (flags & ~(QS_ADJ_STATE_IS_FINAL | QS_ADJ_WIDE_TILES))
    return fail(QS_EINVAL, "qs_grad_adjoint: unknown flags");
  int rc = check_terms("qs_grad_adjoint", nterms, x, z, coeff);
  if (rc) return rc;
  std::vector<qs::XGate> gates;
  Status st = qs::normalize_ops(s->impl.n, ops, nops, theta, nparams, &gates);
  if (!st.good()) return done(st);
  qs::PauliTable t;
  st = qs::build_pauli_table(s->impl.n, nterms, x, z, coeff, &t);
  if (!st.good()) return done(st);
  return done(qs::run_adjoint(&s->impl, &lambda->impl, gates, nparams, t, flags, energy, grad));
}

int qs_plan(int n, int dtype, const qs_op* ops, int nops, const double* theta, int nparams,
            int flags, qs_plan_info* info, int32_t* order, int32_t* pass_of) {
  if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_EINVAL, "qs_plan: bad dtype");
  if (n < 1 || n > max_qubits(dtype)) return fail(QS_ERANGE, "qs_plan: n out of range");
  if (nops < 0 || (nops > 0 && !ops)) return fail(QS_EINVAL, "qs_plan: bad op list");
  if (nparams < 0) return fail(QS_EINVAL, "qs_plan: nparams < 0");
  if (flags & ~(QS_RUN_NO_FUSION | QS_RUN_WIDE_TILES | QS_PLAN_ADJOINT_REVERSE))
    return fail(QS_EINVAL, "qs_plan: unknown flags");
  const bool reverse = (flags & QS_PLAN_ADJOINT_REVERSE) != 0;
  if (reverse && (flags & QS_RUN_NO_FUSION))
    return fail(QS_EINVAL, "qs_plan: QS_PLAN_ADJOINT_REVERSE with QS_RUN_NO_FUSION");
  std::vector<qs::XGate> gates;
  Status st = qs::normalize_ops(n, ops, nops, theta, nparams, &gates);
  if (!st.good()) return done(st);
  qs::Plan plan;
  const bool wide = (flags & QS_RUN_WIDE_TILES) != 0;
  if (reverse) {
    // as the adjoint's reverse sweep plans it
    std::vector<qs::XGate> rev;
    qs::reverse_daggered(gates, &rev);
    qs::plan_gates(n, dtype, rev, true, &plan, /*allow_single=*/false, qs::kAdjMaxSlots, /*grad=*/true, wide);
  } else {
    qs::plan_gates(n, dtype, gates, !(flags & QS_RUN_NO_FUSION), &plan, true, 1 << 30, false, wide);
  }
  const double tiles = reverse ? 2.0 : 1.0;  // psi and lambda in the reverse sweep
  if (info) {
    memset(info, 0, sizeof(*info));
    const double S = (double)((size_t)1 << n) * (double)qs::amp_bytes(dtype);
    for (const qs::Pass& p : plan.passes) {
      ++info->passes;
      if (p.kind == qs::kPassFused) {
        ++info->fused;
        info->remaps += p.remaps;
        info->fused_ops += p.nops;
        info->hbm_bytes += tiles * 2 * S;
      } else if (p.kind == qs::kPass1q) {
        ++info->single_1q;
        info->hbm_bytes += tiles * 2 * S;
      } else {
        ++info->single_cu;
        info->hbm_bytes += tiles * S;
      }
    }
  }
  for (int g = 0; g < nops; ++g) {
    if (order) order[g] = plan.order[g];
    if (pass_of) pass_of[g] = plan.pass_of[g];
  }
  return QS_OK;
}

int qs_plan_reorder(int n, int nlocal, const qs_op* ops, int nops, const double* theta,
                    int nparams, qs_reorder_info* info, qs_op* out_ops, int32_t* remap_at,
                    int32_t* remap_perm, int cap, int32_t* final_perm) {
  if (n < 1 || n > QS_MAX_QUBITS_C64) return fail(QS_ERANGE, "qs_plan_reorder: n out of range");
  if (nlocal < 1 || nlocal > n) return fail(QS_EINVAL, "qs_plan_reorder: nlocal out of range");
  if (nops < 0 || (nops > 0 && !ops)) return fail(QS_EINVAL, "qs_plan_reorder: bad op list");
  if (nparams < 0) return fail(QS_EINVAL, "qs_plan_reorder: nparams < 0");
  if (out_ops && (cap < 0 || !final_perm || (cap > 0 && (!remap_at || !remap_perm))))
    return fail(QS_EINVAL, "qs_plan_reorder: NULL output array");
  std::vector<qs::XGate> gates;
  Status st = qs::normalize_ops(n, ops, nops, theta, nparams, &gates);
  if (!st.good()) return done(st);
  qs::ReorderPlan plan;
  st = qs::plan_reorder(n, nlocal, gates, &plan);
  if (!st.good()) return done(st);
  if (info) *info = plan.info;
  if (!out_ops) return QS_OK;
  const int R = (int)plan.remap_at.size();
  if (R > cap) return fail(QS_ERANGE, "qs_plan_reorder: cap smaller than the number of reorderings");
  for (int g = 0; g < nops; ++g) {
    out_ops[g] = ops[g];
    out_ops[g].target = plan.tgt[g];
    if (ops[g].kind == QS_OP_CU) out_ops[g].control = plan.ctl[g];
  }
  for (int r = 0; r < R; ++r) remap_at[r] = plan.remap_at[r];
  if (R > 0) memcpy(remap_perm, plan.remap_perm.data(), (size_t)R * n * sizeof(int32_t));
  memcpy(final_perm, plan.final_perm.data(), (size_t)n * sizeof(int32_t));
  return QS_OK;
}

int qs_run_reordered(qs_state* s, int nlocal, const qs_op* ops, int nops, const double* theta,
                     int nparams, int flags, qs_reorder_info* info) {
  if (!valid_state(s)) return fail(QS_EINVAL, "qs_run_reordered: bad state");
  if (nlocal < 1 || nlocal > s->impl.n) return fail(QS_EINVAL, "qs_run_reordered: nlocal out of range");
  if (nops < 0 || (nops > 0 && !ops)) return fail(QS_EINVAL, "qs_run_reordered: bad op list");
  if (nparams < 0) return fail(QS_EINVAL, "qs_run_reordered: nparams < 0");
  if (flags & ~(QS_RUN_NO_FUSION | QS_RUN_WIDE_TILES)) return fail(QS_EINVAL, "qs_run_reordered: unknown flags");
  std::vector<qs::XGate> gates;
  Status st = qs::normalize_ops(s->impl.n, ops, nops, theta, nparams, &gates);
  if (!st.good()) return done(st);
  return done(qs::run_reordered(&s->impl, nlocal, gates, flags, info));
}

int qs_batch_create(int dtype, int ncircuits, const int32_t* n, const int64_t* op_off,
                    const qs_op* ops, const int64_t* par_off, const double* theta,
                    const int64_t* term_off, const uint64_t* x, const uint64_t* z,
                    const double* coeff, void* stream, qs_batch** out) {
  if (!out) return fail(QS_EINVAL, "qs_batch_create: out is NULL");
  *out = nullptr;
  if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_EINVAL, "qs_batch_create: bad dtype");
  if (ncircuits < 0) return fail(QS_EINVAL, "qs_batch_create: ncircuits < 0");
  if (!op_off || !par_off || !term_off) return fail(QS_EINVAL, "qs_batch_create: NULL offsets");
  if (op_off[0] != 0 || par_off[0] != 0 || term_off[0] != 0)
    return fail(QS_EINVAL, "qs_batch_create: offsets must start at 0");
  for (int c = 0; c < ncircuits; ++c)
    if (op_off[c + 1] < op_off[c] || par_off[c + 1] < par_off[c] || term_off[c + 1] < term_off[c])
      return fail(QS_EINVAL, "qs_batch_create: offsets decrease at circuit " + std::to_string(c));
  if (ncircuits > 0 && !n) return fail(QS_EINVAL, "qs_batch_create: n is NULL");
  if (op_off[ncircuits] > 0 && !ops) return fail(QS_EINVAL, "qs_batch_create: ops is NULL");
  if (par_off[ncircuits] > 0 && !theta) return fail(QS_EINVAL, "qs_batch_create: theta is NULL");
  if (term_off[ncircuits] > 0 && (!x || !z || !coeff))
    return fail(QS_EINVAL, "qs_batch_create: NULL term array");
  if (par_off[ncircuits] > INT32_MAX || term_off[ncircuits] > INT32_MAX)
    return fail(QS_ERANGE, "qs_batch_create: too many parameters or terms");
  qs::BatchImpl* b = nullptr;
  Status st = qs::batch_create(dtype, ncircuits, n, op_off, ops, par_off, theta, term_off, x, z,
                               coeff, (hipStream_t)stream, &b);
  if (!st.good()) return done(st);
  qs_batch* h = new (std::nothrow) qs_batch;
  if (!h) {
    qs::batch_destroy(b);
    return fail(QS_ENOMEM, "qs_batch_create: handle allocation failed");
  }
  h->impl = b;
  *out = h;
  return QS_OK;
}

int qs_batch_run(qs_batch* b, const qs_batch_tuning* tuning, double* energy, double* grad) {
  if (!b || !b->impl) return fail(QS_EINVAL, "qs_batch_run: bad batch");
  return done(qs::batch_run(b->impl, tuning, energy, grad));
}

int qs_batch_destroy(qs_batch* b) {
  if (!b) return QS_OK;
  qs::batch_destroy(b->impl);
  delete b;
  return QS_OK;
}

int qs_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst) return fail(QS_EINVAL, "qs_stream_copy: NULL pointer");
  if ((((uintptr_t)src) | ((uintptr_t)dst) | bytes) & 15)
    return fail(QS_EINVAL, "qs_stream_copy: pointers and size must be multiples of 16");
  const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
  if (a < b + bytes && b < a + bytes) return fail(QS_EINVAL, "qs_stream_copy: buffers overlap");
  if (bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
      (void)hipGetLastError();
      return fail(QS_ENODEV, "qs_stream_copy: no HIP device");
    }
    int rc = check_device_buffer(src, bytes, dev, "qs_stream_copy: src");
    if (rc) return rc;
    rc = check_device_buffer(dst, bytes, dev, "qs_stream_copy: dst");
    if (rc) return rc;
  }
  return done(qs::launch_stream_copy(src, dst, bytes, (hipStream_t)stream));
}

}  // extern "C"
