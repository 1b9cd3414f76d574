// qs_internal.h -- host-side structures and kernel launchers of libqs.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "qs.h"

namespace qs {

// Status carried from launchers to the C ABI.
struct Status {
  int code = QS_OK;
  std::string msg;
  static Status ok() { return {}; }
  bool good() const { return code == QS_OK; }
};
Status hip_status(hipError_t e, const char* what);

// Grow-only device buffer owned by a state handle.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Pinned host staging buffer paired with a device buffer: uploads of small
// tables (gate lists, Pauli terms) are queued on the state's stream; an
// event recorded after each copy guards the host side against reuse.
struct Staging {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};

struct StateImpl {
  int n = 0;
  int dtype = 0;
  void* ptr = nullptr;
  size_t bytes = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  DevBuf red;        // reduction partials
  DevBuf table;      // uploaded tables
  Staging stage;     // pinned host side of `table`
  double* result_host = nullptr;  // pinned, for reduction results
  size_t result_bytes = 0;
};

// Bytes per amplitude.
inline size_t amp_bytes(int dtype) { return dtype == QS_C128 ? 16 : 8; }

Status ensure_dev(StateImpl* s, DevBuf& b, size_t bytes);
Status ensure_result_host(StateImpl* s, size_t bytes);
// Copy `bytes` of host data into the state's table buffer (at `offset`).
Status upload_table(StateImpl* s, const void* src, size_t bytes);

// ---------------------------------------------------------------- gates
Status launch_init_basis(StateImpl* s, uint64_t index);
Status launch_apply_1q(StateImpl* s, int k, const double* q);
Status launch_apply_cu(StateImpl* s, int c, int t, const double* q);
Status launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream);

// ------------------------------------------------------------ reductions
// Per-qubit P(bit = 1), total norm^2 and optionally the full |a_i|^2 vector.
Status launch_probabilities(StateImpl* s, double* p1_host, double* norm2_host, double* full_dev);

// Pauli-sum terms grouped by x mask, in the device layout of the reduction
// kernels (see qs_reduce.hip).
struct PauliGroup {
  uint64_t x;
  int32_t first;  // index of the first term of the group
  int32_t count;
};
struct PauliTerm {
  uint64_t z;
  double cr, ci;  // coeff * i^(number of Y factors), as a complex number
};
struct PauliTable {
  std::vector<PauliGroup> groups;
  std::vector<PauliTerm> terms;
};
Status build_pauli_table(int n, int nterms, const uint64_t* x, const uint64_t* z,
                         const double* coeff, PauliTable* out);
// <psi|H|psi> (synchronises).
Status launch_expect(StateImpl* s, const PauliTable& t, double* out_host);
// dst = H src (asynchronous).
Status launch_apply_pauli_sum(StateImpl* src, StateImpl* dst, const PauliTable& t);
// <a|b> into device double2 at dev_out (asynchronous).
Status launch_inner_dev(StateImpl* a, StateImpl* b, double* dev_out);

// ------------------------------------------------------- circuits / plan
// Gate in the executor's normalized form: a 2x2 matrix (double), target,
// optional control, and (for rotations) the generator kind and parameter.
struct XGate {
  int kind;      // QS_OP_U, QS_OP_CU, or a rotation kind
  int target;
  int control;   // -1 if none
  int param;     // rotations only
  double m[8];   // the matrix actually applied
};
Status normalize_ops(int n, const qs_op* ops, int nops, const double* theta, int nparams,
                     std::vector<XGate>* out);
Status run_gates(StateImpl* s, const std::vector<XGate>& gates, int flags);

// ----------------------------------------------------------- adjoint
Status run_adjoint(StateImpl* s, StateImpl* lam, const std::vector<XGate>& gates,
                   int nparams, const PauliTable& h, int flags, double* energy, double* grad);

}  // namespace qs

struct qs_state {
  qs::StateImpl impl;
};
