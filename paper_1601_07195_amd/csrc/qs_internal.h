// qs_internal.h -- host-side structures and kernel launchers of libqs.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdlib.h>
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
  int cus = 0;       // compute units of the device (0 = not queried yet)
  int grid_limit = 0;  // cap on a fused pass's workgroups (0 = automatic)
  int exec = QS_EXEC_AUTO;  // fused passes: compiled per shape or interpreted
  double verify_diff = -1.0, verify_drift = -1.0;  // last QS_RUN_VERIFY results
  DevBuf red;        // reduction partials
  DevBuf scal;       // small device results (energy)
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
// Dense 2^k x 2^k gate (u: 2 * 4^k doubles, row-major (re, im)) on targets.
Status launch_apply_kq(StateImpl* s, int k, const int32_t* targets, const double* u);
// Relabel qubit q as perm[q] in place (perm: host, a permutation of 0..n-1).
Status launch_permute(StateImpl* s, const int32_t* perm);

// ------------------------------------------------------------ reductions
// Per-qubit P(bit = 1), total norm^2 and optionally the full |a_i|^2 vector.
Status launch_probabilities(StateImpl* s, double* p1_host, double* norm2_host, double* full_dev);
// The same sums with the partials in a static per-device array (no
// allocation); p1_dev / norm2_dev are device outputs.  Asynchronous.
Status launch_probabilities_noalloc(StateImpl* s, double* p1_dev, double* norm2_dev,
                                    double* full_dev);

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
// max_i |a_i - b_i| for b a device state of a's shape (synchronises).
// Dynamic LDS bytes that cap a streaming launch of `block`-thread
// workgroups (already holding `static_lds` bytes) at `waves` waves per
// SIMD (0: no cap); QS_STREAM_WAVES, when set, replaces `waves`.
size_t stream_lds(int block, size_t static_lds, int waves);
Status max_abs_diff(StateImpl* a, const void* b, double* out_host);
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

// Qubit-reordering plan for a state split by its top n - nlocal qubits.
struct ReorderPlan {
  std::vector<int> tgt, ctl;         // each gate's target / control position (-1: none)
  std::vector<int> remap_at;         // reordering r comes just before gate remap_at[r]
  std::vector<int32_t> remap_perm;   // its permutation of positions, n entries each
  std::vector<int32_t> final_perm;   // back to the caller's qubit order
  qs_reorder_info info;
};
Status plan_reorder(int n, int nlocal, const std::vector<XGate>& gates, ReorderPlan* out);
Status run_reordered(StateImpl* s, int nlocal, const std::vector<XGate>& gates, int flags,
                     qs_reorder_info* info);

// ------------------------------------------------------- fusion planning
// A fused pass keeps one tile of 2^T amplitudes on chip per workgroup: the
// kLaneQ low qubits (coalesced) plus high qubits chosen per pass.  Each of
// the 256 threads holds 2^NREG amplitudes in registers: its 8 thread-index
// bits and NREG register-index bits are mapped to tile bits by an FMap.
constexpr int kFuseThreadBits = 8;
struct FuseGeom {
  int nreg;   // register bits per thread (4 for complex128, 5 for complex64)
  int T;      // tile bits = nreg + 8
  int L;      // low qubits always in the tile (6 for complex128, 7 for complex64)
  int lane0;  // first lane tile bit (0 for complex128; 1 for complex64, whose
              // tile bit 0 is inside the 16-byte unit)
};
// wide: fewer low qubits fixed in every tile (4 at complex128, 5 at
// complex64, instead of 6 / 7): three more free tile qubits per pass, so
// fewer passes, each moving its data in 256-byte contiguous runs.
FuseGeom fuse_geom(int dtype, bool wide = false);

struct FMap {
  int8_t thr[8];  // tile bit held by thread-index bit i
  int8_t reg[5];  // tile bit held by register-index bit k (nreg used)
  int8_t pad[3];
};

// Bit "spec": where a qubit currently lives for a fused op.
enum SpecWhere { kInReg = 0, kInThread = 1, kOutside = 2, kNoBit = 3 };
inline int32_t make_spec(int where, int index) { return (where << 8) | index; }

// kOpPhaseRun: phase ops (diagonal, d0 = 1) on one target `tgt` (a register
// bit, a thread bit or outside the tile) whose controls are not register
// bits.  The kernel multiplies their d1 into one per-lane factor and scales
// the target-bit-1 amplitudes once.  Entries controlled outside the tile
// come from two tables indexed by the tile index (m[0]: byte offset from the
// maps, m[1]: low-table bits, m[2]: present); two or more entries with no
// control or a thread-bit control come from one table indexed by the thread
// (m[3]: byte offset, m[4]: present); otherwise `aux` explicit entries follow
// (kOpPhaseEntry, the control spec in `ctl`).
enum FOpKind { kOpRemap = 0, kOpU = 1, kOpDiag = 2, kOpPhaseRun = 3, kOpPhaseEntry = 4 };
// FOp::kind bits 8..15: the Pauli generator of a gradient op; bit 16 on a
// diagonal op: d0 = 1 (a phase), set when the plan is uploaded.
constexpr int32_t kDiagPhase = 1 << 16;
// A U op whose matrix has real entries, flagged at upload.
constexpr int32_t kUReal = 1 << 17;
struct FOp {
  int32_t kind;
  int32_t tgt;   // kOpU: register bit; kOpDiag: spec of the target; kOpRemap: new FMap index
  int32_t ctl;   // spec of the control (kNoBit when none)
  int32_t aux;   // kOpRemap: old FMap index; adjoint: gradient slot in the pass or -1
  double m[8];   // kOpU: the 2x2; kOpDiag: d0 = (m[0], m[1]), d1 = (m[6], m[7])
};

enum PassKind { kPassFused = 0, kPass1q = 1, kPassCU = 2 };
struct Pass {
  int kind;
  int grad_first, ngrad;  // fused adjoint: rows of this pass's gradient slots in Plan::grad_rows
  int gate;          // streaming passes: index of the gate
  int op_first, nops;  // fused: range in Plan::ops
  int map_load, map_store;
  int nh;            // fused: number of high tile qubits
  int8_t hpos[8];    // fused: the high tile qubits, ascending
  int remaps;
};
struct Plan {
  FuseGeom geom;  // the tile geometry the plan was made for
  std::vector<Pass> passes;
  std::vector<FOp> ops;
  std::vector<FMap> maps;
  std::vector<int> order;  // gate indices in execution order
  std::vector<int> pass_of;  // pass of each gate (by gate index)
  std::vector<int> grad_rows;  // per fused pass slot: the gate's param (gradient row)
  // Phase-run tables (re, im pairs): for a run's entries controlled by qubits
  // outside the tile, the product of their phases by the tile index, split
  // into a table over its low bits and one over its high bits.
  std::vector<double> run_tab;
};
// Plan `gates` (applied in list order) for an n-qubit state of `dtype`.
// allow_single: a pass with one gate may use the streaming kernels.
// max_grad: at most this many gradient-carrying gates (XGate::param >= 0)
// per fused pass.
// grad: gates with param >= 0 get gradient slots (adjoint sweeps) and are
// never merged with other gates; otherwise consecutive gates on the same
// target and control may be merged into one op.
void plan_gates(int n, int dtype, const std::vector<XGate>& gates, bool fuse, Plan* out,
                bool allow_single = true, int max_grad = 1 << 30, bool grad = false,
                bool wide = false);

// Fused adjoint reverse sweep (n >= tile bits): `rev` holds the daggered
// gates in reverse order; rotations keep their kind and carry in `param` the
// index of their gradient row.  On return rows[i] is the gradient row of
// slot i and slot_sums_dev[i] (device, in the state's reduction buffer) its
// contribution, summed in a fixed order.
Status run_adjoint_fused(StateImpl* s, StateImpl* lam, const std::vector<XGate>& rev,
                         std::vector<int>* rows, double** slot_sums_dev, bool wide = false);
// out[r] = sum of part[r * ncols + c] over c, fixed order (one workgroup per row).
Status launch_sum_rows(StateImpl* s, const double* part, int nrows, int ncols, double* out);
constexpr int kAdjMaxSlots = 64;  // gradient rows per fused adjoint pass
bool gate_is_diagonal(const XGate& g);

// ------------------------------------------- fused passes compiled per shape
// A pass's kernel is generated from its plan (straight-line code, every
// structural field fixed) and compiled through hipRTC; kernels are cached by
// their text.  entry < 0: the pass runs on the interpreter kernels.
struct JitPass {
  int entry = -1;
};
struct JitStats {
  long long kernels = 0;         // kernels compiled by this process
  long long cached = 0;          // kernels held in the cache
  long long modules_loaded = 0;  // code objects loaded on a device
  double compile_seconds = 0.0;  // wall time spent compiling
  long long loaded_from_disk = 0;  // kernels found in the on-disk cache
  long long programs_clang = 0;    // programs compiled by child clang processes
  long long programs_hiprtc = 0;   // programs compiled in-process by hipRTC
};
// Kernel text of one fused pass (after the kernel's name); empty when the
// generator does not take the pass.
std::string jit_pass_text(const Plan& plan, const Pass& p, int n, int dtype, bool adjoint);
// Compile (or find in the cache) the kernels of every fused pass of `plan`.
Status jit_prepare(const Plan& plan, int n, int dtype, bool adjoint, std::vector<JitPass>* out);
// The pass's kernel on `device` (its module is loaded on first use).
Status jit_function(const JitPass& jp, int device, hipFunction_t* fn);
JitStats jit_stats();
// Whether the state's fused passes run compiled kernels (QS_EXEC_AUTO: from
// kJitAutoMinQubits qubits up, or as the QS_FUSED_EXEC environment variable
// says: "compiled" or "interpreted").
bool use_compiled_passes(const StateImpl* s);
constexpr int kJitAutoMinQubits = 26;
// Plan a gate list as qs_run would (adjoint: also the reverse sweep of
// qs_grad_adjoint) and compile its pass kernels; *nkernels: how many.
Status precompile_passes(int n, int dtype, const std::vector<XGate>& gates, bool adjoint,
                         bool wide, int* nkernels);
// The reverse sweep's gate list: U_j^dagger in reverse order.
void reverse_daggered(const std::vector<XGate>& gates, std::vector<XGate>* rev);

// ----------------------------------------------------------- adjoint
Status run_adjoint(StateImpl* s, StateImpl* lam, const std::vector<XGate>& gates,
                   int nparams, const PauliTable& h, int flags, double* energy, double* grad);

// ------------------------------------------------------------ batches
struct BatchImpl;
Status batch_create(int dtype, int ncirc, const int32_t* n, const int64_t* op_off,
                    const qs_op* ops, const int64_t* par_off, const double* theta,
                    const int64_t* term_off, const uint64_t* x, const uint64_t* z,
                    const double* coeff, hipStream_t stream, BatchImpl** out);
Status batch_run(BatchImpl* b, const qs_batch_tuning* tune, double* energy, double* grad);
void batch_destroy(BatchImpl* b);

}  // namespace qs

struct qs_state {
  qs::StateImpl impl;
};
struct qs_batch {
  qs::BatchImpl* impl;
};
