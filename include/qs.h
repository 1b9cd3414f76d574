/*
 * qs.h -- C ABI of libqs, a state-vector quantum circuit simulator for one
 * AMD Instinct MI355X (gfx950).
 *
 * The problem statement follows qHiPSTER (Smelyanskiy, Sawaya, Aspuru-Guzik,
 * arXiv:1601.07195), Sec. 2 "Background":
 *   - an n-qubit pure state is 2^n complex amplitudes stored densely in index
 *     order; qubit q is bit q of the amplitude index (so a gate on qubit k
 *     pairs amplitudes 2^k apart);
 *   - a single-qubit gate applies a 2x2 matrix Q to every such pair, Eq. (2);
 *   - a controlled gate applies Q to target t only where control bit c is 1,
 *     Eq. (3).
 *
 * Conventions shared by every entry point
 *   - Amplitudes are interleaved (re, im).  dtype QS_C128 stores two doubles
 *     per amplitude (16 B), QS_C64 two floats (8 B).  Every reduction
 *     (probabilities, norms, expectation values, gradients) accumulates in
 *     double precision on the GPU for both dtypes.
 *   - A 2x2 gate is 8 doubles, row-major q11, q12, q21, q22, each as (re, im);
 *     it maps (alpha_{..0..}, alpha_{..1..}) to Q (alpha_{..0..}, alpha_{..1..}).
 *     Unitarity is the caller's responsibility (it is never checked).
 *   - Rotations are R_P(theta) = exp(-i theta P / 2) for P in {X, Y, Z}.
 *   - Pauli strings are given by two bit masks: bit q of x is set where the
 *     factor on qubit q is X or Y, bit q of z where it is Z or Y.
 *   - "dev" pointers are device memory on the state's GPU, owned by the
 *     caller (e.g. a torch tensor); "host" pointers are ordinary host memory,
 *     read or written before the call returns.
 *   - All work is queued on the stream bound to the state (see qs_create).
 *     Calls that return only device results are asynchronous; calls that
 *     return host values (probabilities, expectation, energy, gradient)
 *     synchronise that stream before returning.
 *   - Every argument is validated on the host before any GPU work is queued;
 *     on error nothing is launched and the state is unchanged.  The return
 *     value is QS_OK (0) or a negative QS_E* code; qs_last_error() gives a
 *     message for the calling thread's most recent failure.
 *   - A state handle must not be used from two host threads at once.
 */
#ifndef QS_H_
#define QS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define QS_OK 0
#define QS_EINVAL (-1)      /* bad argument (index out of range, NULL, c == t, ...) */
#define QS_ENOMEM (-2)      /* device or host allocation failed */
#define QS_EHIP (-3)        /* a HIP runtime call or kernel launch failed */
#define QS_ENODEV (-4)      /* no usable gfx950 device */
#define QS_ERANGE (-5)      /* size out of range (n too large, buffer too small) */
#define QS_EVERIFY (-6)     /* a QS_RUN_VERIFY check failed */

/* Amplitude types. */
#define QS_C64 1            /* complex64: float re, float im */
#define QS_C128 2           /* complex128: double re, double im */

/* Largest n per dtype: the state must fit one MI355X (288 GB HBM3E). */
#define QS_MAX_QUBITS_C128 33
#define QS_MAX_QUBITS_C64 34

/* Gate kinds of a qs_op. */
#define QS_OP_U 0           /* general 1-qubit gate `mat` on `target` (Eq. 2) */
#define QS_OP_CU 1          /* controlled `mat`: control `control`, target `target` (Eq. 3) */
#define QS_OP_RX 2          /* exp(-i theta X / 2) on `target`, theta = theta[param] */
#define QS_OP_RY 3          /* exp(-i theta Y / 2) */
#define QS_OP_RZ 4          /* exp(-i theta Z / 2) */

/* One gate of a circuit (80 bytes, no padding). */
typedef struct qs_op {
  int32_t kind;     /* QS_OP_* */
  int32_t target;   /* 0 <= target < n */
  int32_t control;  /* QS_OP_CU: 0 <= control < n, control != target; else ignored */
  int32_t param;    /* rotations: index into theta; else ignored */
  double mat[8];    /* QS_OP_U / QS_OP_CU: the 2x2 gate; else ignored */
} qs_op;

typedef struct qs_state qs_state; /* opaque handle, owned by the library */

/* Library version as 10000*major + 100*minor + patch. */
int qs_version(void);

/* Static text for a status code. */
const char* qs_strerror(int code);

/* Message for the calling thread's last failed call ("" if none). */
const char* qs_last_error(void);

/*
 * Bind an n-qubit state to caller-owned device memory (Sec. 2: 2^n
 * amplitudes of `dtype`, i.e. 2^n * 16 or 2^n * 8 bytes).
 *   n        1 <= n <= QS_MAX_QUBITS_C128 (QS_C128) or QS_MAX_QUBITS_C64 (QS_C64)
 *   dtype    QS_C64 or QS_C128
 *   dev_ptr  device pointer, 256-byte aligned, at least 2^n amplitudes; the
 *            caller keeps ownership and must keep it alive until qs_destroy
 *   bytes    size of the buffer at dev_ptr (QS_ERANGE if too small)
 *   stream   hipStream_t to queue work on (NULL = the null stream)
 *   out      receives the handle
 * The amplitudes are not touched (use qs_init_basis).  No GPU work is done
 * here; the device is the one current on the calling thread, and dev_ptr
 * must be device memory of that device (checked with the runtime's pointer
 * attributes, so a host pointer is refused here rather than faulting later).
 * Errors: QS_EINVAL (NULL out/dev_ptr, bad dtype, misaligned, not device
 * memory of the current device), QS_ERANGE (bytes, or the allocation behind
 * dev_ptr, too small), QS_ENOMEM (handle allocation), QS_ENODEV (no device
 * current, or the current device is not a gfx950).
 */
int qs_create(int n, int dtype, void* dev_ptr, size_t bytes, void* stream,
              qs_state** out);

/* Release the handle and the library's scratch memory (not dev_ptr).
 * Waits for the state's queued work first.  NULL is accepted. */
int qs_destroy(qs_state* s);

/* Queue later work of this state on another hipStream_t. */
int qs_set_stream(qs_state* s, void* stream);

/*
 * Cap the number of workgroups of this state's fused passes (qs_run's
 * cache-blocked passes, Sec. 4.4, and the reverse sweep of qs_grad_adjoint).
 * 0, the default, lets the library choose (one workgroup per tile up to a
 * launch limit).  A positive cap below the number of tiles makes every
 * workgroup process several tiles in turn (a persistent grid), e.g. to leave
 * compute units to concurrent work.  States are unaffected bit for bit;
 * gradients change only in the rounding of their fixed-order sums, which
 * depend on how tiles are shared among workgroups.
 * Errors: QS_EINVAL (bad state, negative cap).
 */
int qs_set_grid_limit(qs_state* s, int max_workgroups);

/*
 * How this state's fused passes (qs_run's cache-blocked passes, Sec. 4.4,
 * and the reverse sweep of qs_grad_adjoint) execute:
 *   QS_EXEC_INTERPRETED  one precompiled kernel per dtype decodes the
 *                        pass's op list as it runs;
 *   QS_EXEC_COMPILED     each pass gets its own straight-line kernel,
 *                        generated from its op list and compiled at run time
 *                        (ROCm clang, or hipRTC; see qs_precompile) the
 *                        first time a pass of that shape runs,
 *                        then cached for the process: the same circuit form
 *                        with other matrices or angles runs without
 *                        compiling again;
 *   QS_EXEC_AUTO         (default) compiled for n >= 26, interpreted below;
 *                        the environment variable QS_FUSED_EXEC set to
 *                        "compiled" or "interpreted" overrides AUTO for every
 *                        state.
 * Both give the same amplitudes up to floating-point rounding (the order of
 * operations inside a pass may differ).  A pass the generator does not take
 * runs interpreted.  Compilation needs no GPU (see qs_precompile); its cost
 * is reported by qs_jit_stats.
 * Compiled passes also choose their tile order, that is which workgroup
 * takes which tile: 2^k regions of the tiles walked side by side,
 * k = 0..7.  Each order the tile count allows is timed on one launch, with
 * HIP events on the state's stream that are read at a later launch once
 * complete.  From then on, for the rest of the process, that kernel at that
 * tile count uses the fastest order.  The order changes no result bit.  The
 * environment variable QS_TILE_ORDER=k fixes the order instead.
 * Errors: QS_EINVAL (bad state or mode).
 */
#define QS_EXEC_AUTO 0
#define QS_EXEC_INTERPRETED 1
#define QS_EXEC_COMPILED 2
int qs_set_fused_exec(qs_state* s, int mode);

/*
 * Compile, without running anything, the fused-pass kernels that qs_run
 * (and, with QS_PRECOMPILE_ADJOINT, the reverse sweep of qs_grad_adjoint)
 * would use for this gate list on an n-qubit state of `dtype`, so that a
 * later call starts without compiling.  Host only; no GPU is needed.
 * Arguments as for qs_plan.  *nkernels (may be NULL) receives the number of
 * distinct pass kernels the list needs.
 * Errors: QS_EINVAL (malformed list), QS_EHIP (compiler failure; the message
 * holds the compiler's log).
 */
#define QS_PRECOMPILE_ADJOINT 1
int qs_precompile(int n, int dtype, const qs_op* ops, int nops, const double* theta,
                  int nparams, int flags, int32_t* nkernels);

/* Counters of the compiled-pass cache of this process.  Kernels are
 * compiled by the ROCm clang driver ($QS_JIT_CLANG, $ROCM_PATH/llvm/bin or
 * /opt/rocm/llvm/bin) in parallel child processes, or in-process by hipRTC
 * when no driver is found, when a child compilation fails, or with
 * QS_JIT_COMPILER=hiprtc (hipRTC serialises compilations).  With the
 * environment variable QS_JIT_CACHE_DIR naming a writable directory,
 * compiled kernels are also kept there and loaded by later processes
 * (each kernel's text is stored beside it and compared in full). */
typedef struct qs_jit_stats {
  int64_t kernels_compiled;  /* kernels compiled so far */
  int64_t kernels_cached;    /* kernels held in the cache */
  int64_t modules_loaded;    /* code objects loaded onto devices */
  double compile_seconds;    /* host wall time spent compiling */
  int64_t kernels_from_disk; /* kernels loaded from the on-disk cache */
  int64_t programs_clang;    /* compilations run by the ROCm clang driver in child processes */
  int64_t programs_hiprtc;   /* compilations run in-process by hipRTC (the fallback) */
} qs_jit_stats;
int qs_get_jit_stats(qs_jit_stats* out);

/* State = computational basis state |index> (index < 2^n); |0...0> for 0. */
int qs_init_basis(qs_state* s, uint64_t index);

/*
 * Single-qubit gate on qubit k, in place: Eq. (2) of Sec. 2, i.e. Q applied
 * to every pair (i, i + 2^k) with bit k of i clear (the loop nest of
 * Fig. 2).  q: host, 8 doubles as above.  Errors: QS_EINVAL (k out of range,
 * NULL), QS_EHIP.
 */
int qs_apply_1q(qs_state* s, int k, const double* q);

/*
 * Controlled gate, in place: Eq. (3) of Sec. 2, i.e. Q applied to the pairs
 * (i, i + 2^t) whose control bit c is 1; the other amplitudes are neither
 * read nor written.  Errors: QS_EINVAL (c or t out of range, c == t, NULL).
 */
int qs_apply_cu(qs_state* s, int c, int t, const double* q);

/*
 * Dense gate on a block of k qubits, in place: Eq. (2) read for k qubits
 * (the paper fuses gates on a set of qubits into one pass, Sec. 4.4; this
 * takes the block's product as one matrix).  Every group of 2^k amplitudes
 * whose indices differ only in the target bits, listed in the order of that
 * k-bit index, is replaced by u times the group.
 *   k        1 .. QS_KQ_MAX
 *   targets  host, k distinct qubits in [0, n); bit j of u's row and column
 *            index is qubit targets[j]
 *   u        host, 2^k x 2^k complex entries, row-major, each (re, im):
 *            2 * 4^k doubles (a complex64 state uses them rounded to float)
 * Asynchronous on the state's stream; the matrix is copied before return.
 * u is not checked for unitarity.  complex128 gates on five qubits run on
 * the FP64 matrix cores (the gate as a dense real contraction), the others
 * on the vector units.
 * Errors: QS_EINVAL (k out of range, a target out of range or repeated,
 * NULL), QS_ENOMEM, QS_EHIP.
 */
#define QS_KQ_MAX 5
int qs_apply_kq(qs_state* s, int k, const int32_t* targets, const double* u);

/*
 * Apply a gate list in order, in place.  Consecutive gates may be fused
 * into one pass over the state that keeps a block of amplitudes on chip
 * while several gates are applied to it (cache blocking by gate fusion,
 * Sec. 4.4 and Fig. 4); gates acting on disjoint qubits may be reordered
 * past each other.  The result equals applying the gates one by one up to
 * floating-point rounding.
 *   ops     host array of nops records
 *   theta   host array of nparams angles (may be NULL if no rotations)
 *   flags   QS_RUN_* bits
 * Errors: QS_EINVAL for any malformed op (checked before any launch).
 */
#define QS_RUN_NO_FUSION 1  /* one streaming pass per gate (no cache blocking) */
/* Fused passes keep 4 (complex128) or 5 (complex64) low qubits in every
 * tile instead of 6 / 7: three more free tile qubits, so fewer passes over
 * the state, each moving its data in 256-byte contiguous runs instead of
 * 1 KiB ones (a lower fraction of peak bandwidth per pass, less time per
 * circuit).  Also accepted by qs_plan, qs_run_reordered and qs_precompile. */
#define QS_RUN_WIDE_TILES 2
/* Debug check (costs a scratch copy of the state and a second, unfused
 * run): the list runs as asked, and also, on a copy of the input, as one
 * streaming kernel per gate (Eq. 2 / 3 gate by gate); the call fails with
 * QS_EVERIFY when the two results differ, or the norm moves, by more than
 * rounding allows (64 units in the last place of the amplitude type times
 * sqrt(gates + 1)).  A non-unitary gate (the paper assumes unitary ones,
 * Sec. 2) fails the norm check.  qs_get_verify returns the last figures. */
#define QS_RUN_VERIFY 4
int qs_run(qs_state* s, const qs_op* ops, int nops, const double* theta,
           int nparams, int flags);

/* Results of the state's last QS_RUN_VERIFY run: max_i |fused_i - per-gate_i|
 * and |<psi|psi>_after - <psi|psi>_before| (-1 before any verified run).
 * Either pointer may be NULL.  Errors: QS_EINVAL (bad state). */
int qs_get_verify(qs_state* s, double* max_abs_diff, double* norm_drift);

/*
 * Qubit reordering in place (the state reordering of Sec. 6): qubit q is
 * relabelled perm[q], so the amplitude at index i moves to the index whose
 * bit perm[q] equals bit q of i, for every q.  A swap of two qubits is the
 * permutation that exchanges them.
 *   perm  host, n int32: a permutation of 0 .. n-1 (copied before return)
 * Runs as at most two passes of disjoint qubit swaps, each of one to three
 * launches: swaps of two qubits above the 1 KiB block bits (6 for complex128,
 * 7 for complex64) move only the blocks that change place, 2 (1 - 2^-k) S
 * bytes for k swaps (S = the state's bytes); swaps that touch a block bit
 * move 2 S bytes per launch of up to four.  The identity launches nothing.
 * Asynchronous on the state's stream; no scratch memory.
 * Errors: QS_EINVAL (NULL, not a permutation), QS_EHIP.
 */
int qs_permute_qubits(qs_state* s, const int32_t* perm);

/*
 * Counts of a qubit-reordering plan for a state split over 2^(n - nlocal)
 * shards by its top n - nlocal qubits (Sec. 3.2's distribution, with the
 * reordering of Sec. 6).  Traffic is the bytes each shard sends plus
 * receives, in units of its own share of the state.
 */
typedef struct qs_reorder_info {
  int32_t remaps;            /* reorderings inserted before gates */
  int32_t swaps;             /* upper/local qubit swaps they make in total */
  int32_t restore_swaps;     /* upper positions the final reordering (back to
                                the caller's order) refills; 0 = none needed */
  int32_t global_gates;      /* non-diagonal gates whose target is an upper
                                qubit in the caller's order: one pairwise
                                exchange each in Sec. 3.2's scheme */
  double traffic_reordered;  /* all reorderings, the final one included: a
                                reordering of k swaps keeps 2^-k of each
                                shard's amplitudes, 2 (1 - 2^-k) */
  double traffic_pairwise;   /* the pairwise exchanges as Table 2 counts them:
                                2 per global gate (cases 2 and 6), 1 if its
                                control is local (case 5) */
} qs_reorder_info;

/*
 * Plan the reordering of a gate list (host only, no GPU needed).  A
 * non-diagonal gate whose target sits at an upper position triggers one
 * reordering that swaps it in, with every other upper qubit needed before
 * the local qubit it would displace; diagonal gates and controls never need
 * one.  Running, for r = 0, 1, ..., the gates out_ops[remap_at[r-1] ..
 * remap_at[r]) (from 0 for r = 0) followed by qs_permute_qubits(remap_perm +
 * r * n), then the remaining gates and qs_permute_qubits(final_perm), equals
 * qs_run of the original list.
 *   nlocal      1 .. n: qubits below it are local to a shard
 *   theta       as for qs_run (needed only to validate rotations)
 *   info        host, may be NULL
 *   out_ops     host, nops records or NULL: the gates with target and control
 *               replaced by their positions at that point; if NULL only info
 *               is filled and the arrays below are not touched
 *   remap_at    host, cap int32: the gate each reordering precedes
 *   remap_perm  host, cap * n int32: the reorderings
 *   cap         capacity of remap_at / remap_perm in reorderings
 *   final_perm  host, n int32: the reordering back to the caller's order
 * Errors: QS_EINVAL (bad arguments or op list), QS_ERANGE (cap smaller than
 * info->remaps; info is still filled).
 */
int qs_plan_reorder(int n, int nlocal, const qs_op* ops, int nops, const double* theta,
                    int nparams, qs_reorder_info* info, qs_op* out_ops, int32_t* remap_at,
                    int32_t* remap_perm, int cap, int32_t* final_perm);

/*
 * qs_run through a reordering plan: the gates between reorderings run as
 * qs_run runs them (flags as there), the reorderings as qs_permute_qubits,
 * and the state ends in the caller's qubit order, equal to qs_run's result
 * up to floating-point rounding.  This is how one shard's share of a split
 * state would be processed on one GPU; info (host, may be NULL) receives
 * the plan's counts.
 */
int qs_run_reordered(qs_state* s, int nlocal, const qs_op* ops, int nops, const double* theta,
                     int nparams, int flags, qs_reorder_info* info);

/*
 * Measurement probabilities of the state (not part of the paper; the
 * per-qubit marginals of |alpha_i|^2):
 *   p1     host, n doubles or NULL: p1[k] = sum over i with bit k set of |alpha_i|^2
 *   norm2  host, 1 double or NULL: sum of all |alpha_i|^2
 *   full   dev, 2^n doubles or NULL: full[i] = |alpha_i|^2; device memory
 *          of the state's GPU (QS_EINVAL otherwise)
 *   full_bytes  size of `full` (QS_ERANGE if smaller than 2^n doubles)
 * Sums are double, accumulated in a fixed order (bitwise reproducible run to
 * run).  Synchronises the stream when p1 or norm2 is given.
 */
int qs_probabilities(qs_state* s, double* p1, double* norm2, void* full,
                     size_t full_bytes);

/*
 * qs_probabilities for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and the same fixed-order sums, so the values equal those of
 * qs_probabilities bit for bit, but nothing is allocated -- no hipMalloc,
 * hipFree or pinned host buffer -- and nothing is copied to the host.
 *   p1_dev     dev, n doubles or NULL: P(bit k = 1) as for qs_probabilities
 *   norm2_dev  dev, 1 double or NULL: sum of all |alpha_i|^2
 *   full, full_bytes  as for qs_probabilities
 * Every output is device memory of the state's GPU (QS_EINVAL otherwise),
 * 8-byte aligned.  Fully asynchronous on the state's stream; the results are
 * valid once that stream reaches this point.
 * Scratch: the partial sums live in one fixed device array of
 * QS_NOALLOC_SCRATCH_BYTES per GPU, set up on the first call on that GPU and
 * held until the process ends.  All calls on one GPU share it, so calls that
 * can overlap in time on one GPU (different streams or host threads) race;
 * calls queued on one stream are ordered and safe.  Every partial a call
 * reads it writes first, so nothing needs clearing between calls.  A state
 * whose partials would not fit gets QS_ERANGE (no state of n <= 34 does).
 * Errors: QS_EINVAL, QS_ERANGE, QS_ENODEV, QS_EHIP.
 */
#define QS_NOALLOC_SCRATCH_BYTES ((size_t)2048 * 35 * 8 + 35 * 8) /* 573,720 bytes */
int qs_probabilities_noalloc(qs_state* s, double* p1_dev, double* norm2_dev, void* full,
                             size_t full_bytes);

/*
 * Expectation value <psi|H|psi> of H = sum_j coeff[j] P_j, P_j the Pauli
 * string (x[j], z[j]) (not part of the paper).  The result is not divided
 * by the norm.  x, z, coeff: host arrays of nterms (nterms >= 0; every mask
 * must lie within the n qubits).  out: host, 1 double.  Synchronises.
 */
int qs_expect_pauli(qs_state* s, int nterms, const uint64_t* x,
                    const uint64_t* z, const double* coeff, double* out);

/*
 * dst = H src for H = sum_j coeff[j] P_j (both states of the same n and
 * dtype, distinct memory).  Asynchronous.
 */
int qs_apply_pauli_sum(qs_state* src, qs_state* dst, int nterms,
                       const uint64_t* x, const uint64_t* z,
                       const double* coeff);

/*
 * Energy and gradient of E(theta) = <psi(theta)|H|psi(theta)>, psi(theta)
 * = U_N ... U_1 |psi_0>, by the adjoint method (one reverse sweep over two
 * state vectors; Jones & Gacon, arXiv:2009.02823).  Not part of the paper.
 *   s       on entry psi_0 (or psi(theta), see flags); the forward sweep takes
 *           it to psi(theta) and the reverse sweep takes it back, so on
 *           return it holds psi_0 (up to rounding)
 *   ops, nops, theta, nparams   the circuit as for qs_run; rotations carry
 *           the parameters, every other gate is fixed
 *   nterms, x, z, coeff         H as for qs_expect_pauli
 *   lambda  second state (same n, dtype), used as workspace; overwritten
 *   flags   QS_ADJ_* bits: with QS_ADJ_STATE_IS_FINAL the state already
 *           holds psi(theta) (e.g. left by qs_run) and the forward sweep is
 *           skipped; QS_ADJ_WIDE_TILES plans both sweeps on wide tiles
 *   energy  host, 1 double (may be NULL)
 *   grad    host, nparams doubles (dE/dtheta[p], summed over every rotation
 *           that uses parameter p)
 * The gradient is accumulated in double precision for both dtypes, in a
 * fixed order.  Synchronises.
 */
#define QS_ADJ_STATE_IS_FINAL 1
/* fused forward and reverse passes on wide tiles (as QS_RUN_WIDE_TILES):
 * fewer passes, each at a lower fraction of peak bandwidth */
#define QS_ADJ_WIDE_TILES 2
int qs_grad_adjoint(qs_state* s, const qs_op* ops, int nops,
                    const double* theta, int nparams, int nterms,
                    const uint64_t* x, const uint64_t* z, const double* coeff,
                    qs_state* lambda, int flags, double* energy, double* grad);

/*
 * How qs_run would execute a gate list on an n-qubit state of `dtype`
 * (no GPU work; host only).  The planner groups gates into passes over the
 * state -- the GPU form of cache blocking by gate fusion, Sec. 4.4 -- and
 * this reports the result:
 *   info     host, filled with the counts below (may be NULL)
 *   order    host, nops int32 or NULL: gate indices in execution order
 *            (gates only move past gates they commute with)
 *   pass_of  host, nops int32 or NULL: the pass that applies each gate
 *   flags    QS_RUN_NO_FUSION, QS_RUN_WIDE_TILES, or QS_PLAN_ADJOINT_REVERSE
 * hbm_bytes counts algorithmic HBM traffic as Table 2 does: a pass that
 * rewrites the state moves 2 * 2^n * b bytes, a controlled gate run alone
 * 2^n * b (b = bytes per amplitude).
 */
/* Plan the reverse sweep of qs_grad_adjoint instead (the list reversed, each
 * gate replaced by its inverse, one gradient slot per rotation; with
 * QS_RUN_WIDE_TILES as under QS_ADJ_WIDE_TILES): every pass moves psi and
 * lambda, 4 * 2^n * b bytes; order and pass_of index the reversed list
 * (entry j is input gate nops - 1 - j).  Not with QS_RUN_NO_FUSION. */
#define QS_PLAN_ADJOINT_REVERSE 16
typedef struct qs_plan_info {
  int32_t passes;       /* passes over the state in total */
  int32_t fused;        /* passes applying several gates in one round trip */
  int32_t single_1q;    /* single-qubit gates run as their own pass */
  int32_t single_cu;    /* controlled gates run as their own pass */
  int32_t remaps;       /* on-chip register remaps inside fused passes */
  int32_t fused_ops;    /* op records run by fused passes (merged gates + remaps) */
  double hbm_bytes;     /* algorithmic HBM bytes of the whole list */
} qs_plan_info;
int qs_plan(int n, int dtype, const qs_op* ops, int nops, const double* theta,
            int nparams, int flags, qs_plan_info* info, int32_t* order,
            int32_t* pass_of);

/*
 * Batched energy and adjoint gradient of many independent small circuits in
 * one persistent launch.  Batching is not part of the paper; every circuit
 * computes exactly what qs_grad_adjoint computes for it: the gates of
 * Eq. (2) / Eq. (3) from |0...0>, E = <psi|H|psi> for its Pauli sum, and
 * dE/dtheta by one reverse sweep.
 *
 * qs_batch_create(dtype, ncircuits, n, op_off, ops, par_off, theta,
 *                 term_off, x, z, coeff, stream, out)
 *   Circuit c (0 <= c < ncircuits) has
 *     n[c] qubits, 1 <= n[c] <= QS_BATCH_MAX_QUBITS;
 *     gates ops[op_off[c] .. op_off[c+1]) (qs_op records as for qs_run;
 *       a rotation's param indexes the circuit's own parameters);
 *     parameters theta[par_off[c] .. par_off[c+1]);
 *     observable terms x, z, coeff[term_off[c] .. term_off[c+1]) (masks
 *       below 2^n[c], as for qs_expect_pauli).
 *   op_off, par_off, term_off: host int64 arrays of ncircuits + 1
 *   non-decreasing entries starting at 0.  All arrays are host memory and
 *   are copied: the caller may free them on return.  dtype: QS_C64 or
 *   QS_C128, the amplitude type of every circuit (energies and gradients
 *   are accumulated in double precision either way).  stream: the HIP
 *   stream all later work of the batch is queued on (NULL = default).
 *   *out receives the handle; the batch owns its device memory (the
 *   description, a workspace sized at the first run, the outputs).
 *   Errors: QS_EINVAL (NULL array, bad offsets, an invalid gate, control,
 *   parameter index or Pauli mask; the message names the circuit),
 *   QS_ERANGE (n[c] out of range), QS_ENOMEM, QS_ENODEV, QS_EHIP.
 *
 * qs_batch_run(b, tuning, energy, grad)
 *   Runs every circuit once.  energy: host, ncircuits doubles, energy[c] =
 *   E of circuit c (or NULL).  grad: host, par_off[ncircuits] doubles,
 *   grad[par_off[c] + p] = dE_c/dtheta_p, summed over the rotations that
 *   share parameter p (or NULL).  tuning: NULL for the defaults, or the
 *   launch shape (qs_batch_tuning); results do not depend on it beyond
 *   floating-point rounding, and for a fixed tuning they are bitwise
 *   reproducible.  Synchronises the batch's stream before returning.
 *   Calls on one batch from several host threads race.
 *   Errors: QS_EINVAL (NULL batch, tuning out of range), QS_ENOMEM
 *   (workspace), QS_EHIP.
 *
 * qs_batch_destroy(b): waits for the batch's stream, frees everything;
 * NULL is a no-op.
 */
#define QS_BATCH_MAX_QUBITS 24
typedef struct qs_batch qs_batch;
typedef struct qs_batch_tuning {
  int32_t threads;     /* threads per workgroup: 256 or 512 (0 = 256) */
  int32_t lds_bits;    /* C: log2 of the amplitudes per LDS chunk; states of
                          n <= C qubits stay in LDS, with 2 * 2^C amplitudes
                          <= 128 KiB (0 = 11) */
  int32_t khigh;       /* K: chunk qubits above the C - K lowest, chosen per
                          gate segment: 2 .. min(8, C - 6)
                          (0 = min(5, C - 6)) */
  int32_t wg_per_cu;   /* persistent workgroups per compute unit: 1..8 (0 = 2) */
  int32_t order;       /* 0 = longest circuit first, 1 = input order */
} qs_batch_tuning;
int qs_batch_create(int dtype, int ncircuits, const int32_t* n, const int64_t* op_off,
                    const qs_op* ops, const int64_t* par_off, const double* theta,
                    const int64_t* term_off, const uint64_t* x, const uint64_t* z,
                    const double* coeff, void* stream, qs_batch** out);
int qs_batch_run(qs_batch* b, const qs_batch_tuning* tuning, double* energy, double* grad);
int qs_batch_destroy(qs_batch* b);

/*
 * STREAM copy, dst[i] = src[i]: the sustainable-bandwidth probe that the
 * paper's lower bounds are stated against (Sec. 5.2, B_mem "measured by
 * STREAM Copy").  src, dst: device memory of the current device, 16-byte
 * aligned, non-overlapping; bytes: a multiple of 16.  Asynchronous on
 * `stream`.
 * Errors: QS_EINVAL (NULL, misaligned, bytes % 16 != 0, not device memory),
 * QS_ERANGE (an allocation smaller than bytes), QS_ENODEV.
 */
int qs_stream_copy(const void* src, void* dst, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* QS_H_ */
