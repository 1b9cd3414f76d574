// qs_batch.hip -- energy and adjoint gradient of many small circuits in one
// persistent launch.
//
// A grid of a few workgroups per CU pulls circuits from an atomic work
// queue (longest first by default, so the largest circuits do not finish
// last).  One workgroup runs one circuit at a time, start to end:
//   1. psi = |0...0>, then the gates (Eq. 2 / Eq. 3);
//   2. lambda = H psi and E = Re <psi|lambda>;
//   3. the adjoint reverse sweep: for each gate from the last, a rotation
//      adds Im<lambda|P|psi> to its gradient, then U^dagger goes to psi and
//      lambda.
// A state of at most 2^C amplitudes (C = lds_bits) lives in LDS for the
// whole circuit.  A larger one lives in the workgroup's slot of a global
// workspace and is processed in segments: a segment is a set of gates whose
// qubits all lie in one set of C qubits (the C - K lowest plus K chosen
// higher ones); the state is gathered 2^C amplitudes at a time into LDS,
// every gate of the segment is applied there, and the chunk is written
// back.  This is the paper's cache blocking (Sec. 4.4) with LDS as the
// cache and a per-segment choice of the blocked qubits.  The host builds the
// segments greedily and may move a gate ahead of earlier gates it commutes
// with (every shared qubit acted on diagonally by both), which changes
// neither the state nor, since commuting rotations keep their own
// generator, the gradient.
//
// Inside a segment (or a whole LDS-resident state) the gates are grouped
// into register blocks: consecutive gates (again allowing moves past
// commuting gates) whose qubits fit in one set of three.  Each thread loads
// the 8 amplitudes of its 3-qubit sub-cube from LDS into registers, applies
// every gate of the block there, and stores them back: one LDS round trip
// and one barrier per block instead of per gate.  A gate's body is
// specialised at compile time for its (target, control) register bits.
//
// Gradient contributions are double precision: each wavefront reduces its
// lanes by butterfly and adds the result to its own slot of the rotation's
// row in the workspace with a no-return atomic (only that wave's first lane
// touches the slot, so the adds apply in program order); at the end of the
// circuit the workgroup adds the wave slots in a fixed order.  Results are
// bitwise reproducible.
#include <string.h>

#include <algorithm>
#include <memory>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "qs_device.h"
#include "qs_internal.h"

namespace qs {

// Device description of one circuit.
struct BCirc {
  int32_t n, nops, nseg, ngroups;
  int32_t nrot, nblk;
  int64_t rec_off, seg_off, grp_off, rot_off, blk_off;
};
// Matrix forms with cheaper register updates than a general complex 2x2
// (the conjugate transpose of each form has the same form).
enum BForm : uint8_t {
  kFormGen = 0,   // general complex
  kFormReal = 1,  // real entries (RY, H, X)
  kFormDiag = 2,  // diagonal (RZ, phases)
  kFormSwap = 3,  // exactly X under a control (CNOT): a register exchange
};
// One gate in execution order: generator kind, target and control as bits
// of its register block (0..2; control 0xFF: none), matrix form, the
// rotation's ordinal in its circuit (-1: not a rotation) and the matrix
// applied in the forward sweep.
struct BRec {
  uint8_t kind, rt, rc, form;
  int32_t rot;
  int32_t pad2[2];
  double m[8];
};
static_assert(sizeof(BRec) == 80, "gate record layout");
// Register block: gate records [first, first + count) of its circuit, and
// the three LDS-resident bit positions q[0] < q[1] < q[2] held by register
// bits 0, 1, 2.
struct BBlk {
  int32_t first, count;
  uint8_t q[4];
  int32_t pad;
};
static_assert(sizeof(BBlk) == 16, "block record layout");
// Segment: blocks [first, first + count) of its circuit; hpos: the K higher
// qubits (ascending) held by chunk bits C - K .. C - 1.
struct BSeg {
  int32_t first, count;
  uint8_t hpos[8];
};

constexpr int kBatchMaxHigh = 8;

struct BatchDev {
  const BCirc* circ;
  const BRec* recs;
  const BBlk* blks;
  const BSeg* segs;
  const PauliGroup* groups;
  const PauliTerm* terms;   // PauliGroup::first is global into this array
  const int32_t* order;     // circuit of each queue position
  double* energy;
  double* grad_rot;         // one entry per rotation; circuit c's at rot_off
  unsigned int* counter;
  char* ws;                 // per-workgroup slots
  uint64_t ws_slot_bytes;
  uint64_t state_units;     // amplitudes per state in a slot
  int32_t ncirc;
  int32_t lds_bits;         // C
  int32_t khigh;            // K
  int32_t pad;
};

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Copy of *p read through the constant address space: with a uniform p the
// compiler uses scalar loads and keeps the fields in scalar registers (a
// plain load may not, since the kernel writes global memory).  Only for the
// schedule tables, which nothing writes while the kernel runs.
template <typename X>
__device__ __forceinline__ X ldc(const X* p) {
  static_assert(sizeof(X) % 4 == 0, "word-sized table entries");
  typedef const __attribute__((address_space(4))) uint32_t cword;
  uint32_t w[sizeof(X) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(X) / 4); ++i) w[i] = ((cword*)p)[i];
  X v;
  __builtin_memcpy(&v, w, sizeof(X));
  return v;
}

__device__ __forceinline__ uint32_t ins0(uint32_t p, int k) {
  const uint32_t lo = p & ((1u << k) - 1u);
  return ((p ^ lo) << 1) | lo;
}

// LDS slot of amplitude index j: the higher chunks of j XOR-folded into its
// low chunk (3 bits for 16-byte, 4 bits for 8-byte amplitudes), so that the
// lanes of a wave reach distinct banks whatever bits a register block
// strides over.  The map is XOR-linear, so the slot of (a | b) for disjoint
// a and b is slot(a) ^ slot(b), and a bijection on every [0, 2^m).
template <typename T>
struct Swz;
template <>
struct Swz<d2> {
  static __device__ __forceinline__ uint32_t f(uint32_t j) {
    return j ^ (((j >> 3) ^ (j >> 6) ^ (j >> 9) ^ (j >> 12)) & 7u);
  }
};
template <>
struct Swz<f2> {
  static __device__ __forceinline__ uint32_t f(uint32_t j) {
    return j ^ (((j >> 4) ^ (j >> 8) ^ (j >> 12)) & 15u);
  }
};
// Identity map, for states in global memory.
struct NoSwz {
  static __device__ __forceinline__ uint32_t f(uint32_t j) { return j; }
};
// The record's matrix, or its conjugate transpose, in compute precision.
template <typename R>
__device__ __forceinline__ void rec_mat(const BRec& r, bool dag, Mat<R>& q) {
  if (!dag) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      q.r[e] = (R)r.m[2 * e];
      q.i[e] = (R)r.m[2 * e + 1];
    }
  } else {
    q.r[0] = (R)r.m[0]; q.i[0] = -(R)r.m[1];
    q.r[1] = (R)r.m[4]; q.i[1] = -(R)r.m[5];
    q.r[2] = (R)r.m[2]; q.i[2] = -(R)r.m[3];
    q.r[3] = (R)r.m[6]; q.i[3] = -(R)r.m[7];
  }
}

// Gate on register bit K of an 8-amplitude register block.  With a control
// on register bit rc (>= 0) the pairs whose control bit is 0 take the
// identity; rc is uniform, so the coefficients are chosen with scalar
// selects and every pair runs the same arithmetic.
template <int K, typename T, typename R>
__device__ __forceinline__ void blk_gate(T* x, const Mat<R>& q, int rc) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if (r & (1 << K)) continue;
    const bool on = rc < 0 || ((r >> rc) & 1);
    Mat<R> u;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const R id = (e == 0 || e == 3) ? (R)1 : (R)0;
      u.r[e] = on ? q.r[e] : id;
      u.i[e] = on ? q.i[e] : (R)0;
    }
    pair_apply(u, x[r], x[r | (1 << K)]);
  }
}
// Uncontrolled forms on register bit K.
template <int K, typename T, typename R>
__device__ __forceinline__ void blk_gen(T* x, const Mat<R>& q) {
#pragma unroll
  for (int r = 0; r < 8; ++r)
    if (!(r & (1 << K))) pair_apply(q, x[r], x[r | (1 << K)]);
}
template <int K, typename T, typename R>
__device__ __forceinline__ void blk_real(T* x, const Mat<R>& q) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if (r & (1 << K)) continue;
    T& u = x[r];
    T& v = x[r | (1 << K)];
    const R ur = u.x, ui = u.y, vr = v.x, vi = v.y;
    u = T{q.r[0] * ur + q.r[1] * vr, q.r[0] * ui + q.r[1] * vi};
    v = T{q.r[2] * ur + q.r[3] * vr, q.r[2] * ui + q.r[3] * vi};
  }
}
template <int K, typename T, typename R>
__device__ __forceinline__ void blk_diag(T* x, const Mat<R>& q) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int e = (r >> K) & 1 ? 3 : 0;
    const R ar = x[r].x, ai = x[r].y;
    x[r] = T{q.r[e] * ar - q.i[e] * ai, q.r[e] * ai + q.i[e] * ar};
  }
}
// Controlled X: exchange the pairs whose control bit CR is 1.
template <int K, int CR, typename T>
__device__ __forceinline__ void blk_swap(T* x) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if ((r & (1 << K)) || !((r >> CR) & 1)) continue;
    const T t = x[r];
    x[r] = x[r | (1 << K)];
    x[r | (1 << K)] = t;
  }
}

// Dispatch on the uniform form, target bit and control bit.  Each branch
// ends in a distinct empty asm statement: otherwise the optimiser merges
// similar bodies into one with a runtime register index, which puts the
// block in scratch memory.
#define QS_BLK(tag, call) \
  {                       \
    call;                 \
    asm volatile("; blk " tag); \
  }
template <typename T, typename R>
__device__ __forceinline__ void blk_gate_any(T* x, const Mat<R>& q, int rt, int rc, int form) {
  if (rc < 0) {
    if (form == kFormReal) {
      if (rt == 0) QS_BLK("r0", (blk_real<0>(x, q)))
      else if (rt == 1) QS_BLK("r1", (blk_real<1>(x, q)))
      else QS_BLK("r2", (blk_real<2>(x, q)))
    } else if (form == kFormDiag) {
      if (rt == 0) QS_BLK("d0", (blk_diag<0>(x, q)))
      else if (rt == 1) QS_BLK("d1", (blk_diag<1>(x, q)))
      else QS_BLK("d2", (blk_diag<2>(x, q)))
    } else {
      if (rt == 0) QS_BLK("u0", (blk_gen<0>(x, q)))
      else if (rt == 1) QS_BLK("u1", (blk_gen<1>(x, q)))
      else QS_BLK("u2", (blk_gen<2>(x, q)))
    }
  } else if (form == kFormSwap) {
    switch (rt * 4 + rc) {
      case 1: QS_BLK("s01", (blk_swap<0, 1>(x))) break;
      case 2: QS_BLK("s02", (blk_swap<0, 2>(x))) break;
      case 4: QS_BLK("s10", (blk_swap<1, 0>(x))) break;
      case 6: QS_BLK("s12", (blk_swap<1, 2>(x))) break;
      case 8: QS_BLK("s20", (blk_swap<2, 0>(x))) break;
      default: QS_BLK("s21", (blk_swap<2, 1>(x))) break;
    }
  } else {
    if (rt == 0) QS_BLK("c0", (blk_gate<0>(x, q, rc)))
    else if (rt == 1) QS_BLK("c1", (blk_gate<1>(x, q, rc)))
    else QS_BLK("c2", (blk_gate<2>(x, q, rc)))
  }
}
// This thread's share of Im<lambda|P|psi> over the pairs of register bit K
// for P = X (1), Y (2) or Z (3).
template <int K, int P, typename T>
__device__ __forceinline__ double blk_grad(const T* x, const T* y) {
  double g = 0.0;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if (r & (1 << K)) continue;
    const int r1 = r | (1 << K);
    const double a0r = x[r].x, a0i = x[r].y, a1r = x[r1].x, a1i = x[r1].y;
    const double l0r = y[r].x, l0i = y[r].y, l1r = y[r1].x, l1i = y[r1].y;
    // X psi = (a1, a0); Y psi = (-i a1, i a0); Z psi = (a0, -a1)
    if (P == 1) g += im_conj_mul(l0r, l0i, a1r, a1i) + im_conj_mul(l1r, l1i, a0r, a0i);
    if (P == 2) g += im_conj_mul(l0r, l0i, a1i, -a1r) + im_conj_mul(l1r, l1i, -a0i, a0r);
    if (P == 3) g += im_conj_mul(l0r, l0i, a0r, a0i) - im_conj_mul(l1r, l1i, a1r, a1i);
  }
  return g;
}
// Wave total of a gradient partial with DPP moves only (no LDS crossbar):
// row sums (row mirror, half-row mirror, two quad permutations), then the
// last lane of rows 0 and 2 added into rows 1 and 3, and the last lane of
// row 1 into rows 2 and 3.  Lane 63 ends with the total, added in a fixed
// order; rows left out of a step take 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ __forceinline__ double wave_total_last_lane(double v) {
  v += dpp_f64<0x140, 0xF>(v);  // row_mirror
  v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_f64<0x1B, 0xF>(v);   // quad_perm [3, 2, 1, 0]
  v += dpp_f64<0xB1, 0xF>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_f64<0x142, 0xA>(v);  // row_bcast15 into rows 1 and 3
  v += dpp_f64<0x143, 0xC>(v);  // row_bcast31 into rows 2 and 3
  return v;
}

template <typename T>
__device__ __forceinline__ double blk_grad_any(const T* x, const T* y, int pauli, int rt) {
  double g;
  if (pauli == 1) {
    if (rt == 0) QS_BLK("gx0", (g = blk_grad<0, 1>(x, y)))
    else if (rt == 1) QS_BLK("gx1", (g = blk_grad<1, 1>(x, y)))
    else QS_BLK("gx2", (g = blk_grad<2, 1>(x, y)))
  } else if (pauli == 2) {
    if (rt == 0) QS_BLK("gy0", (g = blk_grad<0, 2>(x, y)))
    else if (rt == 1) QS_BLK("gy1", (g = blk_grad<1, 2>(x, y)))
    else QS_BLK("gy2", (g = blk_grad<2, 2>(x, y)))
  } else {
    if (rt == 0) QS_BLK("gz0", (g = blk_grad<0, 3>(x, y)))
    else if (rt == 1) QS_BLK("gz1", (g = blk_grad<1, 3>(x, y)))
    else QS_BLK("gz2", (g = blk_grad<2, 3>(x, y)))
  }
  return g;
}
#undef QS_BLK

// One register block on a 2^m-amplitude LDS array (psi; lambda too in the
// reverse sweep, REV).  Every thread takes 3-qubit sub-cubes in turn; the
// loop's trip count is uniform, so wave reductions see every lane.
template <typename R, typename T, int B, bool REV>
__device__ __forceinline__ void run_block(T* a, T* l, int m, const BBlk& bk, const BRec* recs,
                                          double* gacc, int wave, int lane) {
  constexpr int NW = B / 64;
  const int q0 = bk.q[0], q1 = bk.q[1], q2 = bk.q[2];
  uint32_t off[8];  // LDS slots of the register offsets (uniform)
#pragma unroll
  for (int r = 0; r < 8; ++r)
    off[r] = Swz<T>::f(((uint32_t)(r & 1) << q0) | ((uint32_t)((r >> 1) & 1) << q1) |
                       ((uint32_t)((r >> 2) & 1) << q2));
  const uint32_t nsub = 1u << (m - 3);
  for (uint32_t s0 = 0; s0 < nsub; s0 += B) {
    const uint32_t sub = s0 + threadIdx.x;
    const bool act = sub < nsub;
    const uint32_t base = Swz<T>::f(ins0(ins0(ins0(sub, q0), q1), q2));
    T x[8], y[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      x[r] = act ? a[base ^ off[r]] : make_amp<T>(0.0, 0.0);
      if constexpr (REV) y[r] = act ? l[base ^ off[r]] : make_amp<T>(0.0, 0.0);
    }
    for (int k = 0; k < bk.count; ++k) {
      const int gi = uni(REV ? bk.first + bk.count - 1 - k : bk.first + k);
      const BRec rec = ldc(recs + gi);
      const int rt = rec.rt, rc = rec.rc == 0xFF ? -1 : (int)rec.rc;
      Mat<R> q;
      rec_mat<R>(rec, REV, q);
      if constexpr (REV) {
        if (rec.rot >= 0) {
          const double g = wave_total_last_lane(blk_grad_any(x, y, rec.kind - QS_OP_RX + 1, rt));
          // no-return atomic: the wave does not wait for the update; one lane
          // of one wave owns the slot, so the adds land in program order
          if (lane == 63) atomicAdd(&gacc[rec.rot * NW + wave], g);
        }
        blk_gate_any(y, q, rt, rc, rec.form);
      }
      blk_gate_any(x, q, rt, rc, rec.form);
    }
    if (act) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        a[base ^ off[r]] = x[r];
        if constexpr (REV) l[base ^ off[r]] = y[r];
      }
    }
  }
}

// Global index of chunk element k: low bits of k in place, chunk bits
// C - K .. C - 1 at hpos, plus the chunk's base.
__device__ __forceinline__ uint32_t chunk_index(uint32_t k, uint32_t base, int low, int K,
                                                const int* hp) {
  uint32_t g = base | (k & ((1u << low) - 1u));
  const uint32_t kh = k >> low;
#pragma unroll
  for (int j = 0; j < kBatchMaxHigh; ++j)
    if (j < K) g |= ((kh >> j) & 1u) << hp[j];
  return g;
}
// Base index of chunk ch: the bits of ch go, in ascending order, to the
// qubits >= low that are not among hpos.
__device__ __forceinline__ uint32_t chunk_base(uint32_t ch, int low, int K, const int* hp) {
  uint32_t g = ch << low;
#pragma unroll
  for (int j = 0; j < kBatchMaxHigh; ++j)
    if (j < K) g = ins0(g, hp[j]);
  return g;
}

// Chunk transfer between the workspace and LDS for NA arrays (psi; psi and
// lambda): optionally write the LDS contents back to the chunk at obase,
// then optionally load the chunk at nbase.  Every thread touches only its
// own LDS slots, so the write-back and the load need no barrier between
// them; the loads are issued first so that their latency overlaps the
// write-back.
template <typename T, int B, int NA>
__device__ __forceinline__ void xfer(T* const* lds, T* const* ws, uint32_t M, bool wb,
                                     uint32_t obase, bool ld, uint32_t nbase, int low, int K,
                                     const int* hp) {
  constexpr int UG = NA == 1 ? 8 : 4;
  for (uint32_t k0 = threadIdx.x; k0 < M; k0 += UG * B) {
    T v[NA][UG];
    if (ld) {
#pragma unroll
      for (int u = 0; u < UG; ++u) {
        const uint32_t k = k0 + u * B;
        if (k < M) {
          const uint32_t g = chunk_index(k, nbase, low, K, hp);
#pragma unroll
          for (int a = 0; a < NA; ++a) v[a][u] = ws[a][g];
        }
      }
    }
    if (wb) {
#pragma unroll
      for (int u = 0; u < UG; ++u) {
        const uint32_t k = k0 + u * B;
        if (k < M) {
          const uint32_t g = chunk_index(k, obase, low, K, hp);
#pragma unroll
          for (int a = 0; a < NA; ++a) ws[a][g] = lds[a][Swz<T>::f(k)];
        }
      }
    }
    if (ld) {
#pragma unroll
      for (int u = 0; u < UG; ++u) {
        const uint32_t k = k0 + u * B;
        if (k < M) {
#pragma unroll
          for (int a = 0; a < NA; ++a) lds[a][Swz<T>::f(k)] = v[a][u];
        }
      }
    }
  }
}

template <int B>
__device__ __forceinline__ double wg_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < B / 64; ++j) s += red[j];
  __syncthreads();
  return s;
}

// psi = |0...0> over 2^n amplitudes.
template <typename T, int B>
__device__ __forceinline__ void init_zero_state(T* psi, int n) {
  for (uint32_t i = threadIdx.x; i < (1u << n); i += B) psi[i] = make_amp<T>(i == 0 ? 1.0 : 0.0, 0.0);
}

// lambda = H psi over 2^n amplitudes (terms grouped by x mask); returns this
// thread's part of Re<psi|lambda>.
template <typename T, int B, typename S>
__device__ __forceinline__ double apply_h(const T* psi, T* lam, int n, const PauliGroup* groups,
                                          int ngroups, const PauliTerm* terms) {
  double e = 0.0;
  for (uint32_t i = threadIdx.x; i < (1u << n); i += B) {
    double hr = 0.0, hi = 0.0;
    for (int g = 0; g < ngroups; ++g) {
      const PauliGroup G = ldc(groups + g);
      const uint32_t k = i ^ (uint32_t)G.x;
      const T b = psi[S::f(k)];
      double wr = 0.0, wi = 0.0;
      for (int j = G.first; j < G.first + G.count; ++j) {
        const PauliTerm P = ldc(terms + j);
        const double sgn = (__popc(k & (uint32_t)P.z) & 1) ? -1.0 : 1.0;
        wr += sgn * P.cr;
        wi += sgn * P.ci;
      }
      hr += wr * (double)b.x - wi * (double)b.y;
      hi += wr * (double)b.y + wi * (double)b.x;
    }
    lam[S::f(i)] = make_amp<T>(hr, hi);
    const T a = psi[S::f(i)];
    e += (double)a.x * hr + (double)a.y * hi;
  }
  return e;
}

// Dynamic LDS: psi chunk [2^C], lambda chunk [2^C].
template <typename R, typename T, int B>
__global__ void __launch_bounds__(B) k_batch(BatchDev d) {
  extern __shared__ uint4 lds_raw[];
  __shared__ int s_idx;
  __shared__ double red[B / 64];
  constexpr int NW = B / 64;
  const int C = d.lds_bits, K = d.khigh, low = C - K;
  T* lpsi = (T*)lds_raw;
  T* llam = lpsi + (1u << C);
  T* wpsi = (T*)(d.ws + (uint64_t)blockIdx.x * d.ws_slot_bytes);
  T* wlam = wpsi + d.state_units;
  double* gacc = (double*)(wlam + d.state_units);  // [rotation][wave]
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;

  for (;;) {
    if (threadIdx.x == 0) s_idx = (int)atomicAdd(d.counter, 1u);
    __syncthreads();
    const int qi = uni(s_idx);
    __syncthreads();
    if (qi >= d.ncirc) break;
    const int ci = uni(d.order[qi]);
    const BCirc cc = ldc(d.circ + ci);
    const int n = cc.n;
    const bool whole = n <= C;
    // bits of the LDS-resident part; states below 3 qubits are padded with
    // zero amplitudes that no gate touches
    const int m = whole ? max(n, 3) : C;
    const uint32_t nch = whole ? 1u : 1u << (n - C);
    const uint32_t M = 1u << m;
    const BRec* recs = d.recs + cc.rec_off;
    const BBlk* blks = d.blks + cc.blk_off;
    const BSeg* segs = d.segs + cc.seg_off;

    // 1. |0...0>, gradient slots cleared, forward sweep
    if (whole) init_zero_state<T, B>(lpsi, m);
    else init_zero_state<T, B>(wpsi, n);
    for (int r = threadIdx.x; r < cc.nrot * NW; r += B) gacc[r] = 0.0;
    __syncthreads();
    T* const pa[2] = {lpsi, llam};
    T* const wa[2] = {wpsi, wlam};
    for (int sg = 0; sg < cc.nseg; ++sg) {
      const BSeg seg = ldc(segs + sg);
      int hp[kBatchMaxHigh];
#pragma unroll
      for (int j = 0; j < kBatchMaxHigh; ++j) hp[j] = seg.hpos[j];
      uint32_t prev = 0;
      for (uint32_t ch = 0; ch < nch; ++ch) {
        const uint32_t base = whole ? 0u : chunk_base(ch, low, K, hp);
        if (!whole) xfer<T, B, 1>(pa, wa, M, ch > 0, prev, true, base, low, K, hp);
        __syncthreads();
        for (int bi = seg.first; bi < seg.first + seg.count; ++bi) {
          const BBlk bk = ldc(blks + uni(bi));
          run_block<R, T, B, false>(lpsi, nullptr, m, bk, recs, gacc, wave, lane);
          __syncthreads();
        }
        prev = base;
      }
      if (!whole) {
        xfer<T, B, 1>(pa, wa, M, true, prev, false, 0u, low, K, hp);
        __syncthreads();
      }
    }

    // 2. lambda = H psi, E = Re<psi|lambda>
    double e;
    if (whole) {
      for (uint32_t i = (1u << n) + threadIdx.x; i < M; i += B)
        llam[Swz<T>::f(i)] = make_amp<T>(0.0, 0.0);
      e = apply_h<T, B, Swz<T>>(lpsi, llam, n, d.groups + cc.grp_off, cc.ngroups, d.terms);
    } else {
      e = apply_h<T, B, NoSwz>(wpsi, wlam, n, d.groups + cc.grp_off, cc.ngroups, d.terms);
    }
    e = wg_sum<B>(e, red);  // its barriers also publish lambda

    // 3. reverse sweep, segments and gates in reverse order
    for (int sg = cc.nseg - 1; sg >= 0; --sg) {
      const BSeg seg = ldc(segs + sg);
      int hp[kBatchMaxHigh];
#pragma unroll
      for (int j = 0; j < kBatchMaxHigh; ++j) hp[j] = seg.hpos[j];
      uint32_t prev = 0;
      for (uint32_t ch = 0; ch < nch; ++ch) {
        const uint32_t base = whole ? 0u : chunk_base(ch, low, K, hp);
        if (!whole) xfer<T, B, 2>(pa, wa, M, ch > 0, prev, true, base, low, K, hp);
        __syncthreads();
        for (int bi = seg.first + seg.count - 1; bi >= seg.first; --bi) {
          const BBlk bk = ldc(blks + uni(bi));
          run_block<R, T, B, true>(lpsi, llam, m, bk, recs, gacc, wave, lane);
          __syncthreads();
        }
        prev = base;
      }
      if (!whole) {
        xfer<T, B, 2>(pa, wa, M, true, prev, false, 0u, low, K, hp);
        __syncthreads();
      }
    }

    // 4. outputs; wave slots added in a fixed order (the workgroup barrier
    // after the last block orders the adds before these loads, which read the
    // device cache where the atomics were performed)
    for (int r = threadIdx.x; r < cc.nrot; r += B) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w)
        s += __hip_atomic_load(&gacc[r * NW + w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      d.grad_rot[cc.rot_off + r] = s;
    }
    if (threadIdx.x == 0) d.energy[ci] = e;
    __syncthreads();
  }
}

__global__ void k_batch_reset(unsigned int* counter) {
  if (threadIdx.x == 0) *counter = 0u;
}

// ----------------------------------------------------------------- host

namespace {

Status fail_st(int code, const std::string& msg) {
  Status s;
  s.code = code;
  s.msg = msg;
  return s;
}

struct HostOp {
  uint8_t kind, form;
  int8_t target, control;  // control -1: none
  uint32_t qmask;          // qubits acted on
  uint32_t dmask;          // qubits acted on diagonally (a control; a diagonal target)
  int32_t mat, rot, param;
};

}  // namespace

struct BatchImpl {
  int dtype = 0, ncirc = 0, nmax = 0, nrot_max = 0;
  hipStream_t stream = nullptr;
  int device = 0, cus = 0;
  // host description
  std::vector<int32_t> n;
  std::vector<int64_t> op_off, par_off, grp_off, rot_off;
  std::vector<int32_t> ngroups, nrot;
  std::vector<HostOp> ops;
  std::vector<double> mats;  // 8 doubles per matrix (fixed matrices shared)
  std::vector<double> cost;
  int64_t nrot_total = 0;
  // device: static part (Pauli tables, orders) and outputs
  void* stat = nullptr;
  const PauliGroup* groups_dev = nullptr;
  const PauliTerm* terms_dev = nullptr;
  const int32_t* order_dev = nullptr;  // [LPT order | input order]
  void* out = nullptr;                 // energy | grad_rot | counter
  // device: schedule for the current (C, K): circuits, gate records, segments
  void* sched = nullptr;
  size_t sched_bytes = 0;
  int sched_C = -1, sched_K = -1;
  const BCirc* circ_dev = nullptr;
  const BRec* recs_dev = nullptr;
  const BBlk* blks_dev = nullptr;
  const BSeg* segs_dev = nullptr;
  int64_t nseg_total = 0, nblk_total = 0;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  double* host_out = nullptr;
  size_t host_out_bytes = 0;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Scan limits of the segment and block builders: gates looked at past the
// first unplaced one, and gates left behind, per segment / block.
constexpr int kSegWindow = 512;
constexpr int kSegSkip = 96;
constexpr int kBlkWindow = 128;
constexpr int kBlkSkip = 24;

// Whether gate h may move ahead of every gate in `later` (each shared qubit
// acted on diagonally by both).
bool moves_past(const BatchImpl& b, int64_t o0, const HostOp& h, const std::vector<int>& later) {
  for (int x : later) {
    const HostOp& o = b.ops[o0 + x];
    if ((h.qmask & o.qmask) & ~(h.dmask & o.dmask)) return false;
  }
  return true;
}

// Split circuit c into segments for chunk size 2^C with K higher chunk
// qubits, and each segment into register blocks.  Appends the circuit's gate
// records (block order), its blocks (first = record index relative to the
// circuit's first record) and its segments (first = block index relative to
// the circuit's first block).
void segment_circuit(const BatchImpl& b, int c, int C, int K, std::vector<BRec>& recs,
                     std::vector<BBlk>& blks, std::vector<BSeg>& segs, int64_t rec0,
                     int64_t blk0) {
  const int n = b.n[c];
  const int64_t o0 = b.op_off[c];
  const int nops = (int)(b.op_off[c + 1] - o0);
  const bool whole = n <= C;
  const int low = whole ? n : C - K;
  const int m = whole ? std::max(n, 3) : C;  // bits of the LDS-resident part
  const uint32_t lowmask = (1u << low) - 1u;
  std::vector<char> used;
  std::vector<int> blk, later;
  auto emit = [&](const std::vector<int>& gates, std::vector<int>& hs) {
    BSeg s;
    memset(&s, 0, sizeof(s));
    s.first = (int32_t)((int64_t)blks.size() - blk0);
    if (!whole) {
      for (int q = low; q < n && (int)hs.size() < K; ++q)
        if (std::find(hs.begin(), hs.end(), q) == hs.end()) hs.push_back(q);
      std::sort(hs.begin(), hs.end());
      for (int j = 0; j < K; ++j) s.hpos[j] = (uint8_t)hs[j];
    }
    auto local = [&](int q) -> int {
      if (whole || q < low) return q;
      return low + (int)(std::find(hs.begin(), hs.end(), q) - hs.begin());
    };
    auto lmask = [&](const HostOp& h) -> uint32_t {
      uint32_t v = 1u << local(h.target);
      if (h.control >= 0) v |= 1u << local(h.control);
      return v;
    };
    // greedy register blocks over the segment's gate list
    const int ng = (int)gates.size();
    used.assign(ng, 0);
    int first = 0;
    while (first < ng) {
      blk.clear();
      later.clear();
      uint32_t set = 0;
      int scanned = 0;
      for (int i = first; i < ng && scanned < kBlkWindow; ++i) {
        if (used[i]) continue;
        ++scanned;
        const HostOp& h = b.ops[o0 + gates[i]];
        const uint32_t lm = lmask(h);
        if (__builtin_popcount(set | lm) <= 3 && moves_past(b, o0, h, later)) {
          set |= lm;
          blk.push_back(i);
          used[i] = 1;
          continue;
        }
        later.push_back(gates[i]);
        if ((int)later.size() > kBlkSkip) break;
      }
      // fill the register set to three bits from the top of the resident part
      for (int q = m - 1; q >= 0 && __builtin_popcount(set) < 3; --q) set |= 1u << q;
      BBlk bk;
      memset(&bk, 0, sizeof(bk));
      bk.first = (int32_t)((int64_t)recs.size() - rec0);
      bk.count = (int32_t)blk.size();
      int pos[32];
      int j = 0;
      for (int q = 0; q < m; ++q)
        if (set >> q & 1u) {
          pos[q] = j;
          bk.q[j++] = (uint8_t)q;
        }
      for (int i : blk) {
        const HostOp& h = b.ops[o0 + gates[i]];
        BRec r;
        memset(&r, 0, sizeof(r));
        r.kind = h.kind;
        r.form = h.form;
        r.rt = (uint8_t)pos[local(h.target)];
        r.rc = h.control < 0 ? (uint8_t)0xFF : (uint8_t)pos[local(h.control)];
        r.rot = h.rot;
        memcpy(r.m, &b.mats[(size_t)h.mat * 8], sizeof(r.m));
        recs.push_back(r);
      }
      blks.push_back(bk);
      while (first < ng && used[first]) ++first;
    }
    s.count = (int32_t)((int64_t)blks.size() - blk0 - s.first);
    segs.push_back(s);
  };
  if (whole) {
    std::vector<int> all(nops), none;
    for (int g = 0; g < nops; ++g) all[g] = g;
    if (nops) emit(all, none);
    return;
  }
  std::vector<char> placed(nops, 0);
  std::vector<int> gates, blocked;
  int first = 0;  // first unplaced gate
  while (first < nops) {
    gates.clear();
    blocked.clear();
    uint32_t hmask = 0;  // higher qubits taken by this segment
    int scanned = 0;
    for (int g = first; g < nops && scanned < kSegWindow; ++g) {
      if (placed[g]) continue;
      ++scanned;
      const HostOp& h = b.ops[o0 + g];
      const uint32_t need = h.qmask & ~lowmask;
      if (__builtin_popcount(hmask | need) <= K && moves_past(b, o0, h, blocked)) {
        hmask |= need;
        gates.push_back(g);
        placed[g] = 1;
        continue;
      }
      blocked.push_back(g);
      if ((int)blocked.size() > kSegSkip) break;
    }
    std::vector<int> hs;
    for (int q = low; q < n; ++q)
      if (hmask >> q & 1u) hs.push_back(q);
    emit(gates, hs);
    while (first < nops && placed[first]) ++first;
  }
}

}  // namespace

// Build and upload the schedule (circuits, gate records, register blocks,
// segments) for (C, K).
static Status build_schedule(BatchImpl* b, int C, int K) {
  if (b->sched_C == C && b->sched_K == K) return Status::ok();
  std::vector<BCirc> circ(b->ncirc);
  std::vector<BRec> recs;
  std::vector<BBlk> blks;
  std::vector<BSeg> segs;
  recs.reserve(b->ops.size());
  for (int c = 0; c < b->ncirc; ++c) {
    BCirc& cc = circ[c];
    memset(&cc, 0, sizeof(cc));
    cc.n = b->n[c];
    cc.nops = (int32_t)(b->op_off[c + 1] - b->op_off[c]);
    cc.ngroups = b->ngroups[c];
    cc.nrot = b->nrot[c];
    cc.rec_off = (int64_t)recs.size();
    cc.blk_off = (int64_t)blks.size();
    cc.grp_off = b->grp_off[c];
    cc.rot_off = b->rot_off[c];
    cc.seg_off = (int64_t)segs.size();
    const size_t seg0 = segs.size();
    segment_circuit(*b, c, C, K, recs, blks, segs, cc.rec_off, cc.blk_off);
    cc.nseg = (int32_t)(segs.size() - seg0);
    cc.nblk = (int32_t)((int64_t)blks.size() - cc.blk_off);
    // every gate exactly once; blocks tile the records and segments tile the
    // blocks; register sets inside the LDS-resident part
    if ((int64_t)recs.size() - cc.rec_off != cc.nops)
      return fail_st(QS_EHIP, "batch schedule: gate count mismatch (internal error)");
    const int m = cc.n <= C ? std::max(cc.n, 3) : C;
    int64_t next_rec = 0, next_blk = 0;
    for (size_t s = seg0; s < segs.size(); ++s) {
      if (segs[s].first != next_blk || segs[s].count < 1)
        return fail_st(QS_EHIP, "batch schedule: segment layout (internal error)");
      next_blk += segs[s].count;
    }
    if (next_blk != cc.nblk) return fail_st(QS_EHIP, "batch schedule: block count (internal error)");
    for (int64_t k = cc.blk_off; k < (int64_t)blks.size(); ++k) {
      const BBlk& bk = blks[k];
      if (bk.first != next_rec || bk.count < 1 || !(bk.q[0] < bk.q[1] && bk.q[1] < bk.q[2]) ||
          bk.q[2] >= m)
        return fail_st(QS_EHIP, "batch schedule: block layout (internal error)");
      next_rec += bk.count;
    }
    for (int64_t g = cc.rec_off; g < (int64_t)recs.size(); ++g)
      if (recs[g].rt > 2 || (recs[g].rc != 0xFF && recs[g].rc > 2) || recs[g].rt == recs[g].rc)
        return fail_st(QS_EHIP, "batch schedule: gate outside its block (internal error)");
  }
  const size_t o_circ = 0;
  const size_t o_recs = align256(o_circ + circ.size() * sizeof(BCirc));
  const size_t o_blks = align256(o_recs + std::max<size_t>(1, recs.size()) * sizeof(BRec));
  const size_t o_segs = align256(o_blks + std::max<size_t>(1, blks.size()) * sizeof(BBlk));
  const size_t total = align256(o_segs + std::max<size_t>(1, segs.size()) * sizeof(BSeg));
  std::vector<char> blob(total, 0);
  memcpy(blob.data() + o_circ, circ.data(), circ.size() * sizeof(BCirc));
  if (!recs.empty()) memcpy(blob.data() + o_recs, recs.data(), recs.size() * sizeof(BRec));
  if (!blks.empty()) memcpy(blob.data() + o_blks, blks.data(), blks.size() * sizeof(BBlk));
  if (!segs.empty()) memcpy(blob.data() + o_segs, segs.data(), segs.size() * sizeof(BSeg));
  Status st = hip_status(hipStreamSynchronize(b->stream), "batch sync");  // earlier runs may read it
  if (!st.good()) return st;
  if (b->sched_bytes < total) {
    if (b->sched) (void)hipFree(b->sched);
    b->sched = nullptr;
    b->sched_bytes = 0;
    b->sched_C = b->sched_K = -1;
    if (hipMalloc(&b->sched, total) != hipSuccess) {
      (void)hipGetLastError();
      return fail_st(QS_ENOMEM, "batch schedule allocation failed");
    }
    b->sched_bytes = total;
  }
  st = hip_status(hipMemcpy(b->sched, blob.data(), total, hipMemcpyHostToDevice),
                  "batch schedule upload");
  if (!st.good()) return st;
  char* a = (char*)b->sched;
  b->circ_dev = (const BCirc*)(a + o_circ);
  b->recs_dev = (const BRec*)(a + o_recs);
  b->blks_dev = (const BBlk*)(a + o_blks);
  b->segs_dev = (const BSeg*)(a + o_segs);
  b->nseg_total = (int64_t)segs.size();
  b->nblk_total = (int64_t)blks.size();
  b->sched_C = C;
  b->sched_K = K;
  return Status::ok();
}

// Whether a gate acts diagonally on its target for every parameter value.
static bool diag_target(const XGate& g) {
  if (g.param >= 0) return g.kind == QS_OP_RZ;
  return g.m[2] == 0.0 && g.m[3] == 0.0 && g.m[4] == 0.0 && g.m[5] == 0.0;
}

// Register-update form of a gate (the same for every parameter value).
static uint8_t gate_form(const XGate& g) {
  if (g.param >= 0) return g.kind == QS_OP_RY ? kFormReal : g.kind == QS_OP_RZ ? kFormDiag : kFormGen;
  const double* m = g.m;
  if (g.control >= 0) {
    const bool x = m[0] == 0.0 && m[1] == 0.0 && m[2] == 1.0 && m[3] == 0.0 && m[4] == 1.0 &&
                   m[5] == 0.0 && m[6] == 0.0 && m[7] == 0.0;
    return x ? kFormSwap : kFormGen;
  }
  if (diag_target(g)) return kFormDiag;
  if (m[1] == 0.0 && m[3] == 0.0 && m[5] == 0.0 && m[7] == 0.0) return kFormReal;
  return kFormGen;
}

Status batch_create(int dtype, int ncirc, const int32_t* n, const int64_t* op_off,
                    const qs_op* ops, const int64_t* par_off, const double* theta,
                    const int64_t* term_off, const uint64_t* x, const uint64_t* z,
                    const double* coeff, hipStream_t stream, BatchImpl** outp) {
  std::unique_ptr<BatchImpl> b(new (std::nothrow) BatchImpl());
  if (!b) return fail_st(QS_ENOMEM, "batch handle allocation failed");
  b->dtype = dtype;
  b->ncirc = ncirc;
  b->stream = stream;
  b->n.assign(n, n + ncirc);
  b->op_off.assign(op_off, op_off + ncirc + 1);
  b->par_off.assign(par_off, par_off + ncirc + 1);
  b->grp_off.resize(ncirc);
  b->rot_off.resize(ncirc);
  b->ngroups.resize(ncirc);
  b->nrot.resize(ncirc);
  b->ops.reserve((size_t)op_off[ncirc]);
  std::unordered_map<std::string, int32_t> fixed_index;  // identical fixed matrices shared
  std::vector<PauliGroup> groups;
  std::vector<PauliTerm> terms;
  std::vector<XGate> gx;
  int64_t rot_total = 0;
  for (int c = 0; c < ncirc; ++c) {
    const std::string who = "qs_batch_create: circuit " + std::to_string(c) + ": ";
    const int nc = n[c];
    if (nc < 1 || nc > QS_BATCH_MAX_QUBITS) return fail_st(QS_ERANGE, who + "n out of range");
    if (op_off[c + 1] < op_off[c] || par_off[c + 1] < par_off[c] || term_off[c + 1] < term_off[c])
      return fail_st(QS_EINVAL, who + "offsets decrease");
    if (op_off[c + 1] - op_off[c] > (1 << 30)) return fail_st(QS_ERANGE, who + "too many gates");
    const int np = (int)(par_off[c + 1] - par_off[c]);
    Status st = normalize_ops(nc, ops + op_off[c], (int)(op_off[c + 1] - op_off[c]),
                              np ? theta + par_off[c] : (const double*)nullptr, np, &gx);
    if (!st.good()) return fail_st(st.code, who + st.msg);
    b->rot_off[c] = rot_total;
    int nr = 0;
    for (const XGate& g : gx) {
      HostOp h;
      h.kind = (uint8_t)g.kind;
      h.form = gate_form(g);
      h.target = (int8_t)g.target;
      h.control = (int8_t)g.control;
      h.param = g.param;
      h.rot = g.param >= 0 ? nr++ : -1;
      h.qmask = 1u << g.target;
      h.dmask = diag_target(g) ? 1u << g.target : 0u;
      if (g.control >= 0) {
        h.qmask |= 1u << g.control;
        h.dmask |= 1u << g.control;
      }
      if (g.param >= 0) {
        h.mat = (int32_t)(b->mats.size() / 8);
        b->mats.insert(b->mats.end(), g.m, g.m + 8);
      } else {
        const std::string key((const char*)g.m, sizeof(g.m));
        auto it = fixed_index.find(key);
        if (it == fixed_index.end()) {
          it = fixed_index.emplace(key, (int32_t)(b->mats.size() / 8)).first;
          b->mats.insert(b->mats.end(), g.m, g.m + 8);
        }
        h.mat = it->second;
      }
      b->ops.push_back(h);
    }
    if (b->mats.size() / 8 > (size_t)INT32_MAX) return fail_st(QS_ERANGE, who + "too many gates");
    b->nrot[c] = nr;
    rot_total += nr;
    PauliTable t;
    const int nt = (int)(term_off[c + 1] - term_off[c]);
    st = build_pauli_table(nc, nt, nt ? x + term_off[c] : nullptr, nt ? z + term_off[c] : nullptr,
                           nt ? coeff + term_off[c] : nullptr, &t);
    if (!st.good()) return fail_st(st.code, who + st.msg);
    b->grp_off[c] = (int64_t)groups.size();
    b->ngroups[c] = (int32_t)t.groups.size();
    for (PauliGroup g : t.groups) {
      g.first += (int32_t)terms.size();
      groups.push_back(g);
    }
    terms.insert(terms.end(), t.terms.begin(), t.terms.end());
    // work estimate for longest-first ordering: state size x (gates + groups)
    b->cost.push_back((double)(gx.size() * 3 + t.groups.size() + 1) * (double)(1ull << nc));
    b->nmax = std::max(b->nmax, nc);
    b->nrot_max = std::max(b->nrot_max, nr);
  }
  b->nrot_total = rot_total;
  if (hipGetDevice(&b->device) != hipSuccess) {
    (void)hipGetLastError();
    return fail_st(QS_ENODEV, "qs_batch_create: no HIP device");
  }
  if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess ||
      b->cus <= 0) {
    (void)hipGetLastError();
    return fail_st(QS_EHIP, "qs_batch_create: compute unit count unavailable");
  }
  // static arena: groups | terms | order (LPT, then input order)
  const size_t o_groups = 0;
  const size_t o_terms = align256(o_groups + std::max<size_t>(1, groups.size()) * sizeof(PauliGroup));
  const size_t o_order = align256(o_terms + std::max<size_t>(1, terms.size()) * sizeof(PauliTerm));
  const size_t total = align256(o_order + 2 * (size_t)ncirc * sizeof(int32_t));
  std::vector<char> blob(total, 0);
  if (!groups.empty()) memcpy(blob.data() + o_groups, groups.data(), groups.size() * sizeof(PauliGroup));
  if (!terms.empty()) memcpy(blob.data() + o_terms, terms.data(), terms.size() * sizeof(PauliTerm));
  std::vector<int32_t> ord(2 * (size_t)ncirc);
  for (int c = 0; c < ncirc; ++c) ord[c] = ord[ncirc + c] = c;
  std::stable_sort(ord.begin(), ord.begin() + ncirc,
                   [&](int a, int c) { return b->cost[a] > b->cost[c]; });
  if (ncirc) memcpy(blob.data() + o_order, ord.data(), ord.size() * sizeof(int32_t));
  if (hipMalloc(&b->stat, total) != hipSuccess) {
    (void)hipGetLastError();
    return fail_st(QS_ENOMEM, "qs_batch_create: arena allocation failed");
  }
  Status st = hip_status(hipMemcpy(b->stat, blob.data(), total, hipMemcpyHostToDevice), "batch upload");
  if (!st.good()) {
    (void)hipFree(b->stat);
    return st;
  }
  char* a = (char*)b->stat;
  b->groups_dev = (const PauliGroup*)(a + o_groups);
  b->terms_dev = (const PauliTerm*)(a + o_terms);
  b->order_dev = (const int32_t*)(a + o_order);
  const size_t out_bytes = ((size_t)ncirc + (size_t)rot_total + 1) * sizeof(double);
  if (hipMalloc(&b->out, out_bytes) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(b->stat);
    return fail_st(QS_ENOMEM, "qs_batch_create: output allocation failed");
  }
  *outp = b.release();
  return Status::ok();
}

void batch_destroy(BatchImpl* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  if (b->stat) (void)hipFree(b->stat);
  if (b->out) (void)hipFree(b->out);
  if (b->sched) (void)hipFree(b->sched);
  if (b->ws) (void)hipFree(b->ws);
  if (b->host_out) (void)hipHostFree(b->host_out);
  delete b;
}

template <typename R, typename T, int B>
static Status launch_batch(const BatchDev& d, unsigned grid, size_t lds, hipStream_t stream) {
  auto kern = k_batch<R, T, B>;
  Status st = hip_status(hipFuncSetAttribute((const void*)kern,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds),
                         "batch LDS attribute");
  if (!st.good()) return st;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(B), lds, stream, d);
  return hip_status(hipGetLastError(), "batch launch");
}

// Largest workspace the batch may hold (slots of psi, lambda and gradient rows).
constexpr size_t kBatchWsCap = (size_t)16 << 30;

Status batch_run(BatchImpl* b, const qs_batch_tuning* tune, double* energy, double* grad) {
  const size_t ab = amp_bytes(b->dtype);
  int threads = 256, wgcu = 2, order = 0, K = 0;
  int C = 11;
  if (tune) {
    if (tune->threads) threads = tune->threads;
    if (tune->lds_bits) C = tune->lds_bits;
    if (tune->wg_per_cu) wgcu = tune->wg_per_cu;
    K = tune->khigh;
    order = tune->order;
  }
  if (K == 0) K = std::min(5, C - 6);
  if (threads != 256 && threads != 512)
    return fail_st(QS_EINVAL, "qs_batch_run: threads must be 256 or 512");
  if (C < 8 || C > 13 || (size_t)2 * ((size_t)1 << C) * ab > (size_t)128 * 1024)
    return fail_st(QS_EINVAL, "qs_batch_run: lds_bits out of range for this dtype");
  if (K < 2 || K > kBatchMaxHigh || K > C - 6)
    return fail_st(QS_EINVAL, "qs_batch_run: khigh out of range");
  if (wgcu < 1 || wgcu > 8) return fail_st(QS_EINVAL, "qs_batch_run: wg_per_cu out of range");
  if (order != 0 && order != 1) return fail_st(QS_EINVAL, "qs_batch_run: order must be 0 or 1");
  if (b->ncirc == 0) return Status::ok();
  Status st = build_schedule(b, C, K);
  if (!st.good()) return st;
  const size_t lds = 2 * ((size_t)1 << C) * ab;
  const int NW = threads / 64;
  const uint64_t units = b->nmax > C ? 1ull << b->nmax : 0;
  const size_t slot = align256(2 * units * ab + (size_t)b->nrot_max * NW * sizeof(double));
  int64_t grid = std::min<int64_t>((int64_t)b->cus * wgcu, b->ncirc);
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, (int64_t)(kBatchWsCap / std::max<size_t>(slot, 1))));
  const size_t need = slot * (size_t)grid;
  if (b->ws_bytes < need) {
    if (b->ws) {
      st = hip_status(hipStreamSynchronize(b->stream), "batch sync");
      if (!st.good()) return st;
      (void)hipFree(b->ws);
    }
    b->ws = nullptr;
    b->ws_bytes = 0;
    if (hipMalloc(&b->ws, need) != hipSuccess) {
      (void)hipGetLastError();
      return fail_st(QS_ENOMEM, "qs_batch_run: workspace allocation of " + std::to_string(need) +
                                    " bytes failed");
    }
    b->ws_bytes = need;
  }
  BatchDev d;
  memset(&d, 0, sizeof(d));
  d.circ = b->circ_dev;
  d.recs = b->recs_dev;
  d.blks = b->blks_dev;
  d.segs = b->segs_dev;
  d.groups = b->groups_dev;
  d.terms = b->terms_dev;
  d.order = b->order_dev + (order == 1 ? b->ncirc : 0);
  d.energy = (double*)b->out;
  d.grad_rot = d.energy + b->ncirc;
  d.counter = (unsigned int*)(d.grad_rot + b->nrot_total);
  d.ws = (char*)b->ws;
  d.ws_slot_bytes = slot;
  d.state_units = units;
  d.ncirc = b->ncirc;
  d.lds_bits = C;
  d.khigh = K;
  hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, b->stream, d.counter);
  if (b->dtype == QS_C128)
    st = threads == 256 ? launch_batch<double, d2, 256>(d, (unsigned)grid, lds, b->stream)
                        : launch_batch<double, d2, 512>(d, (unsigned)grid, lds, b->stream);
  else
    st = threads == 256 ? launch_batch<float, f2, 256>(d, (unsigned)grid, lds, b->stream)
                        : launch_batch<float, f2, 512>(d, (unsigned)grid, lds, b->stream);
  if (!st.good()) return st;
  const size_t nout = (size_t)b->ncirc + (size_t)b->nrot_total;
  if (b->host_out_bytes < nout * sizeof(double)) {
    if (b->host_out) (void)hipHostFree(b->host_out);
    b->host_out = nullptr;
    b->host_out_bytes = 0;
    if (hipHostMalloc((void**)&b->host_out, nout * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail_st(QS_ENOMEM, "qs_batch_run: pinned host allocation failed");
    }
    b->host_out_bytes = nout * sizeof(double);
  }
  st = hip_status(hipMemcpyAsync(b->host_out, b->out, nout * sizeof(double), hipMemcpyDeviceToHost,
                                 b->stream), "batch result copy");
  if (!st.good()) return st;
  st = hip_status(hipStreamSynchronize(b->stream), "batch sync");
  if (!st.good()) return st;
  if (energy) memcpy(energy, b->host_out, (size_t)b->ncirc * sizeof(double));
  if (grad) {
    const int64_t np = b->par_off[b->ncirc];
    for (int64_t p = 0; p < np; ++p) grad[p] = 0.0;
    for (int c = 0; c < b->ncirc; ++c)
      for (int64_t g = b->op_off[c]; g < b->op_off[c + 1]; ++g) {
        const HostOp& h = b->ops[g];
        if (h.rot >= 0) grad[b->par_off[c] + h.param] += b->host_out[b->ncirc + b->rot_off[c] + h.rot];
      }
  }
  return Status::ok();
}

}  // namespace qs
