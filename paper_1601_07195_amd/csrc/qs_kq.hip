// qs_kq.hip -- a dense gate on a block of k <= 5 qubits.
//
// One thread per group of 2^k amplitudes that differ only in the target
// bits: the group's base index is the thread's group number with a zero
// inserted at every target position (ascending), so consecutive lanes read
// consecutive bases (coalesced whenever the lowest qubits are not targets),
// and member r of the group sits at base | off[r].  The group is loaded into
// registers, each output row is a sum of 2^k complex products with the
// matrix entries (uniform: scalar loads), and is stored where it was read.
// Bytes: 2 * 2^n * b per gate, like a single-qubit gate; arithmetic 8 * 2^k
// flop per amplitude, so k <= 4 stays HBM-bound at complex128 and k = 5
// approaches the FP64 vector rate: complex128 k = 5 therefore runs as a
// dense real contraction on the FP64 matrix cores (k_apply_kq_mfma).
#include <string.h>

#include <algorithm>
#include <vector>

#include "qs_device.h"
#include "qs_internal.h"

namespace qs {

constexpr int kKqBlock = 256;
// Workgroup size of the direct kernel: 64 for k <= 2 (measured faster with
// the highest targets), 256 above.
template <int K>
constexpr int kq_block() { return K <= 2 ? 64 : kKqBlock; }

typedef double d4 __attribute__((ext_vector_type(4)));

struct KqArgs {
  uint64_t ngroups;
  uint64_t off[32];  // offset of group member r
  int32_t spos[QS_KQ_MAX];  // target positions, ascending
  int32_t k;
};

// Copy of *p read through the constant address space (scalar loads for a
// uniform p); for the gate matrix, which nothing writes during the kernel.
template <typename R>
__device__ __forceinline__ R ldc_r(const R* p) {
  return *(const __attribute__((address_space(4))) R*)p;
}

template <typename R, typename T, int K>
__global__ void __launch_bounds__(kq_block<K>())
k_apply_kq(T* __restrict__ a, const R* __restrict__ u, KqArgs A) {
  constexpr int D = 1 << K;
  constexpr int B = kq_block<K>();
  const uint64_t stride = (uint64_t)gridDim.x * B;
  for (uint64_t g = (uint64_t)blockIdx.x * B + threadIdx.x; g < A.ngroups; g += stride) {
    uint64_t base = g;
#pragma unroll
    for (int j = 0; j < K; ++j) base = insert0(base, A.spos[j]);
    T v[D];
#pragma unroll
    for (int c = 0; c < D; ++c) v[c] = gload<true>(a + (base | A.off[c]));
#pragma unroll 1
    for (int r = 0; r < D; ++r) {
      const R* row = u + 2 * D * r;
      R sr = (R)0, si = (R)0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const R ur = ldc_r(row + 2 * c), ui = ldc_r(row + 2 * c + 1);
        sr += ur * v[c].x - ui * v[c].y;
        si += ur * v[c].y + ui * v[c].x;
      }
      gstore<true>(a + (base | A.off[r]), T{sr, si});
    }
  }
}

// Low targets (some target among the 6 lowest bits): the groups of one
// workgroup are staged through LDS.  The workgroup's tile is every index
// whose bits outside P vary only with the workgroup number, where P = the
// targets plus the `ln` lowest non-target bits (ln = log2 of the threads);
// tile element q has bit b at index bit P[b].  P[0 .. ln) are index bits
// 0 .. ln-1, so load and store instruction i moves elements
// q = i * 2^ln + lane: 2^ln consecutive amplitudes, coalesced.  Thread t
// owns the group whose non-target tile bits spell t.
struct KqLdsArgs {
  uint64_t ntiles;
  uint64_t hi_off[32];  // index offset of instruction i's elements (the P bits above ln)
  uint32_t mq[32];      // tile element offset of group member r (target bits of q)
  int32_t ppos[QS_KQ_MAX + 6];  // P, ascending
  int32_t tq_bit[6];    // tile bit that thread bit b sets
  int32_t np, ln;
};

template <typename T>
__device__ __forceinline__ uint32_t kq_slot(uint32_t q);
template <>
__device__ __forceinline__ uint32_t kq_slot<d2>(uint32_t q) {
  return q ^ (((q >> 3) ^ (q >> 6) ^ (q >> 9)) & 7u);
}
template <>
__device__ __forceinline__ uint32_t kq_slot<f2>(uint32_t q) {
  return q ^ (((q >> 4) ^ (q >> 8)) & 15u);
}

template <typename R, typename T, int K>
__global__ void __launch_bounds__(64)
k_apply_kq_lds(T* __restrict__ a, const R* __restrict__ u, KqLdsArgs A) {
  constexpr int D = 1 << K;
  __shared__ T tile[64 * D];
  const uint32_t lane = threadIdx.x;
  const uint32_t nth = 1u << A.ln;
  uint32_t tq = 0;  // this thread's group: its non-target tile bits
  for (int b = 0; b < A.ln; ++b) tq |= ((lane >> b) & 1u) << A.tq_bit[b];
  for (uint64_t w = blockIdx.x; w < A.ntiles; w += gridDim.x) {
    uint64_t base = w;
    for (int j = 0; j < A.np; ++j) base = insert0(base, A.ppos[j]);
    // eight loads in flight at a time keeps k = 5 within a few waves' registers
#pragma unroll 8
    for (int i = 0; i < D; ++i)
      tile[kq_slot<T>(i * nth + lane)] = gload<true>(a + (base | lane | A.hi_off[i]));
    __syncthreads();
    T v[D];
#pragma unroll
    for (int c = 0; c < D; ++c) v[c] = tile[kq_slot<T>(tq | A.mq[c])];
#pragma unroll 1
    for (int r = 0; r < D; ++r) {
      const R* row = u + 2 * D * r;
      R sr = (R)0, si = (R)0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const R ur = ldc_r(row + 2 * c), ui = ldc_r(row + 2 * c + 1);
        sr += ur * v[c].x - ui * v[c].y;
        si += ur * v[c].y + ui * v[c].x;
      }
      tile[kq_slot<T>(tq | A.mq[r])] = T{sr, si};
    }
    __syncthreads();
#pragma unroll 8
    for (int i = 0; i < D; ++i)
      gstore<true>(a + (base | lane | A.hi_off[i]), tile[kq_slot<T>(i * nth + lane)]);
    __syncthreads();
  }
}

// complex128, k = 5 (the template also takes k = 4, where the vector
// kernels measure faster): the gate as a dense real contraction on the FP64
// matrix cores.  With D = 2^k members per group, the 2D x 2D real matrix
// M = [[Re u, -Im u], [Im u, Re u]] maps (Re v, Im v) of a group to those
// of u v.  A wave applies M to 16 groups at once: C (2D x 16) = M B, as
// 2D/16 row blocks x 2D/4 steps of v_mfma_f64_16x16x4 (A: a 16 x 4 block of
// M, lane i + 16 kk holding A[i][kk]; B: 4 x 16, lane jj + 16 kk holding
// B[kk][jj]; C: lane jj + 16 (i % 4) holding C[i][jj] as item i / 4).  Lane
// l works on group l % 16 and, with q = l / 16, loads members q, q + 4, ...
// (row 4 ks + q of B is part (4 ks + q) / D of member (4 ks + q) % D), and
// stores members 16 mb + q + 4 i (rows of C's block mb).  M's blocks are staged once
// per workgroup in LDS in operand order: one conflict-free 8-byte LDS load
// per lane feeds each MFMA.  Loads of 16 consecutive groups cover whole
// lines whatever the targets, so no LDS tile of the state is needed.
constexpr int kKqMfmaBlock = 256;

struct KqMfmaArgs {
  uint64_t nbatches;           // batches of 16 groups
  int32_t spos[QS_KQ_MAX];     // target positions, ascending
  int32_t tpos[QS_KQ_MAX];     // target of bit j of a member index
};

template <int K>
__device__ __forceinline__ uint64_t kq_member_off(int r, const KqMfmaArgs& A) {
  uint64_t o = 0;
#pragma unroll
  for (int t = 0; t < K; ++t) o |= (uint64_t)((r >> t) & 1) << A.tpos[t];
  return o;
}

template <int K>
__global__ void __launch_bounds__(kKqMfmaBlock)
k_apply_kq_mfma(d2* __restrict__ a, const double* __restrict__ frag, KqMfmaArgs A) {
  constexpr int D = 1 << K, M = 2 * D, MB = M / 16, KS = M / 4, NV = D / 4;
  __shared__ double sa[MB * KS * 64];
  for (int i = threadIdx.x; i < MB * KS * 64; i += kKqMfmaBlock) sa[i] = frag[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, j = lane & 15, q = lane >> 4;
  uint64_t ld[NV], st[NV];
#pragma unroll
  for (int s = 0; s < NV; ++s) {
    ld[s] = kq_member_off<K>(q + 4 * s, A);
    st[s] = kq_member_off<K>(16 * (s / 4) + q + 4 * (s % 4), A);
  }
  const uint64_t nw = (uint64_t)gridDim.x * (kKqMfmaBlock / 64);
  for (uint64_t bt = (uint64_t)blockIdx.x * (kKqMfmaBlock / 64) + threadIdx.x / 64; bt < A.nbatches;
       bt += nw) {
    uint64_t base = bt * 16 + j;
#pragma unroll
    for (int t = 0; t < K; ++t) base = insert0(base, A.spos[t]);
    d2 v[NV];
#pragma unroll
    for (int s = 0; s < NV; ++s) v[s] = gload<true>(a + (base | ld[s]));
    d4 acc[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const double b = ks < NV ? v[ks].x : v[ks - NV].y;
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
        acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[(mb * KS + ks) * 64 + lane], b, acc[mb], 0, 0, 0);
    }
    // real rows in blocks 0 .. MB/2 - 1, the imaginary rows MB/2 blocks later
#pragma unroll
    for (int s = 0; s < NV; ++s)
      gstore<true>(a + (base | st[s]), d2{acc[s / 4][s % 4], acc[s / 4 + MB / 2][s % 4]});
  }
}

template <typename R, typename T>
static void go_kq_lds(StateImpl* s, int k, const R* u, const KqLdsArgs& A, unsigned grid) {
  T* a = (T*)s->ptr;
  const unsigned th = 1u << A.ln;
  switch (k) {
    case 1: hipLaunchKernelGGL((k_apply_kq_lds<R, T, 1>), dim3(grid), dim3(th), 0, s->stream, a, u, A); break;
    case 2: hipLaunchKernelGGL((k_apply_kq_lds<R, T, 2>), dim3(grid), dim3(th), 0, s->stream, a, u, A); break;
    case 3: hipLaunchKernelGGL((k_apply_kq_lds<R, T, 3>), dim3(grid), dim3(th), 0, s->stream, a, u, A); break;
    case 4: hipLaunchKernelGGL((k_apply_kq_lds<R, T, 4>), dim3(grid), dim3(th), 0, s->stream, a, u, A); break;
    default: hipLaunchKernelGGL((k_apply_kq_lds<R, T, 5>), dim3(grid), dim3(th), 0, s->stream, a, u, A); break;
  }
}

template <int K>
static unsigned kq_grid(uint64_t ngroups) {
  constexpr int B = kq_block<K>();
  const uint64_t want = (ngroups + B - 1) / B;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (1ull << 31) / B));
}

// k <= 2 (one-wave workgroups) run with the paired-stream occupancy cap of
// three waves per SIMD, which measured 2-12 % faster (k = 1 on target 20:
// 5.5 -> 6.2 TB/s); k = 3, 4 measured within noise of uncapped.
template <typename R, typename T>
static void go_kq(StateImpl* s, int k, const R* u, const KqArgs& A) {
  T* a = (T*)s->ptr;
  switch (k) {
    case 1: hipLaunchKernelGGL((k_apply_kq<R, T, 1>), dim3(kq_grid<1>(A.ngroups)), dim3(kq_block<1>()), stream_lds(kq_block<1>(), 0, 3), s->stream, a, u, A); break;
    case 2: hipLaunchKernelGGL((k_apply_kq<R, T, 2>), dim3(kq_grid<2>(A.ngroups)), dim3(kq_block<2>()), stream_lds(kq_block<2>(), 0, 3), s->stream, a, u, A); break;
    case 3: hipLaunchKernelGGL((k_apply_kq<R, T, 3>), dim3(kq_grid<3>(A.ngroups)), dim3(kq_block<3>()), stream_lds(kq_block<3>(), 0, 0), s->stream, a, u, A); break;
    case 4: hipLaunchKernelGGL((k_apply_kq<R, T, 4>), dim3(kq_grid<4>(A.ngroups)), dim3(kq_block<4>()), stream_lds(kq_block<4>(), 0, 0), s->stream, a, u, A); break;
    default: hipLaunchKernelGGL((k_apply_kq<R, T, 5>), dim3(kq_grid<5>(A.ngroups)), dim3(kq_block<5>()), 0, s->stream, a, u, A); break;
  }
}

Status launch_apply_kq(StateImpl* s, int k, const int32_t* targets, const double* u) {
  const int D = 1 << k;
  KqArgs A;
  memset(&A, 0, sizeof(A));
  A.k = k;
  A.ngroups = 1ull << (s->n - k);
  for (int r = 0; r < D; ++r)
    for (int j = 0; j < k; ++j)
      if ((r >> j) & 1) A.off[r] |= 1ull << targets[j];
  int sp[QS_KQ_MAX];
  for (int j = 0; j < k; ++j) sp[j] = targets[j];
  std::sort(sp, sp + k);
  for (int j = 0; j < k; ++j) A.spos[j] = sp[j];
  if (s->dtype == QS_C128 && k == 5 && s->n - k >= 4) {
    // M = [[Re u, -Im u], [Im u, Re u]] in MFMA operand order:
    // frag[(mb * KS + ks) * 64 + l] = M[16 mb + l % 16][4 ks + l / 16]
    const int M = 2 * D, MB = M / 16, KS = M / 4;
    std::vector<double> frag((size_t)MB * KS * 64);
    auto mval = [&](int row, int col) {
      const int r = row % D, c = col % D;
      const double re = u[2 * (r * D + c)], im = u[2 * (r * D + c) + 1];
      if ((row < D) == (col < D)) return re;
      return row < D ? -im : im;
    };
    for (int mb = 0; mb < MB; ++mb)
      for (int ks = 0; ks < KS; ++ks)
        for (int l = 0; l < 64; ++l)
          frag[((size_t)mb * KS + ks) * 64 + l] = mval(16 * mb + l % 16, 4 * ks + l / 16);
    Status st = upload_table(s, frag.data(), frag.size() * sizeof(double));
    if (!st.good()) return st;
    KqMfmaArgs B;
    memset(&B, 0, sizeof(B));
    B.nbatches = A.ngroups / 16;
    for (int j = 0; j < k; ++j) {
      B.spos[j] = sp[j];
      B.tpos[j] = targets[j];
    }
    const uint64_t want = (B.nbatches + kKqMfmaBlock / 64 - 1) / (kKqMfmaBlock / 64);
    // about five workgroups per compute unit (the LDS holds five copies of M)
    const uint64_t cus = s->cus > 0 ? (uint64_t)s->cus : 256;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, cus * 5));
    if (k == 4)
      hipLaunchKernelGGL((k_apply_kq_mfma<4>), dim3(grid), dim3(kKqMfmaBlock), 0, s->stream, (d2*)s->ptr,
                         (const double*)s->table.ptr, B);
    else
      hipLaunchKernelGGL((k_apply_kq_mfma<5>), dim3(grid), dim3(kKqMfmaBlock), 0, s->stream, (d2*)s->ptr,
                         (const double*)s->table.ptr, B);
    return hip_status(hipGetLastError(), "apply_kq (mfma)");
  }
  // the matrix in the compute precision, through the state's table buffer
  const size_t nval = 2 * (size_t)D * D;
  Status st;
  if (s->dtype == QS_C128) {
    st = upload_table(s, u, nval * sizeof(double));
  } else {
    float f[2 * 32 * 32];
    for (size_t i = 0; i < nval; ++i) f[i] = (float)u[i];
    st = upload_table(s, f, nval * sizeof(float));
  }
  if (!st.good()) return st;
  if (sp[0] < 6) {
    // some target among the lane bits: stage the groups through LDS
    KqLdsArgs L;
    memset(&L, 0, sizeof(L));
    const int n = s->n;
    L.ln = std::min(6, n - k);
    int P[QS_KQ_MAX + 6], np = 0;
    uint64_t tmask = 0;
    for (int j = 0; j < k; ++j) tmask |= 1ull << targets[j];
    for (int b = 0, taken = 0; b < n && (taken < L.ln || np < k + L.ln); ++b) {
      const bool tgt = (tmask >> b) & 1;
      if (tgt || taken < L.ln) {
        P[np++] = b;
        taken += !tgt;
      }
    }
    L.np = np;  // k + ln entries
    for (int b = 0; b < np; ++b) L.ppos[b] = P[b];
    // tile bit of each target and of each non-target P entry (ascending)
    int tb_of_target[QS_KQ_MAX];
    for (int j = 0; j < k; ++j)
      for (int b = 0; b < np; ++b)
        if (P[b] == targets[j]) tb_of_target[j] = b;
    for (int b = 0, t = 0; b < np; ++b)
      if (!((tmask >> P[b]) & 1)) L.tq_bit[t++] = b;
    for (int r = 0; r < D; ++r)
      for (int j = 0; j < k; ++j)
        if ((r >> j) & 1) L.mq[r] |= 1u << tb_of_target[j];
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < k; ++j)
        if ((i >> j) & 1) L.hi_off[i] |= 1ull << P[L.ln + j];
    L.ntiles = 1ull << (n - np);
    const unsigned lgrid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(L.ntiles, 1ull << 24));
    if (s->dtype == QS_C128)
      go_kq_lds<double, d2>(s, k, (const double*)s->table.ptr, L, lgrid);
    else
      go_kq_lds<float, f2>(s, k, (const float*)s->table.ptr, L, lgrid);
    return hip_status(hipGetLastError(), "apply_kq");
  }
  if (s->dtype == QS_C128)
    go_kq<double, d2>(s, k, (const double*)s->table.ptr, A);
  else
    go_kq<float, f2>(s, k, (const float*)s->table.ptr, A);
  return hip_status(hipGetLastError(), "apply_kq");
}

}  // namespace qs
