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
// approaches the FP64 vector rate.
#include <string.h>

#include <algorithm>

#include "qs_device.h"
#include "qs_internal.h"

namespace qs {

constexpr int kKqBlock = 256;

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
__global__ void __launch_bounds__(kKqBlock)
k_apply_kq(T* __restrict__ a, const R* __restrict__ u, KqArgs A) {
  constexpr int D = 1 << K;
  const uint64_t stride = (uint64_t)gridDim.x * kKqBlock;
  for (uint64_t g = (uint64_t)blockIdx.x * kKqBlock + threadIdx.x; g < A.ngroups; g += stride) {
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

template <typename R, typename T>
static void go_kq(StateImpl* s, int k, const R* u, const KqArgs& A, unsigned grid) {
  T* a = (T*)s->ptr;
  switch (k) {
    case 1: hipLaunchKernelGGL((k_apply_kq<R, T, 1>), dim3(grid), dim3(kKqBlock), 0, s->stream, a, u, A); break;
    case 2: hipLaunchKernelGGL((k_apply_kq<R, T, 2>), dim3(grid), dim3(kKqBlock), 0, s->stream, a, u, A); break;
    case 3: hipLaunchKernelGGL((k_apply_kq<R, T, 3>), dim3(grid), dim3(kKqBlock), 0, s->stream, a, u, A); break;
    case 4: hipLaunchKernelGGL((k_apply_kq<R, T, 4>), dim3(grid), dim3(kKqBlock), 0, s->stream, a, u, A); break;
    default: hipLaunchKernelGGL((k_apply_kq<R, T, 5>), dim3(grid), dim3(kKqBlock), 0, s->stream, a, u, A); break;
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
  const uint64_t want = (A.ngroups + kKqBlock - 1) / kKqBlock;
  const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, (1ull << 31) / kKqBlock));
  if (s->dtype == QS_C128)
    go_kq<double, d2>(s, k, (const double*)s->table.ptr, A, grid);
  else
    go_kq<float, f2>(s, k, (const float*)s->table.ptr, A, grid);
  return hip_status(hipGetLastError(), "apply_kq");
}

}  // namespace qs
