// qs_gates.hip -- streaming gate kernels: one pass over the state per gate.
//
// Single-qubit gate (qHiPSTER Eq. 2): the 2^(n-1) pairs (i0, i0 + 2^k) with
// bit k of i0 clear are enumerated by a flat pair index p, i0 = p with a 0
// inserted at bit k.  Consecutive lanes take consecutive p, so for every
// target the two streams a[i0] and a[i0 + 2^k] are read and written as
// contiguous 16-byte-per-lane runs (a wavefront touches 1 KiB per access),
// instead of the paper's two-level loop nest (Fig. 2) that a CPU thread walks.
//
// Controlled gate (Eq. 3): only the 2^(n-2) quads with control bit 1 are
// visited: p with 0s inserted at both c and t, then bit c set.  Amplitudes
// with control bit 0 are neither read nor written (half the traffic of a
// single-qubit gate, Table 2 case 3).
//
// complex64 states are moved two amplitudes (16 B) per access: in "vector"
// index space (vector v = amplitudes 2v, 2v+1) a qubit q >= 1 is vector bit
// q-1.  Qubit 0 lives inside a vector; gates on it use the *_inner kernels.
#include "qs_device.h"
#include "qs_internal.h"

namespace qs {

// ----------------------------------------------------------- |index> init
// Writes 16-byte zeros over the state and the 16-byte vector holding the
// amplitude `index` with `one` (1.0 + 0i placed at the right offset).
template <int V>
__global__ void __launch_bounds__(kBlock)
k_init_basis(u64x2* __restrict__ a, uint64_t nvec, uint64_t one_vec, u64x2 one) {
  const uint64_t base = (uint64_t)blockIdx.x * (kBlock * V) + threadIdx.x;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint64_t j = base + (uint64_t)v * kBlock;
    if (j < nvec) a[j] = (j == one_vec) ? one : u64x2{0ull, 0ull};
  }
}

// ------------------------------------------------------- 1-qubit, strided
// `a` in units of T (d2: one c128 amplitude; f2: one c64 amplitude; f4: two
// c64 amplitudes), k the target bit in those units, npairs = pairs of units.
template <typename R, typename T, int V, bool NT>
__global__ void __launch_bounds__(kBlock)
k_apply_1q(T* __restrict__ a, uint64_t npairs, int k, Mat<R> q) {
  const uint64_t s = 1ull << k;
  const uint64_t p0 = (uint64_t)blockIdx.x * (kBlock * V) + threadIdx.x;
  T x[V], y[V];
  uint64_t i0[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint64_t p = p0 + (uint64_t)v * kBlock;
    i0[v] = insert0(p, k);
    if (p < npairs) {
      x[v] = gload<NT>(a + i0[v]);
      y[v] = gload<NT>(a + i0[v] + s);
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint64_t p = p0 + (uint64_t)v * kBlock;
    if (p < npairs) {
      pair_apply(q, x[v], y[v]);
      gstore<NT>(a + i0[v], x[v]);
      gstore<NT>(a + i0[v] + s, y[v]);
    }
  }
}

// complex64, target qubit 0: each f4 holds one whole pair.
template <int V, bool NT>
__global__ void __launch_bounds__(kBlock)
k_apply_1q_inner(f4* __restrict__ a, uint64_t nvec, Mat<float> q) {
  const uint64_t base = (uint64_t)blockIdx.x * (kBlock * V) + threadIdx.x;
  f4 x[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint64_t j = base + (uint64_t)v * kBlock;
    if (j < nvec) x[v] = gload<NT>(a + j);
  }
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint64_t j = base + (uint64_t)v * kBlock;
    if (j < nvec) {
      pair_apply_inner(q, x[v]);
      gstore<NT>(a + j, x[v]);
    }
  }
}

// ---------------------------------------------------- controlled, strided
// Units as in k_apply_1q; c, t are unit bits; nquads = 2^(units_log2 - 2).
template <typename R, typename T, int V, bool NT>
__global__ void __launch_bounds__(kBlock)
k_apply_cu(T* __restrict__ a, uint64_t nquads, int c, int t, Mat<R> q) {
  const int lo = c < t ? c : t, hi = c < t ? t : c;
  const uint64_t cm = 1ull << c, s = 1ull << t;
  const uint64_t p0 = (uint64_t)blockIdx.x * (kBlock * V) + threadIdx.x;
  T x[V], y[V];
  uint64_t i0[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint64_t p = p0 + (uint64_t)v * kBlock;
    i0[v] = insert0(insert0(p, lo), hi) | cm;
    if (p < nquads) {
      x[v] = gload<NT>(a + i0[v]);
      y[v] = gload<NT>(a + i0[v] + s);
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint64_t p = p0 + (uint64_t)v * kBlock;
    if (p < nquads) {
      pair_apply(q, x[v], y[v]);
      gstore<NT>(a + i0[v], x[v]);
      gstore<NT>(a + i0[v] + s, y[v]);
    }
  }
}

// complex64, target qubit 0, control c >= 1 (vector bit cv = c - 1): the
// vectors with bit cv set each hold one pair to update.
template <int V, bool NT>
__global__ void __launch_bounds__(kBlock)
k_apply_cu_inner(f4* __restrict__ a, uint64_t nsel, int cv, Mat<float> q) {
  const uint64_t base = (uint64_t)blockIdx.x * (kBlock * V) + threadIdx.x;
  const uint64_t cm = 1ull << cv;
  f4 x[V];
  uint64_t j[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint64_t p = base + (uint64_t)v * kBlock;
    j[v] = insert0(p, cv) | cm;
    if (p < nsel) x[v] = gload<NT>(a + j[v]);
  }
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint64_t p = base + (uint64_t)v * kBlock;
    if (p < nsel) {
      pair_apply_inner(q, x[v]);
      gstore<NT>(a + j[v], x[v]);
    }
  }
}

// ------------------------------------------------------------- launchers

template <typename R>
Mat<R> to_mat(const double* q) {
  Mat<R> m;
  for (int e = 0; e < 4; ++e) {
    m.r[e] = (R)q[2 * e];
    m.i[e] = (R)q[2 * e + 1];
  }
  return m;
}

constexpr int kV = 4;      // units per lane per stream
constexpr bool kNT = true; // non-temporal global accesses

static unsigned grid_for(uint64_t items, int per_block) {
  return (unsigned)((items + per_block - 1) / per_block);
}

Status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return Status::ok();
  Status s;
  s.code = QS_EHIP;
  s.msg = std::string(what) + ": " + hipGetErrorString(e);
  return s;
}

static Status last_launch(const char* what) { return hip_status(hipGetLastError(), what); }

Status launch_init_basis(StateImpl* s, uint64_t index) {
  const uint64_t nvec = (((uint64_t)1 << s->n) * amp_bytes(s->dtype)) / 16;
  uint64_t one_vec;
  u64x2 one;
  const unsigned long long one_bits_d = 0x3FF0000000000000ull;  // 1.0 (double)
  const unsigned long long one_bits_f = 0x3F800000ull;          // 1.0f in the low word
  if (s->dtype == QS_C128) {
    one_vec = index;
    one = u64x2{one_bits_d, 0ull};
  } else {
    one_vec = index >> 1;
    one = (index & 1) ? u64x2{0ull, one_bits_f} : u64x2{one_bits_f, 0ull};
  }
  hipLaunchKernelGGL((k_init_basis<kV>), dim3(grid_for(nvec, kBlock * kV)), dim3(kBlock), 0,
                     s->stream, (u64x2*)s->ptr, nvec, one_vec, one);
  return last_launch("init_basis");
}

Status launch_apply_1q(StateImpl* s, int k, const double* q) {
  const int n = s->n;
  if (s->dtype == QS_C128) {
    const uint64_t np = (uint64_t)1 << (n - 1);
    hipLaunchKernelGGL((k_apply_1q<double, d2, kV, kNT>), dim3(grid_for(np, kBlock * kV)),
                       dim3(kBlock), 0, s->stream, (d2*)s->ptr, np, k, to_mat<double>(q));
    return last_launch("apply_1q c128");
  }
  const Mat<float> m = to_mat<float>(q);
  if (n == 1 || k == 0) {
    const uint64_t nvec = (uint64_t)1 << (n - 1);
    hipLaunchKernelGGL((k_apply_1q_inner<kV, kNT>), dim3(grid_for(nvec, kBlock * kV)),
                       dim3(kBlock), 0, s->stream, (f4*)s->ptr, nvec, m);
    return last_launch("apply_1q c64 inner");
  }
  const uint64_t np = (uint64_t)1 << (n - 2);
  hipLaunchKernelGGL((k_apply_1q<float, f4, kV, kNT>), dim3(grid_for(np, kBlock * kV)),
                     dim3(kBlock), 0, s->stream, (f4*)s->ptr, np, k - 1, m);
  return last_launch("apply_1q c64");
}

Status launch_apply_cu(StateImpl* s, int c, int t, const double* q) {
  const int n = s->n;
  if (s->dtype == QS_C128) {
    const uint64_t nq = (uint64_t)1 << (n - 2);
    hipLaunchKernelGGL((k_apply_cu<double, d2, kV, kNT>), dim3(grid_for(nq, kBlock * kV)),
                       dim3(kBlock), 0, s->stream, (d2*)s->ptr, nq, c, t, to_mat<double>(q));
    return last_launch("apply_cu c128");
  }
  const Mat<float> m = to_mat<float>(q);
  if (t == 0) {
    const uint64_t nsel = (uint64_t)1 << (n - 2);
    hipLaunchKernelGGL((k_apply_cu_inner<kV, kNT>), dim3(grid_for(nsel, kBlock * kV)),
                       dim3(kBlock), 0, s->stream, (f4*)s->ptr, nsel, c - 1, m);
    return last_launch("apply_cu c64 inner");
  }
  if (c == 0) {
    // Control inside a vector: single 8-byte amplitudes.
    const uint64_t nq = (uint64_t)1 << (n - 2);
    hipLaunchKernelGGL((k_apply_cu<float, f2, kV, kNT>), dim3(grid_for(nq, kBlock * kV)),
                       dim3(kBlock), 0, s->stream, (f2*)s->ptr, nq, c, t, m);
    return last_launch("apply_cu c64 c0");
  }
  const uint64_t nq = (uint64_t)1 << (n - 3);
  hipLaunchKernelGGL((k_apply_cu<float, f4, kV, kNT>), dim3(grid_for(nq, kBlock * kV)),
                     dim3(kBlock), 0, s->stream, (f4*)s->ptr, nq, c - 1, t - 1, m);
  return last_launch("apply_cu c64");
}

}  // namespace qs
