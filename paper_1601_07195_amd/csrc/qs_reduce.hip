// qs_reduce.hip -- read-mostly passes over the state: measurement
// probabilities, Pauli-sum expectation values, H|psi>, inner products.
//
// Every sum is double precision, for complex64 states too.  Each workgroup
// walks a fixed set of chunks in a fixed order and leaves one partial per
// output; a one-workgroup kernel then adds the partials in a fixed order, so
// results are bitwise reproducible from run to run.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>

#include "qs_device.h"
#include "qs_internal.h"

namespace qs {

constexpr int kMaxQubits = 34;
constexpr int kReduceGrid = 2048;  // workgroups of the partial-sum passes

template <typename T>
__device__ __forceinline__ double norm2_of(const T& v) {
  return (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}

// ------------------------------------------------------------ final sums
// out[c] = sum over rows r of part[r * ncols + c], rows in increasing order
// per lane, then a fixed-shape tree across the workgroup.
__global__ void __launch_bounds__(kBlock)
k_sum_columns(const double* __restrict__ part, int nrows, int ncols, double* __restrict__ out) {
  __shared__ double lds[kBlock / 64];
  for (int c = 0; c < ncols; ++c) {
    double s = 0.0;
    for (int r = threadIdx.x; r < nrows; r += kBlock) s += part[(size_t)r * ncols + c];
    s = block_sum(s, lds);
    if (threadIdx.x == 0) out[c] = s;
  }
}

// --------------------------------------------------------- probabilities
// Chunks of 2^12 amplitudes; in chunk ch lane t reads i = ch*4096 + r*256 + t
// for r = 0..15.  So index bits 0..7 are the lane, bits 8..11 are r (known at
// compile time) and bits >= 12 are the chunk number: each lane keeps its
// total, four sums for bits 8..11 and one per chunk bit.
constexpr int kProbChunkLog = 12;

template <typename T, bool FULL>
__global__ void __launch_bounds__(kBlock)
k_probabilities(const T* __restrict__ a, int n, uint64_t nchunks, double* __restrict__ part,
                double* __restrict__ full) {
  __shared__ double lds[kBlock / 64];
  const uint64_t N = 1ull << n;
  double tot = 0.0, mid[4] = {0.0, 0.0, 0.0, 0.0};
  double hi[kMaxQubits - kProbChunkLog];
#pragma unroll
  for (int b = 0; b < kMaxQubits - kProbChunkLog; ++b) hi[b] = 0.0;

  for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const uint64_t base = ch << kProbChunkLog;
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint64_t i = base + (uint64_t)r * kBlock + threadIdx.x;
      double p = 0.0;
      if (i < N) {
        p = norm2_of(gload<true>(a + i));  // streamed: read once
        if (FULL) full[i] = p;
      }
      s += p;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if ((r >> b) & 1) mid[b] += p;
    }
    tot += s;
#pragma unroll
    for (int b = 0; b < kMaxQubits - kProbChunkLog; ++b)
      if ((ch >> b) & 1) hi[b] += s;
  }
  // Partials row: [P(bit 0) .. P(bit n-1), total].  Each wave reduces every
  // bit with butterfly exchanges (no barrier inside the unrolled loop, so
  // mid[] and hi[] stay in registers); the four wave sums are added in a
  // fixed order afterwards.
  __shared__ double wsum[kMaxQubits + 1][kBlock / 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < kMaxQubits; ++k) {
    double v;
    if (k < 8) v = ((threadIdx.x >> k) & 1) ? tot : 0.0;
    else if (k < kProbChunkLog) v = mid[k - 8];
    else v = hi[k - kProbChunkLog];
    v = wave_sum(v);
    if (lane == 0) wsum[k][w] = v;
  }
  {
    const double t = wave_sum(tot);
    if (lane == 0) wsum[kMaxQubits][w] = t;
  }
  __syncthreads();
  double* row = part + (size_t)blockIdx.x * (n + 1);
  const int k = threadIdx.x;
  if (k <= n) {
    const int src = (k == n) ? kMaxQubits : k;
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < kBlock / 64; ++j) v += wsum[src][j];
    row[k] = v;
  }
}

// complex64: 16-byte units of two amplitudes (bit 0 inside the unit), chunks
// of 2^13 amplitudes: in chunk ch lane t reads unit u = ch*4096 + r*256 + t,
// amplitudes 2u and 2u + 1.  Index bit 0 is the unit half, bits 1..8 the
// lane, bits 9..12 r, bits >= 13 the chunk number.
template <bool FULL>
__global__ void __launch_bounds__(kBlock)
k_probabilities_c64(const f4* __restrict__ a, int n, uint64_t nchunks, double* __restrict__ part,
                    double* __restrict__ full) {
  constexpr int CL = kProbChunkLog + 1;
  const uint64_t NU = 1ull << (n - 1);  // units (n >= 1)
  double tot = 0.0, b0 = 0.0, mid[4] = {0.0, 0.0, 0.0, 0.0};
  double hi[kMaxQubits - CL];
#pragma unroll
  for (int b = 0; b < kMaxQubits - CL; ++b) hi[b] = 0.0;

  for (uint64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const uint64_t base = ch << (CL - 1);
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint64_t u = base + (uint64_t)r * kBlock + threadIdx.x;
      double p = 0.0;
      if (u < NU) {
        const f4 v = gload<true>(a + u);  // streamed: read once
        const double p0 = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        const double p1 = (double)v.z * (double)v.z + (double)v.w * (double)v.w;
        if (FULL) {  // full is only 8-byte aligned
          full[2 * u] = p0;
          full[2 * u + 1] = p1;
        }
        b0 += p1;
        p = p0 + p1;
      }
      s += p;
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if ((r >> b) & 1) mid[b] += p;
    }
    tot += s;
#pragma unroll
    for (int b = 0; b < kMaxQubits - CL; ++b)
      if ((ch >> b) & 1) hi[b] += s;
  }
  __shared__ double wsum[kMaxQubits + 1][kBlock / 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < kMaxQubits; ++k) {
    double v;
    if (k == 0) v = b0;
    else if (k < 9) v = ((threadIdx.x >> (k - 1)) & 1) ? tot : 0.0;
    else if (k < CL) v = mid[k - 9];
    else v = hi[k - CL];
    v = wave_sum(v);
    if (lane == 0) wsum[k][w] = v;
  }
  {
    const double t = wave_sum(tot);
    if (lane == 0) wsum[kMaxQubits][w] = t;
  }
  __syncthreads();
  double* row = part + (size_t)blockIdx.x * (n + 1);
  const int k = threadIdx.x;
  if (k <= n) {
    const int src = (k == n) ? kMaxQubits : k;
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < kBlock / 64; ++j) v += wsum[src][j];
    row[k] = v;
  }
}

// ------------------------------------------------------------ Pauli sums
// For a Pauli string with masks (x, z) and n_Y = popcount(x & z) factors Y:
//   P|k> = i^(n_Y) (-1)^popcount(k & z) |k ^ x>        (Y = i X Z)
// so (P psi)[i] = i^(n_Y) (-1)^popcount((i ^ x) & z) psi[i ^ x].  Terms with
// the same x share the gathered amplitude psi[i ^ x]; each group costs one
// read of the state.  Term coefficients arrive pre-multiplied by i^(n_Y).

// (H psi)[i] restricted to groups [g0, g1): sum over groups of
// psi[i ^ x_g] * sum_{terms j in g} w_j (-1)^popcount((i ^ x_g) & z_j).
template <typename T>
__device__ __forceinline__ void hpsi_at(const T* __restrict__ a, uint64_t i,
                                        const PauliGroup* __restrict__ groups, int ngroups,
                                        const PauliTerm* __restrict__ terms, double& hr,
                                        double& hi_) {
  hr = 0.0;
  hi_ = 0.0;
  for (int g = 0; g < ngroups; ++g) {
    const uint64_t k = i ^ groups[g].x;
    const T b = a[k];
    double wr = 0.0, wi = 0.0;
    const int j1 = groups[g].first + groups[g].count;
    for (int j = groups[g].first; j < j1; ++j) {
      const double sg = parity64(k & terms[j].z) ? -1.0 : 1.0;
      wr += sg * terms[j].cr;
      wi += sg * terms[j].ci;
    }
    const double br = (double)b.x, bi = (double)b.y;
    hr += wr * br - wi * bi;
    hi_ += wr * bi + wi * br;
  }
}

template <typename T, int V>
__global__ void __launch_bounds__(kBlock)
k_expect_pauli(const T* __restrict__ a, uint64_t N, const PauliGroup* __restrict__ groups,
               int ngroups, const PauliTerm* __restrict__ terms, double* __restrict__ part) {
  __shared__ double lds[kBlock / 64];
  double acc = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock * V;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock * V + threadIdx.x; base < N; base += stride) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const uint64_t i = base + (uint64_t)v * kBlock;
      if (i < N) {
        double hr, hi_;
        hpsi_at(a, i, groups, ngroups, terms, hr, hi_);
        const T av = a[i];
        acc += (double)av.x * hr + (double)av.y * hi_;  // Re(conj(a_i) (H psi)_i)
      }
    }
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

template <typename T, int V>
__global__ void __launch_bounds__(kBlock)
k_apply_pauli_sum(const T* __restrict__ a, T* __restrict__ out, uint64_t N,
                  const PauliGroup* __restrict__ groups, int ngroups,
                  const PauliTerm* __restrict__ terms) {
  const uint64_t base = (uint64_t)blockIdx.x * kBlock * V + threadIdx.x;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint64_t i = base + (uint64_t)v * kBlock;
    if (i < N) {
      double hr, hi_;
      hpsi_at(a, i, groups, ngroups, terms, hr, hi_);
      out[i] = make_amp<T>(hr, hi_);
    }
  }
}

// <a|b> partials: re and im per workgroup.
template <typename T, int V>
__global__ void __launch_bounds__(kBlock)
k_inner(const T* __restrict__ a, const T* __restrict__ b, uint64_t N, double* __restrict__ part) {
  __shared__ double lds[kBlock / 64];
  double sr = 0.0, si = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock * V;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock * V + threadIdx.x; base < N; base += stride) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const uint64_t i = base + (uint64_t)v * kBlock;
      if (i < N) {
        const T x = a[i], y = b[i];
        sr += (double)x.x * y.x + (double)x.y * y.y;
        si += (double)x.x * y.y - (double)x.y * y.x;
      }
    }
  }
  sr = block_sum(sr, lds);
  si = block_sum(si, lds);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr;
    part[2 * blockIdx.x + 1] = si;
  }
}

// ------------------------------------------------------------- launchers

static Status last_launch(const char* what) { return hip_status(hipGetLastError(), what); }

static unsigned reduce_grid(uint64_t items, int per_block) {
  const uint64_t g = (items + per_block - 1) / per_block;
  return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(g, kReduceGrid));
}

// Queue the partial-sum pass over the state (partials at `part`, grid rows
// of n + 1) and, when `fin` is given, the fixed-order column sums into
// fin[0 .. n]: P(bit k = 1) for k < n, then the total.
static Status queue_probabilities(StateImpl* s, double* part, double* fin, double* full_dev,
                                  unsigned grid, uint64_t nchunks) {
  const int n = s->n;
  if (s->dtype == QS_C128) {
    if (full_dev)
      hipLaunchKernelGGL((k_probabilities<d2, true>), dim3(grid), dim3(kBlock), 0, s->stream,
                         (const d2*)s->ptr, n, nchunks, part, full_dev);
    else
      hipLaunchKernelGGL((k_probabilities<d2, false>), dim3(grid), dim3(kBlock), 0, s->stream,
                         (const d2*)s->ptr, n, nchunks, part, nullptr);
  } else {
    if (full_dev)
      hipLaunchKernelGGL((k_probabilities_c64<true>), dim3(grid), dim3(kBlock), 0, s->stream,
                         (const f4*)s->ptr, n, nchunks, part, full_dev);
    else
      hipLaunchKernelGGL((k_probabilities_c64<false>), dim3(grid), dim3(kBlock), 0, s->stream,
                         (const f4*)s->ptr, n, nchunks, part, nullptr);
  }
  Status st = last_launch("probabilities");
  if (!st.good() || !fin) return st;
  hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(kBlock), 0, s->stream, part, (int)grid, n + 1,
                     fin);
  return last_launch("probabilities final");
}

// Launch shape of the probabilities pass: chunks of 2^12 (complex128) or
// 2^13 (complex64) amplitudes, at most kReduceGrid workgroups.
static void probabilities_shape(const StateImpl* s, unsigned* grid, uint64_t* nchunks) {
  const uint64_t N = 1ull << s->n;
  const int cl = s->dtype == QS_C128 ? kProbChunkLog : kProbChunkLog + 1;  // log2 amplitudes per chunk
  *nchunks = (N + (1ull << cl) - 1) >> cl;
  *grid = (unsigned)std::min<uint64_t>(*nchunks, kReduceGrid);
}

Status launch_probabilities(StateImpl* s, double* p1_host, double* norm2_host, double* full_dev) {
  const int n = s->n;
  unsigned grid;
  uint64_t nchunks;
  probabilities_shape(s, &grid, &nchunks);
  const size_t ncols = (size_t)n + 1;
  Status st = ensure_dev(s, s->red, (grid * ncols + ncols) * sizeof(double));
  if (!st.good()) return st;
  double* part = (double*)s->red.ptr;
  double* fin = part + grid * ncols;
  const bool sums = p1_host || norm2_host;
  st = queue_probabilities(s, part, sums ? fin : nullptr, full_dev, grid, nchunks);
  if (!st.good() || !sums) return st;
  st = ensure_result_host(s, ncols * sizeof(double));
  if (!st.good()) return st;
  st = hip_status(hipMemcpyAsync(s->result_host, fin, ncols * sizeof(double),
                                 hipMemcpyDeviceToHost, s->stream), "probabilities copy");
  if (!st.good()) return st;
  st = hip_status(hipStreamSynchronize(s->stream), "probabilities sync");
  if (!st.good()) return st;
  if (p1_host)
    for (int k = 0; k < n; ++k) p1_host[k] = s->result_host[k];
  if (norm2_host) *norm2_host = s->result_host[n];
  return Status::ok();
}

// ------------------------------------------------- allocation-free variant
// The partial sums of qs_probabilities_noalloc live in this file-scope
// device array: one copy per GPU, held until the process ends.  In host code
// the name `scratch` is only a host-side stand-in; the device address of
// each GPU's copy is looked up once per device (hipGetSymbolAddress, with
// that device current) and only that address is passed to kernels.
constexpr size_t kNoAllocScratchDoubles = (size_t)kReduceGrid * (kMaxQubits + 1) + (kMaxQubits + 1);
static_assert(kNoAllocScratchDoubles * sizeof(double) == QS_NOALLOC_SCRATCH_BYTES,
              "QS_NOALLOC_SCRATCH_BYTES must match the scratch array");
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kMaxDevices] = {};

static Status scratch_address(int device, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) {
    Status st;
    st.code = QS_ENODEV;
    st.msg = "device index " + std::to_string(device) + " beyond the scratch table";
    return st;
  }
  if (!g_scratch_dev[device]) {
    int cur = -1;
    Status st = hip_status(hipGetDevice(&cur), "scratch: hipGetDevice");
    if (!st.good()) return st;
    if (cur != device) {
      st = hip_status(hipSetDevice(device), "scratch: hipSetDevice");
      if (!st.good()) return st;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    st = hip_status(e, "scratch: hipGetSymbolAddress");
    if (!st.good()) return st;
    if (!ptr) {
      st.code = QS_EHIP;
      st.msg = "scratch: hipGetSymbolAddress returned NULL";
      return st;
    }
    g_scratch_dev[device] = (double*)ptr;
  }
  *out = g_scratch_dev[device];
  return Status::ok();
}

// p1[k] = fin[k] (k < n), norm2 = fin[n]; either output may be absent.
__global__ void k_copy_prob_results(const double* __restrict__ fin, int n, double* __restrict__ p1,
                                    double* __restrict__ norm2) {
  const int k = threadIdx.x;
  if (p1 && k < n) p1[k] = fin[k];
  if (norm2 && k == n) *norm2 = fin[n];
}

Status launch_probabilities_noalloc(StateImpl* s, double* p1_dev, double* norm2_dev,
                                    double* full_dev) {
  const int n = s->n;
  unsigned grid;
  uint64_t nchunks;
  probabilities_shape(s, &grid, &nchunks);
  const size_t ncols = (size_t)n + 1;
  const size_t need = grid * ncols + ncols;
  if (need > kNoAllocScratchDoubles) {
    Status st;
    st.code = QS_ERANGE;
    st.msg = "probabilities need " + std::to_string(need * sizeof(double)) +
             " bytes of scratch, more than the " + std::to_string(QS_NOALLOC_SCRATCH_BYTES) + " held";
    return st;
  }
  double* base = nullptr;
  Status st = scratch_address(s->device, &base);
  if (!st.good()) return st;
  double* part = base;
  double* fin = part + grid * ncols;
  const bool sums = p1_dev || norm2_dev;
  st = queue_probabilities(s, part, sums ? fin : nullptr, full_dev, grid, nchunks);
  if (!st.good() || !sums) return st;
  hipLaunchKernelGGL(k_copy_prob_results, dim3(1), dim3(64), 0, s->stream, fin, n, p1_dev,
                     norm2_dev);
  return last_launch("probabilities results");
}

Status build_pauli_table(int n, int nterms, const uint64_t* x, const uint64_t* z,
                         const double* coeff, PauliTable* out) {
  out->groups.clear();
  out->terms.clear();
  const uint64_t full = (n >= 64) ? ~0ull : ((1ull << n) - 1ull);
  std::map<uint64_t, std::vector<int>> by_x;  // ordered by x: a fixed grouping
  for (int j = 0; j < nterms; ++j) {
    if ((x[j] & ~full) || (z[j] & ~full)) {
      Status s;
      s.code = QS_EINVAL;
      s.msg = "Pauli term " + std::to_string(j) + " acts on a qubit >= n";
      return s;
    }
    by_x[x[j]].push_back(j);
  }
  for (const auto& kv : by_x) {
    PauliGroup g;
    g.x = kv.first;
    g.first = (int32_t)out->terms.size();
    g.count = (int32_t)kv.second.size();
    out->groups.push_back(g);
    for (int j : kv.second) {
      const int ny = __builtin_popcountll(x[j] & z[j]) & 3;
      // i^ny = 1, i, -1, -i
      static const double pr[4] = {1.0, 0.0, -1.0, 0.0};
      static const double pi_[4] = {0.0, 1.0, 0.0, -1.0};
      PauliTerm t;
      t.z = z[j];
      t.cr = coeff[j] * pr[ny];
      t.ci = coeff[j] * pi_[ny];
      out->terms.push_back(t);
    }
  }
  return Status::ok();
}

// Upload groups then terms into the state's table buffer.
static Status upload_pauli(StateImpl* s, const PauliTable& t, const PauliGroup** g,
                           const PauliTerm** tm) {
  const size_t gb = t.groups.size() * sizeof(PauliGroup);
  const size_t tb = t.terms.size() * sizeof(PauliTerm);
  std::vector<char> blob(gb + tb + 16);
  if (gb) memcpy(blob.data(), t.groups.data(), gb);
  if (tb) memcpy(blob.data() + gb, t.terms.data(), tb);
  Status st = upload_table(s, blob.data(), gb + tb);
  if (!st.good()) return st;
  *g = (const PauliGroup*)s->table.ptr;
  *tm = (const PauliTerm*)((char*)s->table.ptr + gb);
  return Status::ok();
}

constexpr int kVR = 2;

Status launch_expect(StateImpl* s, const PauliTable& t, double* out_host) {
  if (t.groups.empty()) {
    *out_host = 0.0;
    return Status::ok();
  }
  const uint64_t N = 1ull << s->n;
  const PauliGroup* g;
  const PauliTerm* tm;
  Status st = upload_pauli(s, t, &g, &tm);
  if (!st.good()) return st;
  const unsigned grid = reduce_grid(N, kBlock * kVR);
  st = ensure_dev(s, s->red, (grid + 1) * sizeof(double));
  if (!st.good()) return st;
  double* part = (double*)s->red.ptr;
  const int ng = (int)t.groups.size();
  if (s->dtype == QS_C128)
    hipLaunchKernelGGL((k_expect_pauli<d2, kVR>), dim3(grid), dim3(kBlock), 0, s->stream,
                       (const d2*)s->ptr, N, g, ng, tm, part);
  else
    hipLaunchKernelGGL((k_expect_pauli<f2, kVR>), dim3(grid), dim3(kBlock), 0, s->stream,
                       (const f2*)s->ptr, N, g, ng, tm, part);
  st = last_launch("expect_pauli");
  if (!st.good()) return st;
  hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(kBlock), 0, s->stream, part, (int)grid, 1,
                     part + grid);
  st = last_launch("expect_pauli final");
  if (!st.good()) return st;
  st = ensure_result_host(s, sizeof(double));
  if (!st.good()) return st;
  st = hip_status(hipMemcpyAsync(s->result_host, part + grid, sizeof(double),
                                 hipMemcpyDeviceToHost, s->stream), "expect copy");
  if (!st.good()) return st;
  st = hip_status(hipStreamSynchronize(s->stream), "expect sync");
  if (!st.good()) return st;
  *out_host = s->result_host[0];
  return Status::ok();
}

Status launch_apply_pauli_sum(StateImpl* src, StateImpl* dst, const PauliTable& t) {
  const uint64_t N = 1ull << src->n;
  const PauliGroup* g;
  const PauliTerm* tm;
  Status st = upload_pauli(src, t, &g, &tm);
  if (!st.good()) return st;
  const int ng = (int)t.groups.size();
  const unsigned grid = (unsigned)((N + kBlock * kVR - 1) / (kBlock * kVR));
  if (src->dtype == QS_C128)
    hipLaunchKernelGGL((k_apply_pauli_sum<d2, kVR>), dim3(grid), dim3(kBlock), 0, src->stream,
                       (const d2*)src->ptr, (d2*)dst->ptr, N, g, ng, tm);
  else
    hipLaunchKernelGGL((k_apply_pauli_sum<f2, kVR>), dim3(grid), dim3(kBlock), 0, src->stream,
                       (const f2*)src->ptr, (f2*)dst->ptr, N, g, ng, tm);
  return last_launch("apply_pauli_sum");
}

Status launch_inner_dev(StateImpl* a, StateImpl* b, double* dev_out) {
  const uint64_t N = 1ull << a->n;
  const unsigned grid = reduce_grid(N, kBlock * kVR);
  Status st = ensure_dev(a, a->red, (2 * grid) * sizeof(double));
  if (!st.good()) return st;
  double* part = (double*)a->red.ptr;
  if (a->dtype == QS_C128)
    hipLaunchKernelGGL((k_inner<d2, kVR>), dim3(grid), dim3(kBlock), 0, a->stream,
                       (const d2*)a->ptr, (const d2*)b->ptr, N, part);
  else
    hipLaunchKernelGGL((k_inner<f2, kVR>), dim3(grid), dim3(kBlock), 0, a->stream,
                       (const f2*)a->ptr, (const f2*)b->ptr, N, part);
  st = last_launch("inner");
  if (!st.good()) return st;
  hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(kBlock), 0, a->stream, part, (int)grid, 2,
                     dev_out);
  return last_launch("inner final");
}

// ------------------------------------------------------------ debug check
// max_i |a_i - b_i| over two states of the same shape (|.| of the complex
// difference, in double precision), one partial per workgroup.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_max_abs_diff(const T* __restrict__ a, const T* __restrict__ b, uint64_t count,
               double* __restrict__ part) {
  __shared__ double lds[kBlock];
  double m = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
    const double dr = (double)a[i].x - (double)b[i].x, di = (double)a[i].y - (double)b[i].y;
    m = fmax(m, sqrt(dr * dr + di * di));
  }
  lds[threadIdx.x] = m;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) lds[threadIdx.x] = fmax(lds[threadIdx.x], lds[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = lds[0];
}

Status max_abs_diff(StateImpl* a, const void* b, double* out_host) {
  const uint64_t count = 1ull << a->n;
  const unsigned grid = (unsigned)std::min<uint64_t>(4096, (count + kBlock - 1) / kBlock);
  Status st = ensure_dev(a, a->red, grid * sizeof(double));
  if (!st.good()) return st;
  double* part = (double*)a->red.ptr;
  if (a->dtype == QS_C128)
    hipLaunchKernelGGL(k_max_abs_diff<d2>, dim3(grid), dim3(kBlock), 0, a->stream, (const d2*)a->ptr,
                       (const d2*)b, count, part);
  else
    hipLaunchKernelGGL(k_max_abs_diff<f2>, dim3(grid), dim3(kBlock), 0, a->stream, (const f2*)a->ptr,
                       (const f2*)b, count, part);
  st = hip_status(hipGetLastError(), "max_abs_diff");
  if (!st.good()) return st;
  std::vector<double> h(grid);
  st = hip_status(hipMemcpyAsync(h.data(), part, grid * sizeof(double), hipMemcpyDeviceToHost, a->stream),
                  "max_abs_diff copy");
  if (!st.good()) return st;
  st = hip_status(hipStreamSynchronize(a->stream), "max_abs_diff sync");
  if (!st.good()) return st;
  double m = 0.0;
  for (double v : h) m = std::max(m, v);
  *out_host = m;
  return Status::ok();
}

}  // namespace qs
