// qs_adjoint.hip -- energy and gradient by the adjoint method.
//
// For E(theta) = <psi_N|H|psi_N>, psi_j = U_j psi_{j-1}, define
// lambda_j = U_{j+1}^dagger ... U_N^dagger H psi_N.  For a rotation
// U_j = exp(-i theta P / 2), dU_j/dtheta = -(i/2) P U_j, hence
//   dE/dtheta_j = 2 Re <lambda_j| -(i/2) P |psi_j> = Im <lambda_j|P|psi_j>.
// One reverse sweep walks j = N..1 carrying (psi_j, lambda_j): it adds
// Im<lambda|P|psi> for rotations and then applies U_j^dagger to both vectors
// (Jones & Gacon, arXiv:2009.02823).  Each reverse step reads and writes two
// state vectors once.
//
// Gradient contributions are double precision for both dtypes: every
// workgroup leaves one partial per rotation in a fixed slot, and the final
// sums add slots in a fixed order (bitwise reproducible).
#include <algorithm>

#include "qs_device.h"
#include "qs_internal.h"

namespace qs {

constexpr int kAdjGrid = 2048;

template <typename R>
Mat<R> to_mat_r(const double* q) {
  Mat<R> m;
  for (int e = 0; e < 4; ++e) {
    m.r[e] = (R)q[2 * e];
    m.i[e] = (R)q[2 * e + 1];
  }
  return m;
}

// Conjugate transpose of a 2x2 in the 8-double layout.
static void dagger(const double* m, double* d) {
  // d11 = conj(m11), d12 = conj(m21), d21 = conj(m12), d22 = conj(m22)
  d[0] = m[0]; d[1] = -m[1];
  d[2] = m[4]; d[3] = -m[5];
  d[4] = m[2]; d[5] = -m[3];
  d[6] = m[6]; d[7] = -m[7];
}

// Reverse step of a rotation on qubit k: gradient partial, then U^dagger on
// psi and lambda.  T is one amplitude (d2 or f2).
template <typename R, typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_rotation(T* __restrict__ psi, T* __restrict__ lam, uint64_t npairs, int k, int pauli,
               Mat<R> udag, double* __restrict__ part) {
  __shared__ double lds[kBlock / 64];
  const uint64_t s = 1ull << k;
  double acc = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x; p < npairs; p += stride) {
    const uint64_t i0 = insert0(p, k), i1 = i0 + s;
    T a0 = psi[i0], a1 = psi[i1], l0 = lam[i0], l1 = lam[i1];
    acc += pair_grad(pauli, a0.x, a0.y, a1.x, a1.y, l0.x, l0.y, l1.x, l1.y);
    pair_apply(udag, a0, a1);
    pair_apply(udag, l0, l1);
    psi[i0] = a0;
    psi[i1] = a1;
    lam[i0] = l0;
    lam[i1] = l1;
  }
  acc = block_sum(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Reverse step of a fixed gate: U^dagger on both vectors (controlled when
// c >= 0).
template <typename R, typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_fixed(T* __restrict__ psi, T* __restrict__ lam, uint64_t nitems, int c, int t, Mat<R> udag) {
  const uint64_t s = 1ull << t;
  const uint64_t p = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= nitems) return;
  uint64_t i0;
  if (c >= 0) {
    const int lo = c < t ? c : t, hi = c < t ? t : c;
    i0 = insert0(insert0(p, lo), hi) | (1ull << c);
  } else {
    i0 = insert0(p, t);
  }
  T a0 = psi[i0], a1 = psi[i0 + s], l0 = lam[i0], l1 = lam[i0 + s];
  pair_apply(udag, a0, a1);
  pair_apply(udag, l0, l1);
  psi[i0] = a0;
  psi[i0 + s] = a1;
  lam[i0] = l0;
  lam[i0 + s] = l1;
}

// out[r] = sum over c of part[r * ncols + c] (fixed order); one workgroup per row.
__global__ void __launch_bounds__(kBlock)
k_sum_rows(const double* __restrict__ part, int ncols, double* __restrict__ out) {
  __shared__ double lds[kBlock / 64];
  const double* row = part + (size_t)blockIdx.x * ncols;
  double s = 0.0;
  for (int c = threadIdx.x; c < ncols; c += kBlock) s += row[c];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

static Status last_launch(const char* what) { return hip_status(hipGetLastError(), what); }

Status launch_sum_rows(StateImpl* s, const double* part, int nrows, int ncols, double* out) {
  hipLaunchKernelGGL(k_sum_rows, dim3(nrows), dim3(kBlock), 0, s->stream, part, ncols, out);
  return last_launch("sum rows");
}

// Unfused reverse sweep (states smaller than one fused tile): one launch per
// gate; rotation r (in reverse order) leaves its partials in row r.
template <typename R, typename T>
static Status reverse_sweep(StateImpl* s, StateImpl* lam, const std::vector<XGate>& gates,
                            double* part, int grid) {
  const int n = s->n;
  int r = 0;
  for (int g = (int)gates.size() - 1; g >= 0; --g) {
    const XGate& x = gates[g];
    double d[8];
    dagger(x.m, d);
    const Mat<R> m = to_mat_r<R>(d);
    if (x.kind == QS_OP_RX || x.kind == QS_OP_RY || x.kind == QS_OP_RZ) {
      const uint64_t np = 1ull << (n - 1);
      const int pauli = x.kind - QS_OP_RX + 1;
      hipLaunchKernelGGL((k_adj_rotation<R, T>), dim3(grid), dim3(kBlock), 0, s->stream,
                         (T*)s->ptr, (T*)lam->ptr, np, x.target, pauli, m,
                         part + (size_t)r * grid);
      ++r;
    } else {
      const uint64_t items = 1ull << (n - (x.control >= 0 ? 2 : 1));
      hipLaunchKernelGGL((k_adj_fixed<R, T>), dim3((unsigned)((items + kBlock - 1) / kBlock)),
                         dim3(kBlock), 0, s->stream, (T*)s->ptr, (T*)lam->ptr, items, x.control,
                         x.target, m);
    }
    Status st = last_launch("adjoint step");
    if (!st.good()) return st;
  }
  return Status::ok();
}

void reverse_daggered(const std::vector<XGate>& gates, std::vector<XGate>* rev) {
  rev->clear();
  rev->reserve(gates.size());
  for (int g = (int)gates.size() - 1; g >= 0; --g) {
    XGate x = gates[g];
    dagger(gates[g].m, x.m);
    rev->push_back(x);
  }
}

Status run_adjoint(StateImpl* s, StateImpl* lam, const std::vector<XGate>& gates, int nparams,
                   const PauliTable& h, int flags, double* energy, double* grad) {
  Status st;
  const bool wide = (flags & QS_ADJ_WIDE_TILES) != 0;
  if (!(flags & QS_ADJ_STATE_IS_FINAL)) {
    st = run_gates(s, gates, wide ? QS_RUN_WIDE_TILES : 0);
    if (!st.good()) return st;
  }
  // lambda = H psi_N, queued on the state's stream.
  StateImpl lam_on_s = *lam;
  lam_on_s.stream = s->stream;
  st = launch_apply_pauli_sum(s, &lam_on_s, h);
  if (!st.good()) return st;
  // E = Re<psi_N|H psi_N> into the handle's small-result buffer.
  st = ensure_dev(s, s->scal, 4 * sizeof(double));
  if (!st.good()) return st;
  double* ev = (double*)s->scal.ptr;
  st = launch_inner_dev(s, &lam_on_s, ev);
  if (!st.good()) return st;

  // Reverse sweep: rows[i] is the gradient row (parameter) of sums[i].
  std::vector<int> rows;
  double* sums = nullptr;
  if (s->n >= fuse_geom(s->dtype).T) {
    std::vector<XGate> rev;
    reverse_daggered(gates, &rev);
    st = run_adjoint_fused(s, &lam_on_s, rev, &rows, &sums, wide);
    if (!st.good()) return st;
  } else {
    for (int g = (int)gates.size() - 1; g >= 0; --g)
      if (gates[g].kind >= QS_OP_RX) rows.push_back(gates[g].param);
    const int nrot = (int)rows.size();
    const uint64_t npairs = 1ull << (s->n - 1);
    const int grid =
        (int)std::max<uint64_t>(1, std::min<uint64_t>(kAdjGrid, (npairs + kBlock - 1) / kBlock));
    st = ensure_dev(s, s->red, ((size_t)nrot * grid + nrot + 2) * sizeof(double));
    if (!st.good()) return st;
    double* part = (double*)s->red.ptr;
    sums = part + (size_t)nrot * grid;
    if (s->dtype == QS_C128)
      st = reverse_sweep<double, d2>(s, &lam_on_s, gates, part, grid);
    else
      st = reverse_sweep<float, f2>(s, &lam_on_s, gates, part, grid);
    if (!st.good()) return st;
    if (nrot > 0) {
      st = launch_sum_rows(s, part, nrot, grid, sums);
      if (!st.good()) return st;
    }
  }
  const size_t nrows = rows.size();
  st = ensure_result_host(s, (nrows + 2) * sizeof(double));
  if (!st.good()) return st;
  if (nrows > 0) {
    st = hip_status(hipMemcpyAsync(s->result_host, sums, nrows * sizeof(double),
                                   hipMemcpyDeviceToHost, s->stream), "adjoint copy");
    if (!st.good()) return st;
  }
  st = hip_status(hipMemcpyAsync(s->result_host + nrows, ev, 2 * sizeof(double),
                                 hipMemcpyDeviceToHost, s->stream), "energy copy");
  if (!st.good()) return st;
  st = hip_status(hipStreamSynchronize(s->stream), "adjoint sync");
  if (!st.good()) return st;
  if (energy) *energy = s->result_host[nrows];
  for (int p = 0; p < nparams; ++p) grad[p] = 0.0;
  for (size_t i = 0; i < nrows; ++i) grad[rows[i]] += s->result_host[i];
  return Status::ok();
}

}  // namespace qs
