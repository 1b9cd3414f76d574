// qs_device.h -- device-side helpers shared by the libqs kernels (gfx950).
//
// Amplitudes are interleaved (re, im): double2 for complex128, float2 for
// complex64; two complex64 amplitudes are moved as one float4 so that every
// lane issues 16-byte global accesses.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qs {

constexpr int kBlock = 256;  // threads per workgroup of the streaming kernels (4 wave64)

// A 2x2 complex matrix in compute precision R: q11, q12, q21, q22.
template <typename R>
struct Mat {
  R r[4];
  R i[4];
};

// out = Q (x, y): one application of Eq. (2) to the amplitude pair (x, y).
template <typename R>
__device__ __forceinline__ void mat_apply(const Mat<R>& q, R& xr, R& xi, R& yr, R& yi) {
  const R ar = q.r[0] * xr - q.i[0] * xi + q.r[1] * yr - q.i[1] * yi;
  const R ai = q.r[0] * xi + q.i[0] * xr + q.r[1] * yi + q.i[1] * yr;
  const R br = q.r[2] * xr - q.i[2] * xi + q.r[3] * yr - q.i[3] * yi;
  const R bi = q.r[2] * xi + q.i[2] * xr + q.r[3] * yi + q.i[3] * yr;
  xr = ar;
  xi = ai;
  yr = br;
  yi = bi;
}

// Native vector types used for 16-byte (and 8-byte) global/LDS accesses.
typedef double d2 __attribute__((ext_vector_type(2)));   // one complex128 amplitude
typedef float f2 __attribute__((ext_vector_type(2)));    // one complex64 amplitude
typedef float f4 __attribute__((ext_vector_type(4)));    // two complex64 amplitudes
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void pair_apply(const Mat<double>& q, d2& x, d2& y) {
  double xr = x.x, xi = x.y, yr = y.x, yi = y.y;
  mat_apply(q, xr, xi, yr, yi);
  x = d2{xr, xi};
  y = d2{yr, yi};
}
__device__ __forceinline__ void pair_apply(const Mat<float>& q, f2& x, f2& y) {
  float xr = x.x, xi = x.y, yr = y.x, yi = y.y;
  mat_apply(q, xr, xi, yr, yi);
  x = f2{xr, xi};
  y = f2{yr, yi};
}
// Two complex64 pairs side by side: (x.xy, y.xy) and (x.zw, y.zw).
__device__ __forceinline__ void pair_apply(const Mat<float>& q, f4& x, f4& y) {
  float ar = x.x, ai = x.y, br = y.x, bi = y.y;
  float cr = x.z, ci = x.w, dr = y.z, di = y.w;
  mat_apply(q, ar, ai, br, bi);
  mat_apply(q, cr, ci, dr, di);
  x = f4{ar, ai, cr, ci};
  y = f4{br, bi, dr, di};
}
// A complex64 pair held in one vector: (v.xy, v.zw).
__device__ __forceinline__ void pair_apply_inner(const Mat<float>& q, f4& v) {
  float ar = v.x, ai = v.y, br = v.z, bi = v.w;
  mat_apply(q, ar, ai, br, bi);
  v = f4{ar, ai, br, bi};
}

// Butterfly partner exchange inside a wavefront (lane ^ m).
__device__ __forceinline__ d2 shfl_xor_unit(d2 v, int m) {
  return d2{__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64)};
}
__device__ __forceinline__ f4 shfl_xor_unit(f4 v, int m) {
  return f4{__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64), __shfl_xor(v.z, m, 64),
            __shfl_xor(v.w, m, 64)};
}

// o = a * x + b * y for complex a, b, x, y.
template <typename R>
__device__ __forceinline__ void cmadd(R ar, R ai, R br, R bi, R xr, R xi, R yr, R yi, R& orr,
                                      R& oi) {
  orr = ar * xr - ai * xi + br * yr - bi * yi;
  oi = ar * xi + ai * xr + br * yi + bi * yr;
}

// Coefficients of one output row of Q for a lane that holds one member of a
// pair: the lane with the target bit clear computes q11 x + q12 y, the lane
// with it set computes q21 y + q22 x (x = own amplitude, y = partner's).
template <typename R>
struct Row {
  R own_r, own_i, par_r, par_i;
};
template <typename R>
__device__ __forceinline__ Row<R> row_for(const Mat<R>& q, bool hi) {
  Row<R> w;
  w.own_r = hi ? q.r[3] : q.r[0];
  w.own_i = hi ? q.i[3] : q.i[0];
  w.par_r = hi ? q.r[2] : q.r[1];
  w.par_i = hi ? q.i[2] : q.i[1];
  return w;
}
__device__ __forceinline__ d2 row_apply(const Row<double>& w, d2 x, d2 y) {
  double o_r, o_i;
  cmadd(w.own_r, w.own_i, w.par_r, w.par_i, x.x, x.y, y.x, y.y, o_r, o_i);
  return d2{o_r, o_i};
}
__device__ __forceinline__ f4 row_apply(const Row<float>& w, f4 x, f4 y) {
  float ar, ai, br, bi;
  cmadd(w.own_r, w.own_i, w.par_r, w.par_i, x.x, x.y, y.x, y.y, ar, ai);
  cmadd(w.own_r, w.own_i, w.par_r, w.par_i, x.z, x.w, y.z, y.w, br, bi);
  return f4{ar, ai, br, bi};
}
// Only the odd amplitude of each complex64 unit (control qubit 0 set).
__device__ __forceinline__ f4 row_apply_odd(const Row<float>& w, f4 x, f4 y) {
  float br, bi;
  cmadd(w.own_r, w.own_i, w.par_r, w.par_i, x.z, x.w, y.z, y.w, br, bi);
  return f4{x.x, x.y, br, bi};
}
// Pair update of the odd amplitudes only (x.zw, y.zw).
__device__ __forceinline__ void pair_apply_odd(const Mat<float>& q, f4& x, f4& y) {
  float cr = x.z, ci = x.w, dr = y.z, di = y.w;
  mat_apply(q, cr, ci, dr, di);
  x = f4{x.x, x.y, cr, ci};
  y = f4{y.x, y.y, dr, di};
}

// Im(conj(l) * w)
__device__ __forceinline__ double im_conj_mul(double lr, double li, double wr, double wi) {
  return lr * wi - li * wr;
}

// Im<lambda|P|psi> restricted to one amplitude pair (target bit 0 / 1),
// P = X (1), Y (2) or Z (3), in double precision.  All three are computed
// and the result is selected: the switch form of this function was lowered
// incorrectly by the gfx950 backend of this toolchain when inlined into a
// loop (the Z case read registers of another case), while the select form
// compiles to straight-line code.
__device__ __forceinline__ double pair_grad(int pauli, double a0r, double a0i, double a1r,
                                            double a1i, double l0r, double l0i, double l1r,
                                            double l1i) {
  // X psi = (a1, a0); Y psi = (-i a1, i a0); Z psi = (a0, -a1)
  const double gx = im_conj_mul(l0r, l0i, a1r, a1i) + im_conj_mul(l1r, l1i, a0r, a0i);
  const double gy = im_conj_mul(l0r, l0i, a1i, -a1r) + im_conj_mul(l1r, l1i, -a0i, a0r);
  const double gz = im_conj_mul(l0r, l0i, a0r, a0i) + im_conj_mul(l1r, l1i, -a1r, -a1i);
  const double gxy = pauli == 1 ? gx : gy;
  return pauli <= 2 ? gxy : gz;
}

// An amplitude of the storage type from double-precision parts.
template <typename T>
__device__ __forceinline__ T make_amp(double re, double im);
template <>
__device__ __forceinline__ d2 make_amp<d2>(double re, double im) { return d2{re, im}; }
template <>
__device__ __forceinline__ f2 make_amp<f2>(double re, double im) {
  return f2{(float)re, (float)im};
}

// Global loads/stores, optionally marked non-temporal (streamed through the
// caches without being kept: the state is far larger than L2 + MALL).
template <bool NT, typename T>
__device__ __forceinline__ T gload(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void gstore(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Index p with a 0 bit inserted at position k (bits >= k move up by one).
__device__ __forceinline__ uint64_t insert0(uint64_t p, int k) {
  const uint64_t lo = p & ((1ull << k) - 1ull);
  return ((p ^ lo) << 1) | lo;
}

// Deterministic wavefront (64-lane) sum by butterfly exchange; every lane
// ends with the same value, added in the same order on every run.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic workgroup sum for kBlock threads; `lds` needs kBlock/64
// doubles.  Every thread receives the result.  Contains barriers: call from
// uniform control flow only.
__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kBlock / 64; ++j) s += lds[j];
  return s;
}

__device__ __forceinline__ int parity64(uint64_t v) { return __popcll(v) & 1; }

}  // namespace qs
