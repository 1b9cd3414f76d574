// qs_gates.hip -- streaming gate kernels: one pass over the state per gate.
//
// Single-qubit gate (qHiPSTER Eq. 2) and controlled gate (Eq. 3), written
// for 64-wide wavefronts and 16-byte accesses instead of the paper's
// two-level loop nest (Fig. 2).
//
// Units.  Every lane moves one 16-byte "unit": a complex128 amplitude, or two
// adjacent complex64 amplitudes.  Unit bit j is qubit j (complex128) or qubit
// j + 1 (complex64); complex64 qubit 0 lies inside a unit.
//
// Three access shapes, picked per gate from its qubits:
//   * exchange (single-qubit target unit bit < 7, controlled < 8): a
//     workgroup reads consecutive units, one per lane; each lane fetches its
//     partner from lane ^ 2^t with a cross-lane shuffle (bit < 6, same
//     wavefront) or through LDS (bits 6, 7), so both members of every pair
//     arrive in one contiguous access;
//   * paired streams (higher targets): lane p handles the pair
//     (i0, i0 + 2^t), i0 = p with a 0 inserted at bit t; consecutive lanes
//     read two contiguous 1 KiB runs;
//   * in-unit (complex64 target qubit 0): each unit holds a whole pair.
// Controls (Eq. 3): when the control's runs of 1s are at least one 128-byte
// line long (control unit bit >= 3) only control-1 units are enumerated
// ("compact"): half the state is neither read nor written, Table 2 case 3.
// Below that, a line mixes control-0 and control-1 amplitudes; the whole
// line is read anyway, so the kernel reads every unit and writes every unit
// back (unchanged where the control is 0), which streams full lines instead
// of scattering half-line accesses.
//
// Launch shape: 16 bytes per lane per stream, 64-lane workgroups for the
// paired-stream kernel and the shuffle exchange (256 lanes for the LDS
// exchange and for launches too large for a one-shot grid), grid-stride
// loops with the grid capped so the dispatch never exceeds 2^31 work-items.
// The paired streams run with an occupancy cap (fewer workgroups in flight
// measured faster on HBM).  Workgroups are dispatched to the 8 XCDs
// round-robin; for some strides the paired-stream kernel is faster when
// each XCD walks one contiguous eighth of the work ("XCD-contiguous"
// order).  The dispatch rules below come from measured sweeps.
#include <algorithm>
#include <cstdlib>

#include "qs_device.h"
#include "qs_internal.h"

namespace qs {

enum CtrlMode { kNone = 0, kCompact = 1, kPred = 2, kInnerCtrl = 3 };

constexpr bool kNT = true;  // non-temporal global accesses (the state >> L2 + MALL)
constexpr int kShflBits = 6;  // lane bits of a wave64
constexpr int kLineUnitBits = 3;  // 128-byte line = 8 units
constexpr int kPairBlock = 64;
constexpr int kShflBlock = 256;
constexpr int kShflWave = 64;  // one-wave workgroups for the shuffle exchange

// Logical workgroup index.  MAP 0: as dispatched.  MAP 1: XCD-contiguous --
// dispatch slot b runs on XCD b % 8, so logical block (b % 8) * (G / 8) +
// b / 8 makes each XCD walk a contiguous eighth; a tail of G % 8 blocks keeps
// its own index (the map stays a permutation of 0..G-1).
template <int MAP>
__device__ __forceinline__ uint64_t logical_block() {
  const uint64_t b = blockIdx.x;
  if constexpr (MAP == 1) {
    const uint64_t per = gridDim.x / 8;
    if (b < per * 8) return (b % 8) * per + b / 8;
  }
  return b;
}

// ------------------------------------------------------------- paired streams
// count work items: kNone / kPred / kInnerCtrl: 2^(u-1) pairs of target t;
// kCompact: 2^(u-2) control-1 pairs (0s inserted at c and t, then bit c set).
template <typename R, typename T, int B, int CM, int MAP>
__global__ void __launch_bounds__(B)
k_pair(T* __restrict__ a, uint64_t count, int t, int c, Mat<R> q) {
  const uint64_t s = 1ull << t;
  const uint64_t stride = (uint64_t)gridDim.x * B;
  const int lo = c < t ? c : t, hi = c < t ? t : c;
  for (uint64_t p = logical_block<MAP>() * B + threadIdx.x; p < count; p += stride) {
    uint64_t i0;
    if constexpr (CM == kCompact) i0 = insert0(insert0(p, lo), hi) | (1ull << c);
    else i0 = insert0(p, t);
    T x = gload<kNT>(a + i0), y = gload<kNT>(a + i0 + s);
    if constexpr (CM == kPred) {
      if ((i0 >> c) & 1) pair_apply(q, x, y);
    } else if constexpr (CM == kInnerCtrl) {
      pair_apply_odd(q, x, y);
    } else {
      pair_apply(q, x, y);
    }
    gstore<kNT>(a + i0, x);
    gstore<kNT>(a + i0 + s, y);
  }
}

// ----------------------------------------------------------------- exchange
// t is the target's bit in the work index j (< 8).  count work items:
// kNone / kPred / kInnerCtrl: all 2^u units; kCompact: the 2^(u-1) units with
// bit c set (unit = j with a 1 inserted at bit c).  LDS = false: partner by
// wavefront shuffle (t < 6); LDS = true: partner through shared memory
// (t = 6, 7).  The loop trip count is uniform over the workgroup (barriers).
template <typename R, typename T, int B, int CM, bool LDS>
__global__ void __launch_bounds__(B)
k_exchange(T* __restrict__ a, uint64_t count, int t, int c, Mat<R> q) {
  __shared__ T buf[LDS ? B : 1];
  const int m = 1 << t;
  const Row<R> w = row_for(q, (threadIdx.x >> t) & 1);
  const uint64_t stride = (uint64_t)gridDim.x * B;
  for (uint64_t base = (uint64_t)blockIdx.x * B; base < count; base += stride) {
    const uint64_t j = base + threadIdx.x;
    const bool live = j < count;
    uint64_t u;
    if constexpr (CM == kCompact) u = insert0(j, c) | (1ull << c);
    else u = j;
    T x{};
    if (live) x = gload<kNT>(a + u);
    T y;
    if constexpr (LDS) {
      buf[threadIdx.x] = x;
      __syncthreads();
      y = buf[threadIdx.x ^ m];
      __syncthreads();
    } else {
      y = shfl_xor_unit(x, m);
    }
    T o;
    if constexpr (CM == kInnerCtrl) o = row_apply_odd(w, x, y);
    else o = row_apply(w, x, y);
    if constexpr (CM == kPred) o = ((u >> c) & 1) ? o : x;
    if (live) gstore<kNT>(a + u, o);
  }
}

// ---------------------------------------------------- complex64, qubit 0
// Each unit is a pair.  kNone: all 2^u units; kCompact: 2^(u-1) units with
// unit bit c set; kPred: all units, updated where unit bit c is set.
template <int B, int CM>
__global__ void __launch_bounds__(B)
k_inner(f4* __restrict__ a, uint64_t count, int c, Mat<float> q) {
  const uint64_t stride = (uint64_t)gridDim.x * B;
  for (uint64_t j = (uint64_t)blockIdx.x * B + threadIdx.x; j < count; j += stride) {
    uint64_t u;
    if constexpr (CM == kCompact) u = insert0(j, c) | (1ull << c);
    else u = j;
    f4 x = gload<kNT>(a + u);
    if constexpr (CM == kPred) {
      if ((u >> c) & 1) pair_apply_inner(q, x);
    } else {
      pair_apply_inner(q, x);
    }
    gstore<kNT>(a + u, x);
  }
}

// ----------------------------------------------------------- |index> init
// 16-byte zeros everywhere, `one` at the unit holding amplitude `index`.
template <int B>
__global__ void __launch_bounds__(B)
k_init_basis(u64x2* __restrict__ a, uint64_t nvec, uint64_t one_vec, u64x2 one) {
  const uint64_t stride = (uint64_t)gridDim.x * B;
  for (uint64_t j = (uint64_t)blockIdx.x * B + threadIdx.x; j < nvec; j += stride)
    gstore<kNT>(a + j, (j == one_vec) ? one : u64x2{0ull, 0ull});
}

// STREAM "copy" (dst[i] = src[i]) over 16-byte words: the sustainable memory
// bandwidth B_mem that the paper's lower bounds divide by (Sec. 5.2).
template <int B>
__global__ void __launch_bounds__(B)
k_stream_copy(const u64x2* __restrict__ src, u64x2* __restrict__ dst, uint64_t nwords) {
  const uint64_t stride = (uint64_t)gridDim.x * B;
  for (uint64_t i = (uint64_t)blockIdx.x * B + threadIdx.x; i < nwords; i += stride)
    gstore<kNT>(dst + i, gload<kNT>(src + i));
}

// ------------------------------------------------------------------ phases
// A phase gate diag(1, phi) on qubit k, or its controlled form, changes only
// the amplitudes whose bits in `mask` (the target, and the control) are all
// 1: a quarter of the state under a control, half without.  Work item p is
// the index with ones inserted at the mask positions lo < hi (hi < 0: one
// position), so consecutive items stay consecutive above the mask bits.
template <typename R, typename T, int B>
__global__ void __launch_bounds__(B)
k_phase(T* __restrict__ a, uint64_t count, int lo, int hi, R pr, R pi) {
  const uint64_t stride = (uint64_t)gridDim.x * B;
  for (uint64_t p = (uint64_t)blockIdx.x * B + threadIdx.x; p < count; p += stride) {
    uint64_t i = insert0(p, lo) | (1ull << lo);
    if (hi >= 0) i = insert0(i, hi) | (1ull << hi);
    T v = gload<kNT>(a + i);
    const R vr = v.x, vi = v.y;
    v.x = pr * vr - pi * vi;
    v.y = pr * vi + pi * vr;
    gstore<kNT>(a + i, v);
  }
}

// q is exactly diag(1, phi).
static bool is_phase(const double* q) {
  return q[0] == 1.0 && q[1] == 0.0 && q[2] == 0.0 && q[3] == 0.0 && q[4] == 0.0 && q[5] == 0.0;
}

static void go_phase(StateImpl* s, int lo, int hi, const double* q);

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

// Grid for `items` work items, capped at 2^31 work-items per dispatch.
static unsigned grid_for(uint64_t items, int block) {
  const uint64_t want = (items + block - 1) / block;
  const uint64_t cap = (1ull << 31) / (uint64_t)block;
  return (unsigned)std::max<uint64_t>(1, std::min(want, cap));
}

Status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return Status::ok();
  Status s;
  s.code = QS_EHIP;
  s.msg = std::string(what) + ": " + hipGetErrorString(e);
  return s;
}

static Status last_launch(const char* what) { return hip_status(hipGetLastError(), what); }

// Occupancy cap of the streaming gate kernels, in waves per SIMD (0: none),
// applied as dynamic LDS that no kernel reads: a workgroup of `block`
// threads that already holds `static_lds` bytes gets enough more that at
// most the capped number of workgroups share a CU's 160 KiB.  Fewer
// workgroups in flight measured faster on the paired streams (fewer DRAM
// rows open at once), by 3-13 % at most targets; the exchange kernels
// (targets below unit bit 8, 256-thread workgroups) measured slower with
// any cap and run uncapped.  QS_STREAM_WAVES, when set, replaces the cap of
// every streaming launch (0: none), to measure it.
constexpr size_t kCuLds = 160 * 1024;
size_t stream_lds(int block, size_t static_lds, int waves) {
  if (const char* e = getenv("QS_STREAM_WAVES"))
    if (*e) waves = atoi(e);
  if (waves <= 0) return 0;
  const int wg_waves = (block + 63) / 64;
  const int wgs = std::max(1, (waves * 4) / wg_waves);  // 4 SIMDs per CU
  // 512-byte allocation granules; at most 64 KiB per workgroup
  const size_t per = std::min<size_t>(kCuLds / (size_t)wgs, 64 * 1024) & ~(size_t)511;
  return per > static_lds ? per - static_lds : 0;
}

template <typename R, typename T, int CM, int MAP>
static void go_pair(StateImpl* s, uint64_t count, int t, int c, const Mat<R>& q, int waves) {
  hipLaunchKernelGGL((k_pair<R, T, kPairBlock, CM, MAP>), dim3(grid_for(count, kPairBlock)),
                     dim3(kPairBlock), stream_lds(kPairBlock, 0, waves), s->stream, (T*)s->ptr, count, t, c, q);
}
// Whether `count` work items fit one-wave workgroups in a one-shot grid (no
// grid-stride iterations: grid_for caps a launch at 2^31 work items).  The
// shuffle exchange and the complex64 qubit-0 kernel then run one-wave
// workgroups, which measured 4-5 % faster than 256-thread ones at 2^28-2^31
// work items (two or four units per thread, and any occupancy cap,
// measured slower); with grid-stride iterations they measured slower, so
// larger launches keep 256 threads.  The LDS exchange needs its partner
// wave in the workgroup.
static bool one_wave_groups(uint64_t count) { return count <= (1ull << 31); }

// Exchange kernel; t is the target's bit in the work index (< 8).
template <typename R, typename T, int CM>
static void go_exchange(StateImpl* s, uint64_t count, int t, int c, const Mat<R>& q) {
  if (t < kShflBits && one_wave_groups(count))
    hipLaunchKernelGGL((k_exchange<R, T, kShflWave, CM, false>), dim3(grid_for(count, kShflWave)),
                       dim3(kShflWave), stream_lds(kShflWave, 0, 0), s->stream, (T*)s->ptr, count, t, c, q);
  else if (t < kShflBits)
    hipLaunchKernelGGL((k_exchange<R, T, kShflBlock, CM, false>), dim3(grid_for(count, kShflBlock)),
                       dim3(kShflBlock), stream_lds(kShflBlock, 0, 0), s->stream, (T*)s->ptr, count, t, c, q);
  else
    hipLaunchKernelGGL((k_exchange<R, T, kShflBlock, CM, true>), dim3(grid_for(count, kShflBlock)),
                       dim3(kShflBlock), stream_lds(kShflBlock, kShflBlock * sizeof(T), 0), s->stream, (T*)s->ptr,
                       count, t, c, q);
}
template <int CM>
static void go_inner(StateImpl* s, uint64_t count, int c, const Mat<float>& q) {
  if (one_wave_groups(count))
    hipLaunchKernelGGL((k_inner<kShflWave, CM>), dim3(grid_for(count, kShflWave)),
                       dim3(kShflWave), stream_lds(kShflWave, 0, 0), s->stream, (f4*)s->ptr, count, c, q);
  else
    hipLaunchKernelGGL((k_inner<kShflBlock, CM>), dim3(grid_for(count, kShflBlock)),
                       dim3(kShflBlock), stream_lds(kShflBlock, 0, 0), s->stream, (f4*)s->ptr, count, c, q);
}

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
  hipLaunchKernelGGL((k_init_basis<kShflBlock>), dim3(grid_for(nvec, kShflBlock)),
                     dim3(kShflBlock), 0, s->stream, (u64x2*)s->ptr, nvec, one_vec, one);
  return last_launch("init_basis");
}

// Dispatch rules below were chosen from a measured sweep of every target
// (and a grid of control/target pairs) at n = 30 on MI355X.
constexpr int kExchangeBits = 8;  // target bits handled inside a 256-lane workgroup

// Block order and occupancy cap of the paired-stream kernel for a
// single-qubit gate on unit bit t (>= 7) of a 2^u-unit state (units of 16
// bytes: complex128 amplitudes, complex64 pairs).  From a sweep of every
// target over both block orders (plain, or consecutive blocks spread over
// the XCDs) and caps of none, 3 and 4 waves per SIMD at u = 30..33, with
// the u = 30 results repeated at complex64 (which agreed in unit bits):
// three waves per SIMD in the plain order is best or within 1 % nearly
// everywhere; four is 2-3 % better at bits 18-19 and 25-28 up to u = 32;
// the spread order is better at bits 20-22 (20-23 at u = 33), the pair
// distances of 16-128 MiB where the plain order dips most.
static int pair_block_order(int u, int t) {
  if (u >= 33) return (t >= 20 && t <= 23) ? 1 : 0;
  return (t >= 20 && t <= 22) ? 1 : 0;
}
static int pair_waves_1q(int u, int t) {
  if (u >= 33) return 3;
  return (t == 18 || t == 19 || (t >= 25 && t <= 28)) ? 4 : 3;
}
// Controlled gates on the paired streams: three waves per SIMD measured
// faster at most (control, target) pairs of a sweep (up to 21 % with the
// control inside a line, 4-11 % outside).
constexpr int kPairWavesCU = 3;

// QS_1Q_BLOCK_ORDER (0 or 1), when set, forces the block order of the
// paired-stream kernel for every target (to measure both); otherwise
// pair_block_order decides.
static int block_order_env() {
  const char* e = getenv("QS_1Q_BLOCK_ORDER");
  if (!e || !*e) return -1;
  return atoi(e) ? 1 : 0;
}

// Single-qubit gate on unit bit t of a 2^u-unit state.
template <typename R, typename T>
static void units_1q(StateImpl* s, int u, int t, const Mat<R>& q) {
  // unit bit 7 (pair distance 2 KiB) measured 3-4 % faster on the capped
  // paired streams than through the LDS exchange
  if (t < kExchangeBits - 1) {
    go_exchange<R, T, kNone>(s, 1ull << u, t, 0, q);
    return;
  }
  const int forced = block_order_env();
  const int w = pair_waves_1q(u, t);
  if ((forced >= 0 ? forced : pair_block_order(u, t)) == 1) go_pair<R, T, kNone, 1>(s, 1ull << (u - 1), t, 0, q, w);
  else go_pair<R, T, kNone, 0>(s, 1ull << (u - 1), t, 0, q, w);
}

// QS_CU_COMPACT_FROM (0..3), when set, is the lowest control unit bit that
// takes the compact enumeration, replacing the rule below; it exists to
// measure the compact pass over control-1 runs shorter than a line against
// the predicated one.
static int compact_from_env() {
  const char* e = getenv("QS_CU_COMPACT_FROM");
  if (!e || !*e) return -1;
  const int x = atoi(e);
  return x < 0 ? 0 : x > kLineUnitBits ? kLineUnitBits : x;
}

// Whether a controlled gate with control unit bit c and target unit bit t
// takes the compact enumeration.  From a full 128-byte line of control-1
// units up it always does (half the traffic).  Below the line the memory
// side still fetches whole lines, so the compact pass moves as many read
// bytes as the predicated one; with 64-byte runs (unit bit 2) it writes
// half and measured 7-12 % faster for target unit bits 12-23, slower or
// equal elsewhere; with 16- or 32-byte runs it is a third slower.
static bool cu_compact(int c, int t) {
  const int from = compact_from_env();
  if (from >= 0) return c >= from;
  return c >= kLineUnitBits || (c == kLineUnitBits - 1 && t >= 12 && t <= 23);
}

// Controlled gate, control unit bit c, target unit bit t, 2^u units.
template <typename R, typename T>
static void units_cu(StateImpl* s, int u, int c, int t, const Mat<R>& q) {
  const bool compact = cu_compact(c, t);
  if (t < kExchangeBits) {
    if (compact) go_exchange<R, T, kCompact>(s, 1ull << (u - 1), t < c ? t : t - 1, c, q);
    else go_exchange<R, T, kPred>(s, 1ull << u, t, c, q);
  } else if (compact) {
    if (c < kExchangeBits) go_pair<R, T, kCompact, 1>(s, 1ull << (u - 2), t, c, q, kPairWavesCU);
    else go_pair<R, T, kCompact, 0>(s, 1ull << (u - 2), t, c, q, kPairWavesCU);
  } else {
    go_pair<R, T, kPred, 0>(s, 1ull << (u - 1), t, c, q, kPairWavesCU);
  }
}

// Phase gates run with an occupancy cap of six waves per SIMD (2.5-3 %
// faster than uncapped over 1q and controlled phases; three or four slower).
static void go_phase(StateImpl* s, int lo, int hi, const double* q) {
  const uint64_t count = 1ull << (s->n - (hi >= 0 ? 2 : 1));
  if (s->dtype == QS_C128)
    hipLaunchKernelGGL((k_phase<double, d2, kBlock>), dim3(grid_for(count, kBlock)), dim3(kBlock), stream_lds(kBlock, 0, 6),
                       s->stream, (d2*)s->ptr, count, lo, hi, q[6], q[7]);
  else
    hipLaunchKernelGGL((k_phase<float, f2, kBlock>), dim3(grid_for(count, kBlock)), dim3(kBlock), stream_lds(kBlock, 0, 6),
                       s->stream, (f2*)s->ptr, count, lo, hi, (float)q[6], (float)q[7]);
}

Status launch_apply_1q(StateImpl* s, int k, const double* q) {
  const int n = s->n;
  if (is_phase(q)) {  // only the bit-1 half changes
    go_phase(s, k, -1, q);
    return last_launch("apply_1q phase");
  }
  if (s->dtype == QS_C128) {
    units_1q<double, d2>(s, n, k, to_mat<double>(q));
    return last_launch("apply_1q c128");
  }
  const Mat<float> m = to_mat<float>(q);
  if (k == 0) go_inner<kNone>(s, 1ull << (n - 1), 0, m);
  else units_1q<float, f4>(s, n - 1, k - 1, m);
  return last_launch("apply_1q c64");
}

Status launch_apply_cu(StateImpl* s, int c, int t, const double* q) {
  const int n = s->n;
  if (is_phase(q)) {  // only the quarter with control and target bits 1 changes
    go_phase(s, std::min(c, t), std::max(c, t), q);
    return last_launch("apply_cu phase");
  }
  if (s->dtype == QS_C128) {
    units_cu<double, d2>(s, n, c, t, to_mat<double>(q));
    return last_launch("apply_cu c128");
  }
  const Mat<float> m = to_mat<float>(q);
  const int u = n - 1;
  if (t == 0) {  // pair inside each unit; control unit bit c - 1
    const int cv = c - 1;
    if (cu_compact(cv, 0)) go_inner<kCompact>(s, 1ull << (u - 1), cv, m);
    else go_inner<kPred>(s, 1ull << u, cv, m);
  } else if (c == 0) {  // control inside each unit: update odd amplitudes only
    const int tv = t - 1;
    if (tv < kExchangeBits) go_exchange<float, f4, kInnerCtrl>(s, 1ull << u, tv, 0, m);
    else go_pair<float, f4, kInnerCtrl, 0>(s, 1ull << (u - 1), tv, 0, m, kPairWavesCU);
  } else {
    units_cu<float, f4>(s, u, c - 1, t - 1, m);
  }
  return last_launch("apply_cu c64");
}

Status launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t stream) {
  const uint64_t nwords = bytes / 16;
  if (nwords == 0) return Status::ok();
  hipLaunchKernelGGL((k_stream_copy<kPairBlock>), dim3(grid_for(nwords, kPairBlock)),
                     dim3(kPairBlock), 0, stream, (const u64x2*)src, (u64x2*)dst, nwords);
  return last_launch("stream_copy");
}

}  // namespace qs
