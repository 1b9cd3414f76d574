// qs_fused.hip -- one HBM round trip for a whole block of gates.
//
// The GPU form of cache blocking by gate fusion (qHiPSTER Sec. 4.4, Fig. 4):
// a workgroup loads one tile of 2^T amplitudes (the low qubits plus the
// pass's high qubits, see qs_plan.cpp) into registers -- 2^NREG amplitudes
// per thread, 8 for complex128 and 16 for complex64 -- applies every gate of
// the pass there, and writes the tile back.  Register-bit gates are plain
// register arithmetic; a remap moves the tile through LDS so that other tile
// bits become register bits; diagonal gates scale each amplitude by the
// entry its target bit selects, wherever that bit lives (register, thread
// index, or outside the tile).
#include <float.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "qs_device.h"
#include "qs_internal.h"

namespace qs {

constexpr int kFuseBlock = 1 << kFuseThreadBits;  // 256

// Per-pass kernel arguments: the tile's high qubits and, for the load and
// store mappings, the global qubit selected by each thread-index bit and by
// each register-index bit.
struct FusedArgs {
  uint64_t ntiles;
  int32_t L, nh, nops, ngrad;
  int8_t hpos[8];
  int8_t ld_thr[8], st_thr[8];
  int8_t ld_reg[8], st_reg[8];
};

// Device form of an FMap for LDS remaps: tile bit of thread-index bit i in
// nibble i of thr_pack; regoff[r]: byte offset in the remap buffer of the
// register-index part of register r's tile position, already swizzled (the
// swizzle is linear over XOR, and thread and register parts of a position
// have disjoint bits, so a lane's address is swz(thread part) ^ regoff[r]).
struct FMapDev {
  uint32_t thr_pack;
  uint32_t pad[3];
  int32_t regoff[32];
};

// LDS remap buffer swizzle (bank-conflict-free remaps): the element index
// with its higher chunks XOR-folded into the low chunk; shared by the host
// (register offsets) and the device (thread offsets).
__host__ __device__ __forceinline__ int swz_c128(int j) {  // 16-byte elements, 3-bit chunks
  return j ^ (((j >> 3) ^ (j >> 6) ^ (j >> 9)) & 7);
}
__host__ __device__ __forceinline__ int swz_c64(int j) {  // 8-byte elements, 4-bit chunks
  return j ^ (((j >> 4) ^ (j >> 8) ^ (j >> 12)) & 15);
}
template <typename R>
struct LdsAmp;
template <>
struct LdsAmp<double> {
  using T = d2;
  static __device__ __forceinline__ int swz(int j) { return swz_c128(j); }
};
template <>
struct LdsAmp<float> {
  using T = f2;
  static __device__ __forceinline__ int swz(int j) { return swz_c64(j); }
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Tile-local offset of this thread's bits under a packed mapping.
__device__ __forceinline__ int thr_tile_off(uint32_t pack) {
  int o = 0;
#pragma unroll
  for (int i = 0; i < kFuseThreadBits; ++i)
    o |= ((threadIdx.x >> i) & 1) << ((pack >> (4 * i)) & 15);
  return o;
}
// Global offset of this thread's bits (thread bit i selects qubit q[i]).
__device__ __forceinline__ uint64_t thr_global_off(const int8_t* q) {
  uint64_t o = 0;
#pragma unroll
  for (int i = 0; i < kFuseThreadBits; ++i) o |= (uint64_t)((threadIdx.x >> i) & 1) << q[i];
  return o;
}
// Global offset of register index r (compile-time); register bit k selects
// qubit q[k] (uniform): scalar arithmetic.
template <int NREG>
__device__ __forceinline__ uint64_t reg_global_off(const int8_t* q, int r) {
  uint64_t o = 0;
#pragma unroll
  for (int k = 0; k < NREG; ++k)
    if ((r >> k) & 1) o |= 1ull << q[k];
  return o;
}

// Gate on register bit K for every register pair (r, r | 2^K); with a
// control on register bit CR (>= 0) only the pairs whose control bit is 1.
// Both are compile-time constants: a pair that is skipped costs nothing and
// no branch splits the tile's registers (a runtime per-pair branch makes the
// compiler copy the whole tile at every merge).  Amplitudes stay (re, im)
// adjacent in registers, as they are loaded, stored and moved through LDS.
template <int K, int CR, int RA, typename T, typename R>
__device__ __forceinline__ void reg_gate(T* a, const Mat<R>& q) {
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    if (r & (1 << K)) continue;
    if (CR >= 0 && !((r >> CR) & 1)) continue;
    pair_apply(q, a[r], a[r | (1 << K)]);
  }
}

// The same pairs for a real matrix (RY, X, H: half the arithmetic).
template <int K, int CR, int RA, typename T, typename R>
__device__ __forceinline__ void reg_gate_real(T* a, const Mat<R>& q) {
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    if (r & (1 << K)) continue;
    if (CR >= 0 && !((r >> CR) & 1)) continue;
    T& x = a[r];
    T& y = a[r | (1 << K)];
    const R xr = x.x, xi = x.y, yr = y.x, yi = y.y;
    x = T{q.r[0] * xr + q.r[1] * yr, q.r[0] * xi + q.r[1] * yi};
    y = T{q.r[2] * xr + q.r[3] * yr, q.r[2] * xi + q.r[3] * yi};
  }
}

// Im<lambda|P|psi> over the register pairs of bit K (P = X or Y).
template <int K, int RA, typename T>
__device__ __forceinline__ double reg_grad(const T* a, const T* l, int pauli) {
  double g = 0.0;
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    if (r & (1 << K)) continue;
    const int r1 = r | (1 << K);
    g += pair_grad(pauli, a[r].x, a[r].y, a[r1].x, a[r1].y, l[r].x, l[r].y, l[r1].x, l[r1].y);
  }
  return g;
}

// amplitude *= (dr + i di)
template <typename T, typename R>
__device__ __forceinline__ void cscale(T& x, R dr, R di) {
  const R xr = x.x, xi = x.y;
  x = T{dr * xr - di * xi, dr * xi + di * xr};
}

// to, tn: this lane's swizzled byte offsets under the old and new mapping.
template <typename R, int NREG>
__device__ __forceinline__ void remap_tile(typename LdsAmp<R>::T* a, typename LdsAmp<R>::T* lds,
                                           int to, const FMapDev* mo, int tn, const FMapDev* mn) {
  using LT = typename LdsAmp<R>::T;
  constexpr int RA = 1 << NREG;
  char* base = (char*)lds;
#pragma unroll
  for (int r = 0; r < RA; ++r) *(LT*)(base + (to ^ mo->regoff[r])) = a[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < RA; ++r) a[r] = *(const LT*)(base + (tn ^ mn->regoff[r]));
  __syncthreads();
}

// Dispatch on (target register bit k, control register bit cr or -1): one
// specialised, branch-free body per combination.
template <typename R, int NREG, typename T>
__device__ __forceinline__ void reg_gate_any(T* a, const Mat<R>& q, int cr, int k) {
  constexpr int RA = 1 << NREG;
  switch (k * 8 + cr + 1) {
#define QS_REG_GATE(K, CR)                                                  \
  case K * 8 + CR + 1:                                                      \
    if constexpr (K < NREG && CR < NREG) reg_gate<K, CR, RA>(a, q);        \
    break;
    QS_REG_GATE(0, -1) QS_REG_GATE(0, 1) QS_REG_GATE(0, 2) QS_REG_GATE(0, 3)
    QS_REG_GATE(1, -1) QS_REG_GATE(1, 0) QS_REG_GATE(1, 2) QS_REG_GATE(1, 3)
    QS_REG_GATE(2, -1) QS_REG_GATE(2, 0) QS_REG_GATE(2, 1) QS_REG_GATE(2, 3)
    QS_REG_GATE(3, -1) QS_REG_GATE(3, 0) QS_REG_GATE(3, 1) QS_REG_GATE(3, 2)
#undef QS_REG_GATE
    default: break;
  }
}

template <typename R, int NREG, typename T>
__device__ __forceinline__ void reg_real_any(T* a, const Mat<R>& q, int cr, int k) {
  constexpr int RA = 1 << NREG;
  switch (k * 8 + cr + 1) {
#define QS_REG_REAL(K, CR)                                                  \
  case K * 8 + CR + 1:                                                      \
    if constexpr (K < NREG && CR < NREG) reg_gate_real<K, CR, RA>(a, q);   \
    break;
    QS_REG_REAL(0, -1) QS_REG_REAL(0, 1) QS_REG_REAL(0, 2) QS_REG_REAL(0, 3)
    QS_REG_REAL(1, -1) QS_REG_REAL(1, 0) QS_REG_REAL(1, 2) QS_REG_REAL(1, 3)
    QS_REG_REAL(2, -1) QS_REG_REAL(2, 0) QS_REG_REAL(2, 1) QS_REG_REAL(2, 3)
    QS_REG_REAL(3, -1) QS_REG_REAL(3, 0) QS_REG_REAL(3, 1) QS_REG_REAL(3, 2)
#undef QS_REG_REAL
    default: break;
  }
}
// A U op by the form of its matrix (each branch ends in its own empty asm
// statement so that the optimiser keeps the bodies apart).  An exchange body
// for X measured worse: its register renaming across the branches sent the
// tiles to scratch memory.
template <typename R, int NREG, typename T>
__device__ __forceinline__ void reg_form_any(T* a, const Mat<R>& q, int cr, int k, int kw) {
  if (kw & kUReal) {
    reg_real_any<R, NREG>(a, q, cr, k);
    asm volatile("; uform real");
  } else {
    reg_gate_any<R, NREG>(a, q, cr, k);
    asm volatile("; uform general");
  }
}

template <int NREG, typename T>
__device__ __forceinline__ double reg_grad_any(const T* a, const T* l, int pauli, int k) {
  constexpr int RA = 1 << NREG;
  switch (k) {
    case 0: return reg_grad<0, RA>(a, l, pauli);
    case 1: return reg_grad<1, RA>(a, l, pauli);
    case 2: return reg_grad<2, RA>(a, l, pauli);
    default:
      if constexpr (NREG > 3) return reg_grad<(NREG > 3 ? 3 : 0), RA>(a, l, pauli);
      return 0.0;
  }
}

// Diagonal op with its target on register bit K: amplitude *= e0 or e1 by
// its target bit, where its control bit (register creg, uniform) is 1.  PH:
// the op is a phase (e0 = 1), so the registers whose target bit is 0 are
// left alone.
template <int K, bool PH, typename R, int NREG, typename T>
__device__ __forceinline__ void diag_reg(T* a, R e0r, R e0i, R e1r, R e1i, int creg) {
  constexpr int RA = 1 << NREG;
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    const bool bit = (r >> K) & 1;
    if (PH && !bit) continue;
    const bool c_r = creg < 0 || ((r >> creg) & 1);  // uniform
    const R er = bit ? e1r : e0r, ei = bit ? e1i : e0i;
    cscale(a[r], c_r ? er : (R)1, c_r ? ei : (R)0);
  }
}

// Diagonal op on one register tile: amplitude *= d0 or d1 by its target bit
// wherever that bit lives; `on` is false on the lanes whose thread-bit
// control is 0 (identity there); `phase`: d0 = 1.  Register-bit targets go
// to bodies specialised for the bit, each ending in a distinct empty asm
// statement so that the optimiser keeps them apart (merged, they index the
// tile at run time and spill it).
template <typename R, int NREG, typename T>
__device__ __forceinline__ void diag_tile(T* a, R d0r, R d0i, R d1r, R d1i, int tw, int tix,
                                          int creg, bool on, bool phase, uint64_t base) {
  constexpr int RA = 1 << NREG;
  const R e0r = on ? d0r : (R)1, e0i = on ? d0i : (R)0;
  const R e1r = on ? d1r : (R)1, e1i = on ? d1i : (R)0;
  if (tw == kInReg) {
#define QS_DIAG(KK, PP, tag)                                             \
  {                                                                      \
    diag_reg<(KK < NREG ? KK : 0), PP, R, NREG>(a, e0r, e0i, e1r, e1i, creg); \
    asm volatile("; diag " tag);                                         \
  }
    if (phase) {
      if (tix == 0) QS_DIAG(0, true, "p0")
      else if (tix == 1) QS_DIAG(1, true, "p1")
      else if (tix == 2 || NREG == 3) QS_DIAG(2, true, "p2")
      else QS_DIAG(3, true, "p3")
    } else {
      if (tix == 0) QS_DIAG(0, false, "g0")
      else if (tix == 1) QS_DIAG(1, false, "g1")
      else if (tix == 2 || NREG == 3) QS_DIAG(2, false, "g2")
      else QS_DIAG(3, false, "g3")
    }
#undef QS_DIAG
  } else {
    // target bit fixed for the whole thread (thread bit) or tile (outside)
    const bool bit = (tw == kInThread) ? (bool)((threadIdx.x >> tix) & 1)
                                       : (bool)((base >> tix) & 1);
    if (tw == kOutside && phase && !bit) return;  // uniform: a factor of 1
    const R tr = bit ? e1r : e0r, ti = bit ? e1i : e0i;
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const bool c_r = creg < 0 || ((r >> creg) & 1);  // uniform
      cscale(a[r], c_r ? tr : (R)1, c_r ? ti : (R)0);
    }
  }
}

// Gradient partials are summed over each 16-lane row of a wave with four
// DPP steps (row mirror, half-row mirror, two quad permutations: plain
// VALU moves, no LDS crossbar traffic); every lane ends with its row's sum,
// added in a fixed order.  The first lane of each row adds it to its own
// accumulator entry, kAdjRows per gradient slot and workgroup.
constexpr int kAdjRows = kFuseBlock / 16;

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_f64<0x140>(v);  // row_mirror: lane i + lane 15 - i
  v += dpp_f64<0x141>(v);  // row_half_mirror: within each half-row
  v += dpp_f64<0x1B>(v);   // quad_perm [3, 2, 1, 0]
  v += dpp_f64<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  return v;
}

// A slot's kAdjRows row sums, added in row order.
__device__ __forceinline__ double adj_slot_sum(const double* rows) {
  double t = 0.0;
#pragma unroll
  for (int r = 0; r < kAdjRows; ++r) t += rows[r];
  return t;
}

// Apply ops[0 .. nops) to the register tile(s).  `base` is the tile's
// global index base (bits outside the tile).  The op index goes through
// readfirstlane, so op records and mappings are fetched with scalar loads
// and gate coefficients live in scalar registers.  Diagonal entries and
// their controls are resolved into the coefficients (per register index when
// uniform, once per thread for thread-index bits).
//
// ADJ: a second tile (lambda) receives every gate too, and ops with a
// gradient slot first add Im<lambda|P|psi> (P = the rotation's generator,
// X/Y on register pairs, Z by the sign of the target bit) to its row's LDS
// accumulator of that slot.
template <typename R, int NREG, bool ADJ, bool RUNS = false>
__device__ __forceinline__ void run_ops(typename LdsAmp<R>::T* a, typename LdsAmp<R>::T* l,
                                        typename LdsAmp<R>::T* lds, const FOp* __restrict__ ops,
                                        int nops, const FMapDev* __restrict__ maps,
                                        uint64_t base, double* acc, uint64_t tile) {
  constexpr int RA = 1 << NREG;
  // The next op's record is fetched (scalar loads) while this op computes;
  // the table holds one spare record past every pass's last op.
  FOp nxt = ops[0];
  for (int oi = 0; oi < nops; ++oi) {
    const FOp cur = nxt;
    nxt = ops[uniform(oi + 1)];
    const FOp* op = &cur;
    const int kw = op->kind, tgt = op->tgt, ctl = op->ctl, aux = op->aux;
    const int kind = kw & 255, pauli = (kw >> 8) & 255;
    if (kind == kOpRemap) {
      const FMapDev* mo = maps + uniform(aux);
      const FMapDev* mn = maps + uniform(tgt);
      constexpr int ES = (int)sizeof(typename LdsAmp<R>::T);
      const int to = LdsAmp<R>::swz(thr_tile_off(mo->thr_pack)) * ES;
      const int tn = LdsAmp<R>::swz(thr_tile_off(mn->thr_pack)) * ES;
      remap_tile<R, NREG>(a, lds, to, mo, tn, mn);
      if constexpr (ADJ) remap_tile<R, NREG>(l, lds, to, mo, tn, mn);
      continue;
    }
    if (RUNS && kind == kOpPhaseRun) {  // forward passes that hold runs only
      // the product of the run's phases, per lane: entry e contributes its
      // d1 where its control (none or a thread bit) is 1, and the entries
      // controlled outside the tile come as one product from the run's
      // tables; then the target-bit-1 amplitudes (target on a register bit,
      // a thread bit or outside the tile) are scaled once
      // Two or more entries with no control or a thread-bit control come as
      // one value per thread from a third table; a single such entry is read
      // explicitly.  Explicit entries are read four at a time (their scalar
      // loads in flight together) into two product chains, even and odd
      // entries, which are joined at the end.
      auto factor = [&](int ec, double m6, double m7, R& fr, R& fi) {
        const int ew = ec >> 8, eb = ec & 255;
        const bool eon = ew == kNoBit || (ew == kInThread ? (bool)((threadIdx.x >> eb) & 1)
                                                          : (bool)((base >> eb) & 1));
        fr = eon ? (R)m6 : (R)1;
        fi = eon ? (R)m7 : (R)0;
      };
      auto mul_into = [](R& pr_, R& pi_, R dr, R di) {
        const R t = pr_ * dr - pi_ * di;
        pi_ = pr_ * di + pi_ * dr;
        pr_ = t;
      };
      R pr = (R)1, pi = (R)0, qr = (R)1, qi = (R)0;
      if (op->m[4] != 0.0) {
        // entries with no control or a thread-bit control, folded into one
        // product per thread
        const double* tl = (const double*)((const char*)maps + (size_t)op->m[3]);
        pr = (R)tl[2 * threadIdx.x];
        pi = (R)tl[2 * threadIdx.x + 1];
      }
      int e = 1;
      for (; e + 3 <= aux; e += 4) {
        int ec[4];
        double m6[4], m7[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const FOp* en = ops + uniform(oi + e + j);
          ec[j] = en->ctl;
          m6[j] = en->m[6];
          m7[j] = en->m[7];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          R dr, di;
          factor(ec[j], m6[j], m7[j], dr, di);
          if (j & 1) mul_into(qr, qi, dr, di);
          else mul_into(pr, pi, dr, di);
        }
      }
      for (; e <= aux; ++e) {
        const FOp* en = ops + uniform(oi + e);
        R dr, di;
        factor(en->ctl, en->m[6], en->m[7], dr, di);
        mul_into(pr, pi, dr, di);
      }
      mul_into(pr, pi, qr, qi);
      if (op->m[2] != 0.0) {
        // entries controlled outside the tile: their product by the tile
        // index, from the run's two tables (low and high index bits)
        const int lb = (int)op->m[1];
        const double* tlo = (const double*)((const char*)maps + (size_t)op->m[0]);
        const double* thi = tlo + 2 * ((size_t)1 << lb);
        const uint64_t lo = tile & ((1ull << lb) - 1ull), hi = tile >> lb;
        mul_into(pr, pi, (R)tlo[2 * lo], (R)tlo[2 * lo + 1]);
        mul_into(pr, pi, (R)thi[2 * hi], (R)thi[2 * hi + 1]);
      }
      diag_tile<R, NREG>(a, (R)1, (R)0, pr, pi, tgt >> 8, tgt & 255, -1, true, true, base);
      oi += aux;
      nxt = ops[uniform(oi + 1)];
      continue;
    }
    const int cw = ctl >> 8, ci = ctl & 255;
    const int creg = (cw == kInReg) ? ci : -1;
    const bool on = (cw == kInThread) ? (bool)((threadIdx.x >> ci) & 1) : true;
    if (kind == kOpU) {
      // a control outside the tile skips the gate for the whole tile (a
      // uniform branch; the specialised bodies update the tile in place, so
      // the skip costs no register copies); a thread-index control selects
      // identity coefficients per lane
      if (cw == kOutside && !((base >> ci) & 1)) continue;  // per-tile predicate (uniform)
      Mat<R> q;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        q.r[e] = (R)op->m[2 * e];
        q.i[e] = (R)op->m[2 * e + 1];
      }
      if constexpr (ADJ) {
        if (aux >= 0) {  // rotation (never controlled): gradient before the inverse
          const double g = row_sum16(reg_grad_any<NREG>(a, l, pauli, tgt));
          if ((threadIdx.x & 15) == 0) acc[aux * kAdjRows + (threadIdx.x >> 4)] += g;
        }
      }
      if (cw == kInThread) {
        if constexpr (ADJ) {
          // two tiles: masking the lanes off costs less than per-lane
          // coefficients for both (measured)
          if (on) {
            reg_form_any<R, NREG>(a, q, -1, tgt, kw);
            reg_form_any<R, NREG>(l, q, -1, tgt, kw);
          }
        } else {
          Mat<R> ql;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const R one = (e == 0 || e == 3) ? (R)1 : (R)0;
            ql.r[e] = on ? q.r[e] : one;
            ql.i[e] = on ? q.i[e] : (R)0;
          }
          reg_gate_any<R, NREG>(a, ql, -1, tgt);
        }
      } else {
        if constexpr (ADJ) {
          reg_form_any<R, NREG>(a, q, creg, tgt, kw);
          reg_form_any<R, NREG>(l, q, creg, tgt, kw);
        } else {
          reg_gate_any<R, NREG>(a, q, creg, tgt);
        }
      }
    } else {  // diagonal
      if (cw == kOutside && !((base >> ci) & 1)) continue;  // per-tile predicate (uniform)
      const R d0r = (R)op->m[0], d0i = (R)op->m[1], d1r = (R)op->m[6], d1i = (R)op->m[7];
      const int tw = tgt >> 8, tix = tgt & 255;
      if constexpr (ADJ) {
        if (aux >= 0) {  // RZ: Im<lambda|Z|psi> = sum of +-Im(conj(l) a) by the target bit
          double g = 0.0;
          const bool fixed_bit = (tw == kInThread) ? (bool)((threadIdx.x >> tix) & 1)
                                                   : (bool)((base >> tix) & 1);
#pragma unroll
          for (int r = 0; r < RA; ++r) {
            const bool bit = (tw == kInReg) ? (bool)((r >> tix) & 1) : fixed_bit;
            const double t = im_conj_mul(l[r].x, l[r].y, a[r].x, a[r].y);
            g += bit ? -t : t;
          }
          g = row_sum16(g);
          if ((threadIdx.x & 15) == 0) acc[aux * kAdjRows + (threadIdx.x >> 4)] += g;
        }
      }
      const bool phase = (kw >> 16) & 1;
      diag_tile<R, NREG>(a, d0r, d0i, d1r, d1i, tw, tix, creg, on, phase, base);
      if constexpr (ADJ) diag_tile<R, NREG>(l, d0r, d0i, d1r, d1i, tw, tix, creg, on, phase, base);
    }
  }
}

__device__ __forceinline__ uint64_t tile_base(uint64_t tile, const FusedArgs& A) {
  uint64_t x = tile << A.L;
#pragma unroll
  for (int h = 0; h < 8; ++h)
    if (h < A.nh) x = insert0(x, A.hpos[h]);
  return x;
}

// One tile per workgroup (a one-shot grid overlaps the loads, arithmetic and
// stores of different workgroups better than a persistent loop here).

// complex128: one d2 per amplitude.
// RUNS: the pass holds phase runs (a separate instance, so that passes
// without them keep the smaller register budget and schedule).
template <int NREG, bool RUNS>
__global__ void __launch_bounds__(kFuseBlock)
k_fused_c128(d2* __restrict__ a, FusedArgs A, const FOp* __restrict__ ops,
             const FMapDev* __restrict__ maps) {
  constexpr int RA = 1 << NREG;
  __shared__ d2 lds[RA * kFuseBlock];
  d2 t[RA];
  const uint64_t tl = thr_global_off(A.ld_thr), ts = thr_global_off(A.st_thr);
  for (uint64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const uint64_t base = tile_base(tile, A);
#pragma unroll
    for (int r = 0; r < RA; ++r) t[r] = gload<true>(a + (base | tl | reg_global_off<NREG>(A.ld_reg, r)));
    run_ops<double, NREG, false, RUNS>(t, nullptr, lds, ops, A.nops, maps, base, nullptr, tile);
#pragma unroll
    for (int r = 0; r < RA; ++r) gstore<true>(a + (base | ts | reg_global_off<NREG>(A.st_reg, r)), t[r]);
  }
}

// complex64: 16-byte units of two amplitudes; register bit 0 is qubit 0 at
// load and store, so registers (2u, 2u + 1) form one unit.
template <int NREG, bool RUNS>
__global__ void __launch_bounds__(kFuseBlock)
k_fused_c64(f4* __restrict__ a, FusedArgs A, const FOp* __restrict__ ops,
            const FMapDev* __restrict__ maps) {
  constexpr int RA = 1 << NREG;
  __shared__ f2 lds[RA * kFuseBlock];
  f2 t[RA];
  const uint64_t tl = thr_global_off(A.ld_thr), ts = thr_global_off(A.st_thr);
  for (uint64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const uint64_t base = tile_base(tile, A);
#pragma unroll
    for (int r = 0; r < RA; r += 2) {
      const f4 v = gload<true>(a + ((base | tl | reg_global_off<NREG>(A.ld_reg, r)) >> 1));
      t[r] = f2{v.x, v.y};
      t[r + 1] = f2{v.z, v.w};
    }
    run_ops<float, NREG, false, RUNS>(t, nullptr, lds, ops, A.nops, maps, base, nullptr, tile);
#pragma unroll
    for (int r = 0; r < RA; r += 2)
      gstore<true>(a + ((base | ts | reg_global_off<NREG>(A.st_reg, r)) >> 1),
                   f4{t[r].x, t[r].y, t[r + 1].x, t[r + 1].y});
  }
}

// ------------------------------------------------------------- adjoint
// psi and lambda tiles side by side; a persistent grid so that every
// workgroup folds its gradient contributions over many tiles into its LDS
// slots and leaves one partial per slot: part[slot * gridDim.x + block].
template <int NREG>
__global__ void __launch_bounds__(kFuseBlock, 3)  // three waves per SIMD: a few spilled registers cost less than a third fewer waves (measured)
k_fused_adj_c128(d2* __restrict__ psi, d2* __restrict__ lam, FusedArgs A,
                 const FOp* __restrict__ ops, const FMapDev* __restrict__ maps,
                 double* __restrict__ part) {
  constexpr int RA = 1 << NREG;
  __shared__ d2 lds[RA * kFuseBlock];
  __shared__ double acc[kAdjMaxSlots * kAdjRows];
  for (int i = threadIdx.x; i < kAdjMaxSlots * kAdjRows; i += kFuseBlock) acc[i] = 0.0;
  __syncthreads();
  d2 t[RA], l[RA];
  const uint64_t tl = thr_global_off(A.ld_thr), ts = thr_global_off(A.st_thr);
  for (uint64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const uint64_t base = tile_base(tile, A);
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const uint64_t i = base | tl | reg_global_off<NREG>(A.ld_reg, r);
      t[r] = gload<true>(psi + i);
      l[r] = gload<true>(lam + i);
    }
    run_ops<double, NREG, true>(t, l, lds, ops, A.nops, maps, base, acc, tile);
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const uint64_t i = base | ts | reg_global_off<NREG>(A.st_reg, r);
      gstore<true>(psi + i, t[r]);
      gstore<true>(lam + i, l[r]);
    }
  }
  __syncthreads();
  for (int sl = threadIdx.x; sl < A.ngrad; sl += kFuseBlock)
    part[(size_t)sl * gridDim.x + blockIdx.x] = adj_slot_sum(acc + sl * kAdjRows);
}

template <int NREG>
__global__ void __launch_bounds__(kFuseBlock, 3)  // three waves per SIMD, as for complex128
k_fused_adj_c64(f4* __restrict__ psi, f4* __restrict__ lam, FusedArgs A,
                const FOp* __restrict__ ops, const FMapDev* __restrict__ maps,
                double* __restrict__ part) {
  constexpr int RA = 1 << NREG;
  __shared__ f2 lds[RA * kFuseBlock];
  __shared__ double acc[kAdjMaxSlots * kAdjRows];
  for (int i = threadIdx.x; i < kAdjMaxSlots * kAdjRows; i += kFuseBlock) acc[i] = 0.0;
  __syncthreads();
  f2 t[RA], l[RA];
  const uint64_t tl = thr_global_off(A.ld_thr), ts = thr_global_off(A.st_thr);
  for (uint64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const uint64_t base = tile_base(tile, A);
#pragma unroll
    for (int r = 0; r < RA; r += 2) {
      const uint64_t u = (base | tl | reg_global_off<NREG>(A.ld_reg, r)) >> 1;
      const f4 v = gload<true>(psi + u), w = gload<true>(lam + u);
      t[r] = f2{v.x, v.y};
      t[r + 1] = f2{v.z, v.w};
      l[r] = f2{w.x, w.y};
      l[r + 1] = f2{w.z, w.w};
    }
    run_ops<float, NREG, true>(t, l, lds, ops, A.nops, maps, base, acc, tile);
#pragma unroll
    for (int r = 0; r < RA; r += 2) {
      const uint64_t u = (base | ts | reg_global_off<NREG>(A.st_reg, r)) >> 1;
      gstore<true>(psi + u, f4{t[r].x, t[r].y, t[r + 1].x, t[r + 1].y});
      gstore<true>(lam + u, f4{l[r].x, l[r].y, l[r + 1].x, l[r + 1].y});
    }
  }
  __syncthreads();
  for (int sl = threadIdx.x; sl < A.ngrad; sl += kFuseBlock)
    part[(size_t)sl * gridDim.x + blockIdx.x] = adj_slot_sum(acc + sl * kAdjRows);
}

// Host: device tables of a plan's mappings.
static FMapDev fmap_dev(const FMap& m, int nreg, int dtype) {
  FMapDev d;
  memset(&d, 0, sizeof(d));
  for (int i = 0; i < kFuseThreadBits; ++i) d.thr_pack |= (uint32_t)(m.thr[i] & 15) << (4 * i);
  const int es = dtype == QS_C128 ? 16 : 8;
  for (int r = 0; r < (1 << nreg); ++r) {
    int o = 0;
    for (int k = 0; k < nreg; ++k)
      if ((r >> k) & 1) o |= 1 << m.reg[k];
    d.regoff[r] = (dtype == QS_C128 ? swz_c128(o) : swz_c64(o)) * es;
  }
  return d;
}

// Host: global qubits of a mapping's thread and register bits for a pass
// with low qubits L and high qubits hpos.
static void fmap_global(const FMap& m, int nreg, int L, const int8_t* hpos, int8_t* thr,
                        int8_t* reg) {
  auto gq = [&](int tb) { return tb < L ? tb : (int)hpos[tb - L]; };
  for (int i = 0; i < kFuseThreadBits; ++i) thr[i] = (int8_t)gq(m.thr[i]);
  for (int k = 0; k < 8; ++k) reg[k] = (int8_t)(k < nreg ? gq(m.reg[k]) : 0);
}

static Status last_launch(const char* what) { return hip_status(hipGetLastError(), what); }

// Upload a plan's ops and mapping tables into the state's table buffer.
static Status upload_plan(StateImpl* s, const Plan& plan, const FuseGeom& G, const FOp** dops,
                          const FMapDev** dmaps) {
  *dops = nullptr;
  *dmaps = nullptr;
  if (plan.ops.empty()) return Status::ok();
  std::vector<FMapDev> md;
  for (const FMap& m : plan.maps) md.push_back(fmap_dev(m, G.nreg, s->dtype));
  // one zeroed record past the last op: the kernels prefetch op i + 1
  const size_t ob = (plan.ops.size() + 1) * sizeof(FOp), mb = md.size() * sizeof(FMapDev);
  const size_t tb = plan.run_tab.size() * sizeof(double);  // phase-run tables, after the maps
  std::vector<char> blob(ob + mb + tb, 0);
  memcpy(blob.data(), plan.ops.data(), plan.ops.size() * sizeof(FOp));
  if (tb) memcpy(blob.data() + ob + mb, plan.run_tab.data(), tb);
  // diagonal ops with d0 = 1 (phases) leave target-bit-0 amplitudes alone
  FOp* fo = (FOp*)blob.data();
  for (size_t i = 0; i < plan.ops.size(); ++i)
    if ((fo[i].kind & 255) == kOpDiag && fo[i].m[0] == 1.0 && fo[i].m[1] == 0.0)
      fo[i].kind |= kDiagPhase;
  // run tables: offset in run_tab -> byte offset from the maps
  for (size_t i = 0; i < plan.ops.size(); ++i) {
    if ((fo[i].kind & 255) != kOpPhaseRun) continue;
    if (fo[i].m[2] != 0.0) fo[i].m[0] = (double)(mb + (size_t)fo[i].m[0] * sizeof(double));
    if (fo[i].m[4] != 0.0) fo[i].m[3] = (double)(mb + (size_t)fo[i].m[3] * sizeof(double));
  }
  // U ops whose matrix is real (the adjoint kernels use the cheaper body;
  // the forward kernels ignore the flag)
  for (size_t i = 0; i < plan.ops.size(); ++i) {
    const double* m = fo[i].m;
    if ((fo[i].kind & 255) == kOpU && m[1] == 0.0 && m[3] == 0.0 && m[5] == 0.0 && m[7] == 0.0)
      fo[i].kind |= kUReal;
  }
  memcpy(blob.data() + ob, md.data(), mb);
  Status st = upload_table(s, blob.data(), blob.size());
  if (!st.good()) return st;
  *dops = (const FOp*)s->table.ptr;
  *dmaps = (const FMapDev*)((const char*)s->table.ptr + ob);
  return Status::ok();
}

static FusedArgs pass_args(const StateImpl* s, const Plan& plan, const Pass& p, const FuseGeom& G) {
  FusedArgs A;
  memset(&A, 0, sizeof(A));
  A.ntiles = 1ull << (s->n - G.T);
  A.L = G.L;
  A.nh = p.nh;
  A.nops = p.nops;
  A.ngrad = p.ngrad;
  for (int h = 0; h < p.nh; ++h) A.hpos[h] = p.hpos[h];
  fmap_global(plan.maps[p.map_load], G.nreg, G.L, p.hpos, A.ld_thr, A.ld_reg);
  fmap_global(plan.maps[p.map_store], G.nreg, G.L, p.hpos, A.st_thr, A.st_reg);
  return A;
}

bool use_compiled_passes(const StateImpl* s) {
  if (s->exec == QS_EXEC_COMPILED) return true;
  if (s->exec == QS_EXEC_INTERPRETED) return false;
  const char* e = getenv("QS_FUSED_EXEC");
  if (e && !strcmp(e, "compiled")) return true;
  if (e && !strcmp(e, "interpreted")) return false;
  return s->n >= kJitAutoMinQubits;
}

// Tile order of compiled passes.  Which tiles a pass's workgroups hold at
// once decides which addresses are in flight together, and so how its
// accesses spread over HBM channels and banks; it changes no result (each
// tile is computed the same way, and gradient partials are kept per tile).
// Order k splits the tiles into 2^k regions that consecutive workgroups
// walk side by side (k = 0: plain; k = 3: one eighth per XCD).  Traced pass
// by pass over random circuits and the QFT at n = 30 (complex128) and 31
// (complex64), the fastest k differed from pass to pass, by up to 1.5 ms of
// 6-8 ms, the same way in repeated runs, and no rule on the tile's qubits
// predicted it well.  So a compiled kernel times each order once, one per
// launch at a tile count, with events around the launch that are read at a
// later launch once they have completed, and then keeps the fastest.
// Picking from one timed sample per order of k = 0..7 and scoring on
// another run took 5.9 % (complex128) and 3.7 % (complex64) off the random
// circuit against the plain order alone.  QS_TILE_ORDER = k (0..7), when
// set, fixes the order instead.
constexpr int kTileOrders = 8;
struct TileOrderStats {
  hipEvent_t start = nullptr, stop = nullptr;
  int pending = -1;  // order of the timed launch not yet read
  float ms[kTileOrders] = {-1.f, -1.f, -1.f, -1.f, -1.f, -1.f, -1.f, -1.f};
};
static std::mutex g_order_mu;
static std::map<std::tuple<int, hipFunction_t, uint64_t>, TileOrderStats> g_orders;

static int forced_tile_order() {
  const char* e = getenv("QS_TILE_ORDER");
  if (!e || !*e) return -1;
  const int k = atoi(e);
  return k >= 0 && k < kTileOrders ? k : -1;
}

// Orders that differ from one another at ntiles (a power of two): 2^k
// regions of at least two tiles each.
static int tile_orders_at(uint64_t ntiles) {
  int k = 0;
  while (k < kTileOrders && (ntiles >> k) >= 2) ++k;
  return k;
}

// Launch a compiled pass kernel; args: the kernel's arguments in order, the
// last of them *order, which is set here.
static Status launch_compiled(StateImpl* s, const JitPass& jp, unsigned grid, uint64_t ntiles, unsigned* order,
                              void** args) {
  hipFunction_t f = nullptr;
  Status st = jit_function(jp, s->device, &f);
  if (!st.good()) return st;
  auto launch = [&]() {
    return hip_status(hipModuleLaunchKernel(f, grid, 1, 1, kFuseBlock, 1, 1, 0, s->stream, args, nullptr),
                      "compiled fused pass");
  };
  *order = 0;
  const int forced = forced_tile_order();
  // the orders differ only on a one-shot grid of several tiles
  const int norders = tile_orders_at(ntiles);
  if (forced >= 0 || grid != ntiles || norders < 2) {
    if (forced >= 0) *order = (unsigned)forced;
    return launch();
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s->stream, &cap) != hipSuccess) {
    (void)hipGetLastError();
    cap = hipStreamCaptureStatusActive;  // unknown: take no timing
  }
  std::lock_guard<std::mutex> lock(g_order_mu);
  TileOrderStats& o = g_orders[std::make_tuple(s->device, f, ntiles)];
  // Timing never fails a run: if the events cannot be made, recorded or
  // read, the orders not yet timed are dropped and the kernel keeps the
  // fastest timed order (plain if none).
  auto stop_timing = [&]() {
    (void)hipGetLastError();
    for (int k = 0; k < kTileOrders; ++k)
      if (o.ms[k] < 0.f) o.ms[k] = FLT_MAX;
  };
  if (o.pending >= 0) {
    const hipError_t q = hipEventQuery(o.stop);
    if (q == hipSuccess) {
      float ms = 0.f;
      const int k = o.pending;
      o.pending = -1;
      if (hipEventElapsedTime(&ms, o.start, o.stop) == hipSuccess) o.ms[k] = ms;
      else stop_timing();
    } else if (q == hipErrorNotReady) {
      // not an error: keep the runtime's last-error state clean of it
      if (hipPeekAtLastError() == hipErrorNotReady) (void)hipGetLastError();
    } else {
      o.pending = -1;
      stop_timing();
    }
  }
  // next: the lowest order not yet timed; best: the fastest timed (0 if none)
  int next = -1, best = 0;
  for (int k = norders - 1; k >= 0; --k) {
    if (o.ms[k] < 0.f) next = k;
    else if (o.ms[best] < 0.f || o.ms[k] <= o.ms[best]) best = k;
  }
  if (next < 0 || o.pending >= 0 || cap != hipStreamCaptureStatusNone) {
    *order = (unsigned)best;
    return launch();
  }
  if (!o.start) {
    // the events belong to the state's device
    int cur = -1;
    bool ok = hipGetDevice(&cur) == hipSuccess && (cur == s->device || hipSetDevice(s->device) == hipSuccess);
    ok = ok && hipEventCreate(&o.start) == hipSuccess;
    ok = ok && hipEventCreate(&o.stop) == hipSuccess;
    if (cur >= 0 && cur != s->device) (void)hipSetDevice(cur);
    if (!ok) {
      stop_timing();
      *order = (unsigned)best;
      return launch();
    }
  }
  *order = (unsigned)next;
  if (hipEventRecord(o.start, s->stream) != hipSuccess) {
    stop_timing();
    *order = (unsigned)best;
    return launch();
  }
  st = launch();
  if (!st.good()) return st;
  if (hipEventRecord(o.stop, s->stream) != hipSuccess) stop_timing();
  else o.pending = (int)*order;
  return st;
}

Status precompile_passes(int n, int dtype, const std::vector<XGate>& gates, bool adjoint,
                         bool wide, int* nkernels) {
  std::vector<JitPass> jp;
  Plan plan;
  plan_gates(n, dtype, gates, true, &plan, true, 1 << 30, false, wide);
  Status st = jit_prepare(plan, n, dtype, false, &jp);
  if (!st.good()) return st;
  std::vector<int> used;
  auto count = [&](const std::vector<JitPass>& v) {
    for (const JitPass& j : v)
      if (j.entry >= 0 && std::find(used.begin(), used.end(), j.entry) == used.end())
        used.push_back(j.entry);
  };
  count(jp);
  if (adjoint && n >= fuse_geom(dtype).T) {
    std::vector<XGate> rev;
    reverse_daggered(gates, &rev);
    Plan ap;
    plan_gates(n, dtype, rev, true, &ap, /*allow_single=*/false, kAdjMaxSlots, /*grad=*/true, wide);
    st = jit_prepare(ap, n, dtype, true, &jp);
    if (!st.good()) return st;
    count(jp);
  }
  *nkernels = (int)used.size();
  return Status::ok();
}

Status run_gates(StateImpl* s, const std::vector<XGate>& gates, int flags) {
  Plan plan;
  plan_gates(s->n, s->dtype, gates, !(flags & QS_RUN_NO_FUSION), &plan, true, 1 << 30, false,
             (flags & QS_RUN_WIDE_TILES) != 0);
  const FuseGeom G = plan.geom;
  std::vector<JitPass> jp;
  if (use_compiled_passes(s)) {
    Status st = jit_prepare(plan, s->n, s->dtype, false, &jp);
    if (!st.good()) return st;
  }
  const FOp* dops;
  const FMapDev* dmaps;
  Status up = upload_plan(s, plan, G, &dops, &dmaps);
  if (!up.good()) return up;
  for (size_t pi = 0; pi < plan.passes.size(); ++pi) {
    const Pass& p = plan.passes[pi];
    Status st;
    if (p.kind == kPass1q) {
      st = launch_apply_1q(s, gates[p.gate].target, gates[p.gate].m);
    } else if (p.kind == kPassCU) {
      st = launch_apply_cu(s, gates[p.gate].control, gates[p.gate].target, gates[p.gate].m);
    } else {
      const FusedArgs A = pass_args(s, plan, p, G);
      uint64_t cap = (1ull << 31) / kFuseBlock;
      if (s->grid_limit > 0) cap = std::min<uint64_t>(cap, (uint64_t)s->grid_limit);
      const unsigned grid = (unsigned)std::min<uint64_t>(A.ntiles, cap);
      bool runs = false;
      for (int i = p.op_first; i < p.op_first + p.nops; ++i) runs |= plan.ops[i].kind == kOpPhaseRun;
      if (!jp.empty() && jp[pi].entry >= 0) {
        void* a = s->ptr;
        const FOp* o = dops + p.op_first;
        const void* mp = dmaps;
        unsigned long long nt = A.ntiles;
        unsigned order = 0;
        void* args[] = {&a, &o, &mp, &nt, &order};
        st = launch_compiled(s, jp[pi], grid, A.ntiles, &order, args);
        if (!st.good()) return st;
        continue;
      }
      if (s->dtype == QS_C128) {
        if (runs)
          hipLaunchKernelGGL((k_fused_c128<3, true>), dim3(grid), dim3(kFuseBlock), 0, s->stream,
                             (d2*)s->ptr, A, dops + p.op_first, dmaps);
        else
          hipLaunchKernelGGL((k_fused_c128<3, false>), dim3(grid), dim3(kFuseBlock), 0, s->stream,
                             (d2*)s->ptr, A, dops + p.op_first, dmaps);
      } else {
        if (runs)
          hipLaunchKernelGGL((k_fused_c64<4, true>), dim3(grid), dim3(kFuseBlock), 0, s->stream,
                             (f4*)s->ptr, A, dops + p.op_first, dmaps);
        else
          hipLaunchKernelGGL((k_fused_c64<4, false>), dim3(grid), dim3(kFuseBlock), 0, s->stream,
                             (f4*)s->ptr, A, dops + p.op_first, dmaps);
      }
      st = last_launch("fused pass");
    }
    if (!st.good()) return st;
  }
  return Status::ok();
}

// Compute units of the state's device (queried once per handle).
static int device_cus(StateImpl* s) {
  if (s->cus <= 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess ||
        v <= 0) {
      (void)hipGetLastError();
      v = 256;
    }
    s->cus = v;
  }
  return s->cus;
}

constexpr int kAdjWgPerCu = 3;  // resident adjoint workgroups per CU (three waves per SIMD)

Status run_adjoint_fused(StateImpl* s, StateImpl* lam, const std::vector<XGate>& rev,
                         std::vector<int>* rows, double** slot_sums_dev, bool wide) {
  Plan plan;
  plan_gates(s->n, s->dtype, rev, true, &plan, /*allow_single=*/false, kAdjMaxSlots, /*grad=*/true, wide);
  const FuseGeom G = plan.geom;
  std::vector<JitPass> jp;
  Status st;
  if (use_compiled_passes(s)) {
    st = jit_prepare(plan, s->n, s->dtype, true, &jp);
    if (!st.good()) return st;
  }
  const FOp* dops;
  const FMapDev* dmaps;
  st = upload_plan(s, plan, G, &dops, &dmaps);
  if (!st.good()) return st;
  const uint64_t ntiles = 1ull << (s->n - G.T);
  const size_t nslots = plan.grad_rows.size();
  // Up to 2^19 tiles, one workgroup per tile (a one-shot grid: the loads,
  // arithmetic and stores of different workgroups overlap); each pass's
  // partials [slot][tile] are summed right after it, so the buffer holds one
  // pass.  Larger states use a persistent grid and one buffer for all passes.
  // A grid limit below the tile count forces the persistent grid.
  const uint64_t limit = s->grid_limit > 0 ? (uint64_t)s->grid_limit : ~0ull;
  const bool oneshot = ntiles <= (1ull << 19) && limit >= ntiles;
  const unsigned grid =
      oneshot ? (unsigned)ntiles
              : (unsigned)std::min<uint64_t>(std::min<uint64_t>(ntiles, limit),
                                             (uint64_t)device_cus(s) * kAdjWgPerCu);
  const size_t prow = oneshot ? (size_t)kAdjMaxSlots : nslots;
  st = ensure_dev(s, s->red, (prow * grid + nslots + 2) * sizeof(double));
  if (!st.good()) return st;
  double* part = (double*)s->red.ptr;
  double* sums = part + prow * grid;
  for (size_t pi = 0; pi < plan.passes.size(); ++pi) {
    const Pass& p = plan.passes[pi];
    const FusedArgs A = pass_args(s, plan, p, G);
    double* pp = oneshot ? part : part + (size_t)p.grad_first * grid;
    if (!jp.empty() && jp[pi].entry >= 0) {
      void* a = s->ptr;
      void* l = lam->ptr;
      const FOp* o = dops + p.op_first;
      const void* mp = dmaps;
      unsigned long long nt = A.ntiles;
      unsigned order = 0;
      void* args[] = {&a, &l, &o, &mp, &pp, &nt, &order};
      st = launch_compiled(s, jp[pi], grid, A.ntiles, &order, args);
    } else {
      if (s->dtype == QS_C128)
        hipLaunchKernelGGL((k_fused_adj_c128<3>), dim3(grid), dim3(kFuseBlock), 0, s->stream,
                           (d2*)s->ptr, (d2*)lam->ptr, A, dops + p.op_first, dmaps, pp);
      else
        hipLaunchKernelGGL((k_fused_adj_c64<4>), dim3(grid), dim3(kFuseBlock), 0, s->stream,
                           (f4*)s->ptr, (f4*)lam->ptr, A, dops + p.op_first, dmaps, pp);
      st = last_launch("fused adjoint pass");
    }
    if (!st.good()) return st;
    if (oneshot && p.ngrad > 0) {
      st = launch_sum_rows(s, part, p.ngrad, (int)grid, sums + p.grad_first);
      if (!st.good()) return st;
    }
  }
  if (!oneshot && nslots > 0) {
    st = launch_sum_rows(s, part, (int)nslots, (int)grid, sums);
    if (!st.good()) return st;
  }
  *rows = plan.grad_rows;
  *slot_sums_dev = sums;
  return Status::ok();
}

}  // namespace qs
