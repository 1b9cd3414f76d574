// qs_fused.hip -- one HBM round trip for a whole block of gates.
//
// The GPU form of cache blocking by gate fusion (qHiPSTER Sec. 4.4, Fig. 4):
// a workgroup loads one tile of 2^T amplitudes (the low qubits plus the
// pass's high qubits, see qs_plan.cpp) into registers -- 2^NREG amplitudes
// per thread -- applies every gate of the pass there, and writes the tile
// back.  Register-bit gates are plain register arithmetic; a remap moves the
// tile through LDS so that other tile bits become register bits; diagonal
// gates scale each amplitude by the entry its target bit selects, wherever
// that bit lives (register, thread index, or outside the tile).
#include <string.h>

#include <algorithm>

#include "qs_device.h"
#include "qs_internal.h"

namespace qs {

constexpr int kFuseBlock = 1 << kFuseThreadBits;  // 256

struct FusedArgs {
  uint64_t ntiles;
  int L, nh, nops, map_load, map_store;
  int8_t hpos[8];
};

template <typename R>
struct LdsAmp;
template <>
struct LdsAmp<double> {
  using T = d2;
  // 16-byte elements: fold 3-bit chunks of the index into its low 3 bits
  static __device__ __forceinline__ int swz(int j) {
    return j ^ (((j >> 3) ^ (j >> 6) ^ (j >> 9)) & 7);
  }
};
template <>
struct LdsAmp<float> {
  using T = f2;
  // 8-byte elements: fold 4-bit chunks into the low 4 bits
  static __device__ __forceinline__ int swz(int j) {
    return j ^ (((j >> 4) ^ (j >> 8) ^ (j >> 12)) & 15);
  }
};

// Global qubit of tile bit tb.
__device__ __forceinline__ int gq(int tb, const FusedArgs& A) {
  return tb < A.L ? tb : A.hpos[tb - A.L];
}

// Offsets of a mapping: the thread part (per thread) and the register part
// for register index r (uniform), either as tile-local indices (LDS) or as
// global amplitude offsets.
template <int NREG>
__device__ __forceinline__ uint64_t thr_off_global(const FMap& m, const FusedArgs& A) {
  uint64_t o = 0;
#pragma unroll
  for (int i = 0; i < kFuseThreadBits; ++i)
    o |= (uint64_t)((threadIdx.x >> i) & 1) << gq(m.thr[i], A);
  return o;
}
template <int NREG>
__device__ __forceinline__ uint64_t reg_off_global(const FMap& m, const FusedArgs& A, int r) {
  uint64_t o = 0;
#pragma unroll
  for (int k = 0; k < NREG; ++k)
    if ((r >> k) & 1) o |= 1ull << gq(m.reg[k], A);
  return o;
}
template <int NREG>
__device__ __forceinline__ int thr_off_tile(const FMap& m) {
  int o = 0;
#pragma unroll
  for (int i = 0; i < kFuseThreadBits; ++i) o |= ((threadIdx.x >> i) & 1) << m.thr[i];
  return o;
}
template <int NREG>
__device__ __forceinline__ int reg_off_tile(const FMap& m, int r) {
  int o = 0;
#pragma unroll
  for (int k = 0; k < NREG; ++k)
    if ((r >> k) & 1) o |= 1 << m.reg[k];
  return o;
}

// Gate on register bit K for every register pair (r, r | 2^K), optionally
// controlled by register bit creg.
template <int K, int RA, typename R>
__device__ __forceinline__ void reg_gate(R* re, R* im, const Mat<R>& q, int creg) {
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    if (r & (1 << K)) continue;
    const int r1 = r | (1 << K);
    if (creg >= 0 && !((r >> creg) & 1)) continue;
    mat_apply(q, re[r], im[r], re[r1], im[r1]);
  }
}

template <typename R>
__device__ __forceinline__ Mat<R> load_mat(const double* m) {
  Mat<R> q;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    q.r[e] = (R)m[2 * e];
    q.i[e] = (R)m[2 * e + 1];
  }
  return q;
}

// Apply ops[0 .. nops) to the register tile.  `base` is the tile's global
// index base (bits outside the tile).
template <typename R, int NREG>
__device__ __forceinline__ void run_ops(R* re, R* im, typename LdsAmp<R>::T* lds,
                                        const FOp* __restrict__ ops, int nops,
                                        const FMap* __restrict__ maps, uint64_t base) {
  constexpr int RA = 1 << NREG;
  using LT = typename LdsAmp<R>::T;
  for (int o = 0; o < nops; ++o) {
    const FOp& op = ops[o];
    const int kind = op.kind;
    if (kind == kOpRemap) {
      const FMap mo = maps[op.aux], mn = maps[op.tgt];
      const int to = thr_off_tile<NREG>(mo), tn = thr_off_tile<NREG>(mn);
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        LT v;
        v.x = re[r];
        v.y = im[r];
        lds[LdsAmp<R>::swz(to | reg_off_tile<NREG>(mo, r))] = v;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        const LT v = lds[LdsAmp<R>::swz(tn | reg_off_tile<NREG>(mn, r))];
        re[r] = v.x;
        im[r] = v.y;
      }
      __syncthreads();
      continue;
    }
    const int cw = op.ctl >> 8, ci = op.ctl & 255;
    bool on = true;
    int creg = -1;
    if (cw == kInThread) on = (threadIdx.x >> ci) & 1;
    else if (cw == kOutside) on = (base >> ci) & 1;
    else if (cw == kInReg) creg = ci;
    if (!on) continue;
    if (kind == kOpU) {
      const Mat<R> q = load_mat<R>(op.m);
      switch (op.tgt) {
        case 0: reg_gate<0, RA>(re, im, q, creg); break;
        case 1: reg_gate<1, RA>(re, im, q, creg); break;
        case 2: reg_gate<2, RA>(re, im, q, creg); break;
        case 3: reg_gate<3, RA>(re, im, q, creg); break;
        default:
          if constexpr (NREG > 4) reg_gate<(NREG > 4 ? 4 : 0), RA>(re, im, q, creg);
          break;
      }
    } else {  // diagonal
      const R d0r = (R)op.m[0], d0i = (R)op.m[1], d1r = (R)op.m[6], d1i = (R)op.m[7];
      const int tw = op.tgt >> 8, tix = op.tgt & 255;
      const int fixed = (tw == kInThread) ? (int)((threadIdx.x >> tix) & 1)
                                          : (tw == kOutside ? (int)((base >> tix) & 1) : -1);
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        if (creg >= 0 && !((r >> creg) & 1)) continue;
        const int bit = fixed >= 0 ? fixed : ((r >> tix) & 1);
        const R dr = bit ? d1r : d0r, di = bit ? d1i : d0i;
        const R xr = re[r], xi = im[r];
        re[r] = dr * xr - di * xi;
        im[r] = dr * xi + di * xr;
      }
    }
  }
}

__device__ __forceinline__ uint64_t tile_base(uint64_t tile, const FusedArgs& A) {
  uint64_t x = tile << A.L;
  for (int h = 0; h < A.nh; ++h) x = insert0(x, A.hpos[h]);
  return x;
}

// complex128: one d2 per amplitude.
template <int NREG>
__global__ void __launch_bounds__(kFuseBlock)
k_fused_c128(d2* __restrict__ a, FusedArgs A, const FOp* __restrict__ ops,
             const FMap* __restrict__ maps) {
  constexpr int RA = 1 << NREG;
  __shared__ d2 lds[RA * kFuseBlock];
  double re[RA], im[RA];
  const FMap ml = maps[A.map_load], ms = maps[A.map_store];
  const uint64_t tl = thr_off_global<NREG>(ml, A), ts = thr_off_global<NREG>(ms, A);
  for (uint64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const uint64_t base = tile_base(tile, A);
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const d2 v = gload<true>(a + (base | tl | reg_off_global<NREG>(ml, A, r)));
      re[r] = v.x;
      im[r] = v.y;
    }
    run_ops<double, NREG>(re, im, lds, ops, A.nops, maps, base);
#pragma unroll
    for (int r = 0; r < RA; ++r)
      gstore<true>(a + (base | ts | reg_off_global<NREG>(ms, A, r)), d2{re[r], im[r]});
  }
}

// complex64: 16-byte units of two amplitudes; register bit 0 is qubit 0 at
// load and store, so registers (2u, 2u + 1) form one unit.
template <int NREG>
__global__ void __launch_bounds__(kFuseBlock)
k_fused_c64(f4* __restrict__ a, FusedArgs A, const FOp* __restrict__ ops,
            const FMap* __restrict__ maps) {
  constexpr int RA = 1 << NREG;
  __shared__ f2 lds[RA * kFuseBlock];
  float re[RA], im[RA];
  const FMap ml = maps[A.map_load], ms = maps[A.map_store];
  const uint64_t tl = thr_off_global<NREG>(ml, A), ts = thr_off_global<NREG>(ms, A);
  for (uint64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const uint64_t base = tile_base(tile, A);
#pragma unroll
    for (int r = 0; r < RA; r += 2) {
      const f4 v = gload<true>(a + ((base | tl | reg_off_global<NREG>(ml, A, r)) >> 1));
      re[r] = v.x;
      im[r] = v.y;
      re[r + 1] = v.z;
      im[r + 1] = v.w;
    }
    run_ops<float, NREG>(re, im, lds, ops, A.nops, maps, base);
#pragma unroll
    for (int r = 0; r < RA; r += 2)
      gstore<true>(a + ((base | ts | reg_off_global<NREG>(ms, A, r)) >> 1),
                   f4{re[r], im[r], re[r + 1], im[r + 1]});
  }
}

static Status last_launch(const char* what) { return hip_status(hipGetLastError(), what); }

Status run_gates(StateImpl* s, const std::vector<XGate>& gates, int flags) {
  Plan plan;
  plan_gates(s->n, s->dtype, gates, !(flags & QS_RUN_NO_FUSION), &plan);
  const FOp* dops = nullptr;
  const FMap* dmaps = nullptr;
  if (!plan.ops.empty()) {
    const size_t ob = plan.ops.size() * sizeof(FOp), mb = plan.maps.size() * sizeof(FMap);
    std::vector<char> blob(ob + mb);
    memcpy(blob.data(), plan.ops.data(), ob);
    memcpy(blob.data() + ob, plan.maps.data(), mb);
    Status st = upload_table(s, blob.data(), blob.size());
    if (!st.good()) return st;
    dops = (const FOp*)s->table.ptr;
    dmaps = (const FMap*)((const char*)s->table.ptr + ob);
  }
  const FuseGeom G = fuse_geom(s->dtype);
  for (const Pass& p : plan.passes) {
    Status st;
    if (p.kind == kPass1q) {
      st = launch_apply_1q(s, gates[p.gate].target, gates[p.gate].m);
    } else if (p.kind == kPassCU) {
      st = launch_apply_cu(s, gates[p.gate].control, gates[p.gate].target, gates[p.gate].m);
    } else {
      FusedArgs A;
      memset(&A, 0, sizeof(A));
      A.ntiles = 1ull << (s->n - G.T);
      A.L = G.L;
      A.nh = p.nh;
      A.nops = p.nops;
      A.map_load = p.map_load;
      A.map_store = p.map_store;
      for (int h = 0; h < p.nh; ++h) A.hpos[h] = p.hpos[h];
      const unsigned grid = (unsigned)std::min<uint64_t>(A.ntiles, (1ull << 31) / kFuseBlock);
      if (s->dtype == QS_C128)
        hipLaunchKernelGGL((k_fused_c128<4>), dim3(grid), dim3(kFuseBlock), 0, s->stream,
                           (d2*)s->ptr, A, dops + p.op_first, dmaps);
      else
        hipLaunchKernelGGL((k_fused_c64<5>), dim3(grid), dim3(kFuseBlock), 0, s->stream,
                           (f4*)s->ptr, A, dops + p.op_first, dmaps);
      st = last_launch("fused pass");
    }
    if (!st.good()) return st;
  }
  return Status::ok();
}

}  // namespace qs
