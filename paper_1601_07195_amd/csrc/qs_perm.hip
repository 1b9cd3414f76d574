// qs_perm.hip -- qubit reordering in place (the state reordering of Sec. 6).
//
// Relabelling qubit q as perm[q] moves the amplitude of index i to the index
// whose bit perm[q] is bit q of i.  Every permutation of the qubits is the
// product of two involutions (a cycle x0 -> x1 -> ... -> x0 is the product
// of two reflections of its members), and an involution is a set of
// disjoint qubit swaps, which commute with each other.  Each involution is
// applied in place by
//   * k_swap_blocks, for the swaps whose two qubits both lie at or above the
//     block bits (a block is 1 KiB: 64 complex128 or 128 complex64
//     amplitudes).  Blocks move whole, one wave per block, and only blocks
//     that change place are read and written: k such swaps move
//     2 (1 - 2^-k) S bytes (S = the state's size);
//   * k_swap_tile, for the swaps that touch a block bit.  A workgroup loads
//     a tile -- the blocks selected by the upper qubits of those swaps (at
//     most four per launch, padded with unswapped qubits to four) -- into
//     LDS and writes each amplitude back at its swapped place: 2 S bytes
//     per launch.
#include <string.h>

#include <algorithm>
#include <vector>

#include "qs_device.h"
#include "qs_internal.h"

namespace qs {

constexpr int kPermBlock = 256;
constexpr int kTileHigh = 4;    // upper qubits per tile launch
constexpr int kMaxPairs = 17;   // n <= 34

struct BlockSwapArgs {
  uint64_t units;           // 16-byte units in the state
  int32_t npairs;
  int32_t lo[kMaxPairs];    // block-index bits of each swap, lo < hi
  int32_t hi[kMaxPairs];
};

// Block h (64 units) trades places with tau(h), the block index with the
// bits of every swap exchanged; the wave whose block has the smaller index
// of the two does the exchange, the other and every fixed block do nothing.
// A wave takes kSwapBlocks consecutive blocks per step and issues all their
// loads before any store, to keep more bytes in flight.
constexpr int kSwapBlocks = 4;

__global__ void __launch_bounds__(kPermBlock)
k_swap_blocks(u64x2* __restrict__ a, BlockSwapArgs A) {
  constexpr int W = kPermBlock / 64;
  const uint64_t nwaves = (uint64_t)gridDim.x * W;
  const uint64_t lane = threadIdx.x & 63;
  const uint64_t nsteps = A.units / (64 * kSwapBlocks);
  // the wave index through readfirstlane: block indices, partners and the
  // move test are then scalar, and the branch is uniform
  const uint64_t w0 = (uint64_t)blockIdx.x * W + (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  for (uint64_t c = w0; c < nsteps; c += nwaves) {
    uint64_t hs[kSwapBlocks], xs[kSwapBlocks];
    u64x2 vp[kSwapBlocks], vq[kSwapBlocks];
#pragma unroll
    for (int i = 0; i < kSwapBlocks; ++i) {
      const uint64_t h = c * kSwapBlocks + i;
      uint64_t x = h;
      for (int j = 0; j < A.npairs; ++j) {
        const uint64_t d = ((h >> A.lo[j]) ^ (h >> A.hi[j])) & 1ull;
        x ^= (d << A.lo[j]) | (d << A.hi[j]);
      }
      hs[i] = h;
      xs[i] = x;
      if (x > h) {
        vp[i] = gload<true>(a + ((h << 6) | lane));
        vq[i] = gload<true>(a + ((x << 6) | lane));
      }
    }
#pragma unroll
    for (int i = 0; i < kSwapBlocks; ++i)
      if (xs[i] > hs[i]) {
        gstore<true>(a + ((hs[i] << 6) | lane), vq[i]);
        gstore<true>(a + ((xs[i] << 6) | lane), vp[i]);
      }
  }
}

struct TileSwapArgs {
  uint64_t ntiles;
  int32_t L;                // low amplitude bits of a tile (a block, or the whole state)
  int32_t kh;               // upper qubits in the tile, <= kTileHigh
  int32_t hq[kTileHigh];    // their positions, ascending, all >= L
  int32_t npairs;
  int32_t pa[8], pb[8];     // the swaps as tile-element bits (element bit L + j is qubit hq[j])
};

__device__ __forceinline__ uint64_t tile_elem_index(uint64_t base, uint32_t e, const TileSwapArgs& A) {
  uint64_t g = base | (e & ((1u << A.L) - 1u));
  for (int j = 0; j < A.kh; ++j) g |= (uint64_t)((e >> (A.L + j)) & 1u) << A.hq[j];
  return g;
}

__device__ __forceinline__ uint32_t tile_swapped(uint32_t e, const TileSwapArgs& A) {
  uint32_t x = e;
  for (int j = 0; j < A.npairs; ++j) {
    const uint32_t d = ((e >> A.pa[j]) ^ (e >> A.pb[j])) & 1u;
    x ^= (d << A.pa[j]) | (d << A.pb[j]);
  }
  return x;
}

// complex128: one amplitude per 16-byte unit; a full tile is 1024 amplitudes,
// four per thread, whose loads are all issued before the LDS writes.
__global__ void __launch_bounds__(kPermBlock)
k_swap_tile_c128(d2* __restrict__ a, TileSwapArgs A) {
  constexpr int EMAX = 1 << (6 + kTileHigh), PER = EMAX / kPermBlock;
  __shared__ d2 lds[EMAX];
  const uint32_t E = 1u << (A.L + A.kh);
  for (uint64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    uint64_t base = tile << A.L;
    for (int j = 0; j < A.kh; ++j) base = insert0(base, A.hq[j]);
    d2 v[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t e = threadIdx.x + i * kPermBlock;
      if (e < E) v[i] = gload<true>(a + tile_elem_index(base, e, A));
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t e = threadIdx.x + i * kPermBlock;
      if (e < E) lds[e] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t e = threadIdx.x + i * kPermBlock;
      if (e < E) gstore<true>(a + tile_elem_index(base, e, A), lds[tile_swapped(e, A)]);
    }
    __syncthreads();  // the next tile reuses the LDS
  }
}

// complex64: two amplitudes per 16-byte unit (bit 0 inside the unit); a full
// tile is 2048 amplitudes, four units per thread.
__global__ void __launch_bounds__(kPermBlock)
k_swap_tile_c64(f4* __restrict__ a, TileSwapArgs A) {
  constexpr int EMAX = 1 << (7 + kTileHigh), PER = EMAX / 2 / kPermBlock;
  __shared__ f2 lds[EMAX];
  const uint32_t EU = 1u << (A.L + A.kh - 1);
  for (uint64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    uint64_t base = tile << A.L;
    for (int j = 0; j < A.kh; ++j) base = insert0(base, A.hq[j]);
    f4 w[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t v = threadIdx.x + i * kPermBlock;
      if (v < EU) w[i] = gload<true>(a + (tile_elem_index(base, 2 * v, A) >> 1));
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t v = threadIdx.x + i * kPermBlock;
      if (v < EU) {
        lds[2 * v] = f2{w[i].x, w[i].y};
        lds[2 * v + 1] = f2{w[i].z, w[i].w};
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const uint32_t v = threadIdx.x + i * kPermBlock;
      if (v < EU) {
        const f2 x0 = lds[tile_swapped(2 * v, A)], x1 = lds[tile_swapped(2 * v + 1, A)];
        gstore<true>(a + (tile_elem_index(base, 2 * v, A) >> 1), f4{x0.x, x0.y, x1.x, x1.y});
      }
    }
    __syncthreads();
  }
}

// Amplitude bits of one 1 KiB block.
static int block_bits(int dtype) { return dtype == QS_C128 ? 6 : 7; }

// The disjoint swaps of involution inv (inv[inv[q]] == q), in place.
static Status apply_involution(StateImpl* s, const std::vector<int>& inv) {
  const int n = s->n;
  const int C = block_bits(s->dtype);
  const int Lb = std::min(C, n);
  std::vector<std::pair<int, int>> low_low, low_high, high_high;
  for (int q = 0; q < n; ++q) {
    const int r = inv[q];
    if (r <= q) continue;
    if (q >= Lb) high_high.push_back({q, r});
    else if (r < Lb) low_low.push_back({q, r});
    else low_high.push_back({q, r});
  }
  // swaps touching a block bit: tile launches of at most kTileHigh upper qubits
  size_t next = 0;
  while (!low_low.empty() || next < low_high.size()) {
    TileSwapArgs A;
    memset(&A, 0, sizeof(A));
    A.L = Lb;
    std::vector<std::pair<int, int>> chunk(low_high.begin() + next,
                                           low_high.begin() + std::min(low_high.size(), next + kTileHigh));
    next += chunk.size();
    // tile qubits above the block bits: the chunk's upper qubits, padded
    // with the lowest other qubits (no swap) up to kTileHigh, so that every
    // thread moves several amplitudes
    std::vector<int> hq;
    for (auto pr : chunk) hq.push_back(pr.second);
    for (int q = Lb; q < n && (int)hq.size() < kTileHigh; ++q) {
      bool taken = false;
      for (auto pr : low_high) taken |= pr.second == q;
      for (auto pr : high_high) taken |= pr.first == q || pr.second == q;
      if (!taken) hq.push_back(q);
    }
    std::sort(hq.begin(), hq.end());
    A.kh = (int)hq.size();
    for (int j = 0; j < A.kh; ++j) A.hq[j] = hq[j];
    for (auto pr : chunk) {
      const int j = (int)(std::find(hq.begin(), hq.end(), pr.second) - hq.begin());
      A.pa[A.npairs] = pr.first;
      A.pb[A.npairs++] = Lb + j;
    }
    for (auto pr : low_low) {
      A.pa[A.npairs] = pr.first;
      A.pb[A.npairs++] = pr.second;
    }
    low_low.clear();
    if (A.L + A.kh > n || A.npairs > 8) return Status{QS_EINVAL, "permute: bad tile plan"};
    A.ntiles = 1ull << (n - A.L - A.kh);
    // one workgroup per tile (a one-shot grid measured 15 % faster than a
    // grid-stride loop over 2^16 workgroups)
    const unsigned grid = (unsigned)std::min<uint64_t>(A.ntiles, 1u << 30);
    if (s->dtype == QS_C128)
      hipLaunchKernelGGL(k_swap_tile_c128, dim3(grid), dim3(kPermBlock), 0, s->stream, (d2*)s->ptr, A);
    else
      hipLaunchKernelGGL(k_swap_tile_c64, dim3(grid), dim3(kPermBlock), 0, s->stream, (f4*)s->ptr, A);
    Status st = hip_status(hipGetLastError(), "permute (tile)");
    if (!st.good()) return st;
  }
  if (!high_high.empty()) {
    BlockSwapArgs A;
    memset(&A, 0, sizeof(A));
    A.units = ((uint64_t)1 << n) * amp_bytes(s->dtype) / 16;
    for (auto pr : high_high) {
      A.lo[A.npairs] = pr.first - C;
      A.hi[A.npairs++] = pr.second - C;
    }
    if (A.units % (64 * kSwapBlocks)) return Status{QS_EINVAL, "permute: bad block plan"};
    const uint64_t want = A.units / (64 * kSwapBlocks) / (kPermBlock / 64);
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(want, 1u << 14));
    // three waves per SIMD: 2 % faster than uncapped for a swap of two upper qubits
    hipLaunchKernelGGL(k_swap_blocks, dim3(grid), dim3(kPermBlock), stream_lds(kPermBlock, 0, 3), s->stream, (u64x2*)s->ptr, A);
    Status st = hip_status(hipGetLastError(), "permute (blocks)");
    if (!st.good()) return st;
  }
  return Status::ok();
}

Status launch_permute(StateImpl* s, const int32_t* perm) {
  const int n = s->n;
  // cycle x_0 -> x_1 -> ... -> x_{k-1} (perm[x_i] = x_{i+1}) = alpha after
  // beta, with beta(x_i) = x_{-i} and alpha(x_i) = x_{1-i} (indices mod k)
  std::vector<int> alpha(n), beta(n);
  std::vector<char> seen(n, 0);
  for (int q = 0; q < n; ++q) {
    if (seen[q]) continue;
    std::vector<int> cyc;
    for (int x = q; !seen[x]; x = perm[x]) {
      seen[x] = 1;
      cyc.push_back(x);
    }
    const int k = (int)cyc.size();
    for (int i = 0; i < k; ++i) {
      beta[cyc[i]] = cyc[(k - i) % k];
      alpha[cyc[i]] = cyc[(k + 1 - i) % k];
    }
  }
  Status st = apply_involution(s, beta);
  if (!st.good()) return st;
  return apply_involution(s, alpha);
}

}  // namespace qs
