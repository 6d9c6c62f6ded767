// Tile helpers shared by the super-k-mer kernels (kernels_rolling.hip,
// kernels_wide.hip): the granules a lane reads, k-mer validity over a lane's
// window, m-mer and s-mer windows of the staged 2-bit codes, and the tile
// scheduler of plain and persistent (work-queue) launches.
#pragma once

#include "sbf_device.h"
#include "sbf_internal.h"

namespace sbf {

// Granules (16 bases) a lane reads: L + K - 1 bases plus one for the funnel
// shift of the last window.
template <int K, int L>
constexpr int lane_granules() { return (L + K - 1 + 15) / 16 + 1; }

// Bit r: k-mer r of a lane is valid (all its bases are A/C/G/T and no record
// starts inside it).  The lane's bases start at granule g0 of the staged
// tile; k-mers 0..31 are judged on the 64 bases from granule g0 on, k-mers
// 32..L-1 on the 64 bases from granule g0 + 2 on.
template <int K, int L>
__device__ __forceinline__ uint64_t lane_kmer_valid(const uint32_t *s_vb, int g0) {
  static_assert(L % 16 == 0 && L <= 64 && (L <= 32 ? L + K - 1 <= 64 : L + K - 1 <= 96),
                "k-mer validity comes from one or two 64-base windows");
  auto window = [&](int g) {
    uint64_t vbits = 0, sbits = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint32_t vb = s_vb[g0 + g + i];
      vbits |= (uint64_t)(vb & 0xFFFFu) << (16 * i);
      sbits |= (uint64_t)(vb >> 16) << (16 * i);
    }
    return kmer_valid_mask<K>(vbits, sbits);
  };
  if constexpr (L <= 32) {
    return window(0) & ((1ull << L) - 1);
  } else {
    return (window(0) & 0xFFFFFFFFull) | ((window(2) & ((1ull << (L - 32)) - 1)) << 32);
  }
}

// Tile scheduler.  A plain launch runs tile blockIdx.x once; a persistent
// launch (counter not null) keeps taking the next tile index from a device
// counter (the work queue) until all ntiles are taken.  The decision is
// uniform over the workgroup, so every wave leaves the loop together.
struct TileQueue {
  uint32_t *counter;
  uint32_t ntiles;
};

__device__ __forceinline__ bool next_tile(const TileQueue &q, uint32_t *s_slot, bool first, uint64_t &tile) {
  if (q.counter == nullptr) {
    tile = blockIdx.x;
    return first;
  }
  __syncthreads();  // every lane has read the previous slot
  if (threadIdx.x == 0) *s_slot = atomicAdd(q.counter, 1u);
  __syncthreads();
  tile = *s_slot;
  return tile < q.ntiles;
}

// Minimizer hash h_M of the m-mer at window position j (2m-bit value, first
// base most significant; m <= 16 fits 32 bits).  SPLIT selects the split
// 32-bit multiply for m <= 16 (same value).
template <int M, bool SPLIT = false>
__device__ __forceinline__ uint64_t mmer_hash(const uint32_t *a, int j) {
  static_assert(M >= 1 && M <= 32, "m-mers fit 64 bits");
  if constexpr (M <= 16) {
    const uint32_t y = win32(a, j) >> (32 - 2 * M);
    return SPLIT ? minimizer_hash32_split(y) : minimizer_hash32(y);
  } else {
    const uint32_t hi = win32(a, j) >> (64 - 2 * M);
    const uint32_t lo = win32(a, j + M - 16);
    return minimizer_hash(((uint64_t)hi << 32) | lo);
  }
}

template <int S>
__device__ __forceinline__ uint64_t smer_at(const uint32_t *a, int j) {
  if constexpr (S <= 16) {
    return (uint64_t)(win32(a, j) >> (32 - 2 * S));
  } else {
    const uint32_t hi = win32(a, j) >> (64 - 2 * S);
    const uint32_t lo = win32(a, j + S - 16);
    return ((uint64_t)hi << 32) | lo;
  }
}

// Grid of a launch over ntiles tiles: one workgroup per tile, or a persistent
// grid that takes tiles from the queue counter `slot` (reset first).  A batch
// of no more tiles than the persistent grid has workgroups runs as a plain
// launch: the same tiles, one per workgroup, without the counter reset.
inline hipError_t tile_grid(uint64_t ntiles, const LaunchShape &ls, int slot, hipStream_t st, TileQueue &tq,
                     unsigned &grid) {
  tq.counter = nullptr;
  tq.ntiles = (uint32_t)ntiles;
  grid = (unsigned)ntiles;
  if (ls.queue != nullptr && ls.persistent_wgs != 0 && ntiles > ls.persistent_wgs) {
    tq.counter = ls.queue + slot;
    grid = ls.persistent_wgs;
    return launch_fill_u32(tq.counter, 1, 0u, st);
  }
  return hipSuccess;
}

#define SBF_LAUNCH_TILES(KERNEL, WGS, NTILES, SLOT, ...)                      \
  do {                                                                          \
    TileQueue tq_;                                                              \
    unsigned grid_;                                                             \
    hipError_t e_ = tile_grid((NTILES), ls, (SLOT), st, tq_, grid_);            \
    if (e_ != hipSuccess) return e_;                                            \
    hipLaunchKernelGGL(KERNEL, dim3(grid_), dim3(WGS), 0, st, __VA_ARGS__, tq_); \
    e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess) return e_;                                            \
  } while (0)

}  // namespace sbf
