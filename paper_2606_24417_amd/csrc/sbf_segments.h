// Segment updates of the 4-word-shard insert kernels (kernels_rolling.hip,
// kernels_param.hip): a lane's finished super-k-mer segments (shard and four
// mask words) are buffered in LDS and applied to the filter as atomic ORs or
// as read-OR-writes by lane pairs.
#pragma once

#include "sbf_device.h"

namespace sbf {
namespace {

// How a finished segment reaches the filter.  Global atomics on this GPU run
// at a fixed ~27 G ops/s whatever the filter size, while plain random 32-byte
// read-modify-writes run several times faster, so the default insert is two
// passes over the same k-mers:
//   kStore:  read the shard, OR the segment's masks, write it back (a plain
//            load and a store that writes through to the device's coherence
//            point, store_pair_coherent; a read-modify-write racing with
//            another one on the same shard can lose that one's bits, never
//            older bits);
//   repair:  a query walk with REPAIR (query_lane_kernel, query_param_kernel)
//            tests every valid k-mer against its shard and atomically ORs
//            the bits still missing (a few percent of the segments in cache,
//            fewer out of cache).
// After both passes the filter is exactly the OR of every segment, as with
// kAtomic (the paper's four atomicOr per run head).
enum InsertMode : int { kAtomic = 0, kStore = 1 };

// A lane buffers finished segments in LDS and applies them every few k-mers
// (and at the end), loading all buffered shards before the first store, so
// one wait covers several read-modify-writes; a segment that finds the
// buffer full is applied with atomics at once.  kQueueSlots segments per
// lane unless the kernel asks for fewer (LDS per lane: 36 bytes a slot).
constexpr int kQueueSlots = 3;

template <int NW>
__device__ __forceinline__ void atomic_segment(uint64_t *__restrict__ words, uint32_t shard, const uint64_t (&m)[4]) {
  uint64_t *p = words + 4ull * (uint64_t)shard;
#pragma unroll
  for (int w = 0; w < NW; ++w) atomic_or64(p + w, m[w]);
}

// Lane-private LDS buffer of finished segments (structure of arrays, so that
// the 64 lanes of a wave touch consecutive words).
template <int WG, int SLOTS = kQueueSlots>
struct SegmentBuffer {
  uint32_t shard[SLOTS][WG];
  uint64_t mask[SLOTS][4][WG];
};

template <int NW, int MODE, int WG, int SLOTS>
__device__ __forceinline__ void push_segment(SegmentBuffer<WG, SLOTS> &b, int &n, uint64_t *__restrict__ words,
                                             uint32_t shard, const uint64_t (&m)[4]) {
  if (MODE == kAtomic || n >= SLOTS) {
    atomic_segment<NW>(words, shard, m);
    return;
  }
  const int t = threadIdx.x;
  b.shard[n][t] = shard;
#pragma unroll
  for (int w = 0; w < 4; ++w) b.mask[n][w][t] = m[w];
  ++n;
}

// Apply the buffered segments: all loads first, then the stores.
template <int MODE, int WG, int SLOTS>
__device__ __forceinline__ void drain_segments(SegmentBuffer<WG, SLOTS> &b, int &n, uint64_t *__restrict__ words) {
  if constexpr (MODE != kAtomic) {
    // The lanes of each aligned pair read (and below write) both 16-byte
    // halves of one shard in one instruction: load A takes the even lane's
    // shard (low half by the even lane, high half by the odd lane), load B
    // the odd lane's; afterwards each lane swaps the half it read for its
    // partner.  A shard moved by two lanes of one instruction is one 32-byte
    // access instead of two 16-byte ones.
    const int t = threadIdx.x;
    const bool odd = (threadIdx.x & 1) != 0;
    uint32_t sh[SLOTS];
    uint64_t m[SLOTS][4], old[SLOTS][4];
    uint4 la[SLOTS], lb[SLOTS];
    bool own[SLOTS], p_own[SLOTS];
#pragma unroll
    for (int k = 0; k < SLOTS; ++k) {
      own[k] = k < n;
      sh[k] = own[k] ? b.shard[k][t] : 0u;
      if (own[k]) {
#pragma unroll
        for (int w = 0; w < 4; ++w) m[k][w] = b.mask[k][w][t];
      }
      p_own[k] = pair_swap((uint32_t)own[k]) != 0u;
      const uint32_t ps = pair_swap(sh[k]);
      la[k] = make_uint4(0, 0, 0, 0);
      lb[k] = make_uint4(0, 0, 0, 0);
      if (odd ? p_own[k] : own[k])
        la[k] = *reinterpret_cast<const uint4 *>(words + 4ull * (uint64_t)(odd ? ps : sh[k]) + (odd ? 2 : 0));
      if (odd ? own[k] : p_own[k])
        lb[k] = *reinterpret_cast<const uint4 *>(words + 4ull * (uint64_t)(odd ? sh[k] : ps) + (odd ? 2 : 0));
    }
    // Wait for the loads here, on every path: the stores below are
    // conditional, and a load the compiler still counts as outstanding after
    // them would make the next write of its register wait for the stores too
    // (the vector-memory counter retires in order).  s_waitcnt vmcnt(0), the
    // other counters left at their maxima.
    __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
    for (int k = 0; k < SLOTS; ++k) {
      // the even lane keeps A (its low half) and receives its high half from
      // the odd lane's A; the odd lane keeps B (its high half) and receives
      // its low half from the even lane's B
      const uint4 x = odd ? la[k] : lb[k];
      const uint4 px = make_uint4(pair_swap(x.x), pair_swap(x.y), pair_swap(x.z), pair_swap(x.w));
      const uint4 lo = odd ? px : la[k], hi = odd ? lb[k] : px;
      old[k][0] = ((uint64_t)lo.y << 32) | lo.x;
      old[k][1] = ((uint64_t)lo.w << 32) | lo.z;
      old[k][2] = ((uint64_t)hi.y << 32) | hi.x;
      old[k][3] = ((uint64_t)hi.w << 32) | hi.z;
    }
    // a later buffered segment on the same shard carries the earlier masks,
    // since its read does not see the earlier write of this lane
#pragma unroll
    for (int k = 1; k < SLOTS; ++k)
#pragma unroll
      for (int j = 0; j < k; ++j)
        if (k < n && sh[k] == sh[j])
#pragma unroll
          for (int w = 0; w < 4; ++w) m[k][w] |= m[j][w];
    // Stores that write through to the coherence point (store_pair_coherent)
    // cost two partial writes when one lane writes a 32-byte shard as two
    // 16-byte halves, but one when two lanes write its halves in the same
    // instruction.  So the lanes of each aligned pair write each other's
    // shard halves: in store A the pair writes the even lane's shard (low half
    // from the even lane, high half from the odd lane), in store B the odd
    // lane's shard.  A given half of a shard is always written by the same
    // lane of the pair, so a lane's stores to one shard stay in order.
#pragma unroll
    for (int k = 0; k < SLOTS; ++k) {
      uint64_t v[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) v[w] = own[k] ? (old[k][w] | m[k][w]) : 0ull;
      const uint32_t s = sh[k];
      const uint32_t ps = pair_swap(s);
      // the half the other lane writes: the even lane's high, the odd lane's low
      const uint64_t px0 = pair_swap64(odd ? v[0] : v[2]);
      const uint64_t px1 = pair_swap64(odd ? v[1] : v[3]);
      if (odd ? p_own[k] : own[k])
        store_pair_coherent(words + 4ull * (uint64_t)(odd ? ps : s) + (odd ? 2 : 0), odd ? px0 : v[0],
                            odd ? px1 : v[1]);
      if (odd ? own[k] : p_own[k])
        store_pair_coherent(words + 4ull * (uint64_t)(odd ? s : ps) + (odd ? 2 : 0), odd ? v[2] : px0,
                            odd ? v[3] : px1);
    }
    n = 0;
  }
}

}  // namespace
}  // namespace sbf
