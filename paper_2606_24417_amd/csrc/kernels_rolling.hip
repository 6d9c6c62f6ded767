// Super-k-mer ("rolling") insert and query kernels for gfx950.
//
// Instead of one k-mer per lane (the paper's Algorithms 1 and 2 repeat k-m+1
// m-mer hashes and k-s+1 s-mer hashes per k-mer), each lane walks a run of L
// consecutive k-mers and hashes every m-mer and s-mer position once:
//   * the minimum over the w = k-m+1 m-mer hashes of each k-mer comes from a
//     van Herk / Gil-Werman sliding minimum (suffix minima of one block of w
//     hashes against prefix minima of the next: 3 compares per position);
//   * consecutive valid k-mers with the same shard form a segment (the
//     super-k-mer of Section "Minimizers and Super-k-mers", split where the
//     shard changes); the lane ORs the one-hot masks of the segment's s-mers
//     in registers and writes the segment's shard once when it ends - the
//     per-lane form of the paper's segmented reduction (Algorithm 1) - either
//     as four 64-bit atomic ORs or, by default, as a read-OR-write (plain
//     load, device-coherent store) followed by a second pass that atomically
//     restores any bit a racing write dropped;
//   * the default query (query_lane_kernel) walks k-mers the same way, builds
//     each k-mer's mask of (k-s+1)*H bits and tests it against the k-mer's
//     shard, which a lane loads once per run of equal shards (the paper's
//     shard sharing, Algorithm 2); query_rolling_kernel instead stages shards
//     and bit addresses in LDS and tests one k-mer per lane, the first lane of
//     each run of equal shards loading the shard for the others (leader load
//     and ds_bpermute broadcast).
// Every result is bit-identical to the per-k-mer definition: OR is
// commutative and idempotent, and a k-mer is tested in its own shard.
#include "sbf_device.h"
#include "sbf_internal.h"
#include "sbf_segments.h"
#include "sbf_tiles.h"

#include <type_traits>

namespace sbf {
namespace {

template <int H>
__device__ __forceinline__ void smer_onehots(uint64_t g, uint64_t (&oh)[4]) {
  oh[0] = oh[1] = oh[2] = oh[3] = 0;
#pragma unroll
  for (int t = 0; t < H; ++t) oh[t & 3] |= 1ull << bit_address<H>(g, t);
}

// The lane kernels drain their segment buffer every kSubRun k-mers.  With a
// mean super-k-mer of about 8.5 k-mers, a drain every 12 k-mers finds 1.4
// segments on average.
constexpr int kSubRun = 12;

// ---------------------------------------------------------------------------
// Insert: WG lanes x L k-mers per workgroup tile.
// ---------------------------------------------------------------------------
template <int K, int S, int M, int H, int L, int WG, int MODE>
__global__ __launch_bounds__(WG) void insert_rolling_kernel(const uint8_t *__restrict__ seq, uint64_t len,
                                                            const uint32_t *__restrict__ starts, int aligned16,
                                                            uint64_t *__restrict__ words, uint32_t shard_mask, TileQueue tq) {
  constexpr int W = K - M + 1;
  constexpr int Z = K - S;
  constexpr int GPL = L / 16;
  constexpr int NGW = lane_granules<K, L>();
  constexpr int NGRAN = (WG - 1) * GPL + NGW;
  constexpr int NW = H < 4 ? H : 4;
  static_assert(Z >= 0 && W >= 1, "s <= k and m <= k");

  __shared__ uint32_t s_codes[NGRAN];
  __shared__ uint32_t s_vb[NGRAN];
  __shared__ SegmentBuffer<(MODE == kAtomic ? 1 : WG)> s_buf;

  __shared__ uint32_t s_next_tile;
  acquire_device();
  uint64_t tile;
  for (bool first = true; next_tile(tq, &s_next_tile, first, tile); first = false) {
  const uint64_t base = (uint64_t)tile * (uint64_t)(WG * L);
    stage_granules<WG>(seq, len, base, starts, aligned16 != 0, NGRAN, s_codes, s_vb);
    __syncthreads();

    const int g0 = threadIdx.x * GPL;
    uint32_t a[NGW];
#pragma unroll
    for (int i = 0; i < NGW; ++i) a[i] = s_codes[g0 + i];
    const uint64_t kv = lane_kmer_valid<K, L>(s_vb, g0);

    uint64_t seg[4] = {0, 0, 0, 0};  // the open segment's masks
    uint32_t cur = 0;                // and its shard
    bool open = false;
    // The lane's first finished segment is held back: the previous lane of the
    // wave absorbs it into its own last segment when both use one shard (the
    // super-k-mer crossing the lane boundary then costs one update, not two).
    uint64_t fseg[4] = {0, 0, 0, 0};
    uint32_t fsh = 0;
    bool held = false;
    int nbuf = 0;
    // every lane walks, also one without valid k-mers (it opens no segment):
    // the drains exchange data between lanes
    {
      // one-hot masks of s-mers r .. r+Z, OR-ed: A(r).  For Z = 3 the window OR
      // reuses pairs P(j) = oh(j) | oh(j+1): A(r) = P(r) | P(r+2).
      uint64_t oh[L + Z][4];
      uint64_t pr[L + Z][4];
#pragma unroll
      for (int j = 0; j < Z; ++j) smer_onehots<H>(smer_hash(smer_at<S>(a, j)), oh[j]);
      if constexpr (Z == 3) {
#pragma unroll
        for (int j = 0; j + 1 < Z; ++j)
#pragma unroll
          for (int w = 0; w < 4; ++w) pr[j][w] = oh[j][w] | oh[j + 1][w];
      }

      // van Herk sliding minimum: suf[i] = min(h[qW+i .. qW+W-1]) of block q
      uint64_t suf[W];
      {
        uint64_t hb[W];
#pragma unroll
        for (int i = 0; i < W; ++i) hb[i] = mmer_hash<M, true>(a, i);
        suf[W - 1] = hb[W - 1];
#pragma unroll
        for (int i = W - 2; i >= 0; --i) suf[i] = umin64(hb[i], suf[i + 1]);
      }

#pragma unroll
      for (int q = 0; q * W < L; ++q) {
        uint64_t hb[W];
        uint64_t pre = ~0ull;
#pragma unroll
        for (int i = 0; i < W; ++i) {
          const int r = q * W + i;
          if (r < L) {
            uint64_t mu;
            if (i == 0) {
              mu = suf[0];
            } else {
              hb[i - 1] = mmer_hash<M, true>(a, r + W - 1);
              pre = umin64(pre, hb[i - 1]);
              mu = umin64(suf[i], pre);
            }
            // newest s-mer of k-mer r
            smer_onehots<H>(smer_hash(smer_at<S>(a, r + Z)), oh[r + Z]);
            uint64_t A[4];
            if constexpr (Z == 3) {
#pragma unroll
              for (int w = 0; w < 4; ++w) {
                pr[r + 2][w] = oh[r + 2][w] | oh[r + 3][w];
                A[w] = pr[r][w] | pr[r + 2][w];
              }
            } else {
#pragma unroll
              for (int w = 0; w < 4; ++w) {
                uint64_t x = oh[r][w];
#pragma unroll
                for (int j = 1; j <= Z; ++j) x |= oh[r + j][w];
                A[w] = x;
              }
            }
            const bool v = (kv >> r) & 1ull;
            const uint32_t sh = (uint32_t)mu & shard_mask;
            const bool cont = open && v && sh == cur;
            if (open && !cont) {
              if (held) {
                push_segment<NW, MODE>(s_buf, nbuf, words, cur, seg);
              } else {
#pragma unroll
                for (int w = 0; w < 4; ++w) fseg[w] = seg[w];
                fsh = cur;
                held = true;
              }
            }
            const uint64_t keep = cont ? ~0ull : 0ull;
#pragma unroll
            for (int w = 0; w < 4; ++w) seg[w] = (seg[w] & keep) | A[w];
            open = v;
            cur = sh;
            if (r % kSubRun == kSubRun - 1 && r + 1 < L) drain_segments<MODE>(s_buf, nbuf, words);
          }
        }
        if ((q + 1) * W < L) {
          hb[W - 1] = mmer_hash<M, true>(a, (q + 1) * W + W - 1);
          suf[W - 1] = hb[W - 1];
#pragma unroll
          for (int i = W - 2; i >= 0; --i) suf[i] = umin64(hb[i], suf[i + 1]);
        }
      }
    }
    // neighbour merge inside the wave (every lane takes part in the shuffles)
    const int lane = __lane_id();
    const uint32_t n_sh = __shfl_down(fsh, 1, 64);
    const bool n_held = __shfl_down((int)held, 1, 64) != 0 && lane < 63;
    uint64_t n_m[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) n_m[w] = __shfl_down(fseg[w], 1, 64);
    const bool absorb = open && n_held && n_sh == cur;
    if (absorb) {
#pragma unroll
      for (int w = 0; w < 4; ++w) seg[w] |= n_m[w];
    }
    const bool absorbed = __shfl_up((int)absorb, 1, 64) != 0 && lane > 0;
    if (held && !absorbed) push_segment<NW, MODE>(s_buf, nbuf, words, fsh, fseg);
    if (open) push_segment<NW, MODE>(s_buf, nbuf, words, cur, seg);
    drain_segments<MODE>(s_buf, nbuf, words);
  }
}

// ---------------------------------------------------------------------------
// Query: phase 1 (16 k-mers per lane) writes shards and s-mer bit addresses to
// LDS; phase 2 tests one k-mer per lane.
// ---------------------------------------------------------------------------
template <int H>
using bit_pack_t = typename std::conditional<(H <= 4), uint32_t, uint64_t>::type;

template <int H>
__device__ __forceinline__ bit_pack_t<H> pack_bit_addresses(uint64_t g) {
  bit_pack_t<H> p = 0;
#pragma unroll
  for (int t = 0; t < H; ++t) p |= (bit_pack_t<H>)bit_address<H>(g, t) << (8 * t);
  return p;
}

template <int K, int S, int M, int H, int WG, bool SHARE>
__global__ __launch_bounds__(WG) void query_rolling_kernel(const uint8_t *__restrict__ seq, uint64_t len,
                                                           const uint32_t *__restrict__ starts, int aligned16,
                                                           const uint64_t *__restrict__ words, uint32_t shard_mask,
                                                           uint8_t *__restrict__ out, uint64_t n_out, TileQueue tq) {
  constexpr int L = 16;
  constexpr int TILE = WG * L;
  constexpr int W = K - M + 1;
  constexpr int Z = K - S;
  constexpr int NGW = lane_granules<K, L>();
  constexpr int NGRAN = (WG - 1) + NGW;
  static_assert(H <= 8, "bit addresses pack into 8 bytes");
  using Pack = bit_pack_t<H>;

  __shared__ uint32_t s_codes[NGRAN];
  __shared__ uint32_t s_vb[NGRAN];
  __shared__ uint32_t s_shard[TILE];
  __shared__ Pack s_bits[TILE + Z];
  __shared__ uint32_t s_kv[WG];

  __shared__ uint32_t s_next_tile;
  acquire_device();
  uint64_t tile;
  for (bool first = true; next_tile(tq, &s_next_tile, first, tile); first = false) {
  const uint64_t base = (uint64_t)tile * (uint64_t)TILE;
    stage_granules<WG>(seq, len, base, starts, aligned16 != 0, NGRAN, s_codes, s_vb);
    __syncthreads();

    // ---- phase 1: lane t owns k-mers 16t .. 16t+15 of the tile ----
    {
      const int t = threadIdx.x;
      uint32_t a[NGW];
      uint64_t vbits = 0, sbits = 0;
#pragma unroll
      for (int i = 0; i < NGW; ++i) {
        a[i] = s_codes[t + i];
        if (i < 4) {
          const uint32_t vb = s_vb[t + i];
          vbits |= (uint64_t)(vb & 0xFFFFu) << (16 * i);
          sbits |= (uint64_t)(vb >> 16) << (16 * i);
        }
      }
      s_kv[t] = (uint32_t)(kmer_valid_mask<K>(vbits, sbits) & 0xFFFFull);

      uint64_t suf[W];
      {
        uint64_t hb[W];
#pragma unroll
        for (int i = 0; i < W; ++i) hb[i] = mmer_hash<M, true>(a, i);
        suf[W - 1] = hb[W - 1];
#pragma unroll
        for (int i = W - 2; i >= 0; --i) suf[i] = umin64(hb[i], suf[i + 1]);
      }
#pragma unroll
      for (int q = 0; q * W < L; ++q) {
        uint64_t hb[W];
        uint64_t pre = ~0ull;
#pragma unroll
        for (int i = 0; i < W; ++i) {
          const int r = q * W + i;
          if (r < L) {
            uint64_t mu;
            if (i == 0) {
              mu = suf[0];
            } else {
              hb[i - 1] = mmer_hash<M, true>(a, r + W - 1);
              pre = umin64(pre, hb[i - 1]);
              mu = umin64(suf[i], pre);
            }
            s_shard[t * L + r] = (uint32_t)mu & shard_mask;
          }
        }
        if ((q + 1) * W < L) {
          hb[W - 1] = mmer_hash<M, true>(a, (q + 1) * W + W - 1);
          suf[W - 1] = hb[W - 1];
#pragma unroll
          for (int i = W - 2; i >= 0; --i) suf[i] = umin64(hb[i], suf[i + 1]);
        }
      }
#pragma unroll
      for (int j = 0; j < L; ++j) s_bits[t * L + j] = pack_bit_addresses<H>(smer_hash(smer_at<S>(a, j)));
      if (t == WG - 1) {
#pragma unroll
        for (int j = L; j < L + Z; ++j) s_bits[t * L + j] = pack_bit_addresses<H>(smer_hash(smer_at<S>(a, j)));
      }
    }
    __syncthreads();

    // ---- phase 2: one k-mer per lane, consecutive k-mers across the wave ----
    const int lane = threadIdx.x & 63;
#pragma unroll 2
    for (int i = 0; i < L; ++i) {
      const int q = i * WG + threadIdx.x;
      const bool v = (s_kv[q >> 4] >> (q & 15)) & 1u;
      const uint32_t shard = s_shard[q];
      uint32_t wd[8];
      if constexpr (SHARE) {
        const int qp = q > 0 ? q - 1 : 0;
        const bool pv = q > 0 && ((s_kv[qp >> 4] >> (qp & 15)) & 1u);
        const bool head = v && (lane == 0 || !pv || s_shard[qp] != shard);
        const uint64_t heads = __ballot(head);
        const uint64_t upto = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
        const int leader = upto ? 63 - __clzll((long long)upto) : lane;
        if (head) {
          const uint4 *p = reinterpret_cast<const uint4 *>(words + 4ull * (uint64_t)shard);
          const uint4 lo = p[0], hi = p[1];
          wd[0] = lo.x; wd[1] = lo.y; wd[2] = lo.z; wd[3] = lo.w;
          wd[4] = hi.x; wd[5] = hi.y; wd[6] = hi.z; wd[7] = hi.w;
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) wd[j] = 0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) wd[j] = (uint32_t)__builtin_amdgcn_ds_bpermute(leader << 2, (int)wd[j]);
      } else {
        if (v) {
          const uint4 *p = reinterpret_cast<const uint4 *>(words + 4ull * (uint64_t)shard);
          const uint4 lo = p[0], hi = p[1];
          wd[0] = lo.x; wd[1] = lo.y; wd[2] = lo.z; wd[3] = lo.w;
          wd[4] = hi.x; wd[5] = hi.y; wd[6] = hi.z; wd[7] = hi.w;
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) wd[j] = 0;
        }
      }
      uint64_t w4[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) w4[w] = ((uint64_t)wd[2 * w + 1] << 32) | wd[2 * w];
      uint32_t acc = 0xFFFFFFFFu;
#pragma unroll
      for (int p = 0; p <= Z; ++p) {
        const Pack b = s_bits[q + p];
#pragma unroll
        for (int t = 0; t < H; ++t) acc &= (uint32_t)(w4[t & 3] >> ((uint32_t)(b >> (8 * t)) & 63u));
      }
      const uint64_t pos = base + (uint64_t)q;
      if (pos < n_out) out[pos] = v ? (uint8_t)(acc & 1u) : (uint8_t)0;
    }
  }
}

// ---------------------------------------------------------------------------
// Query, lane-sequential: each lane walks L consecutive k-mers like the insert
// kernel.  For k-mer r it forms the OR A(r) of the one-hot masks of its z+1
// s-mers (the same pair trick), issues the two 16-byte loads of its shard, and
// D k-mers later tests (A(r) & ~shard) == 0, so the load latency overlaps the
// hashing of the next k-mers.  A lane loads its own shard only where the shard
// changes (about once per super-k-mer) and otherwise keeps the previous
// words.  Lanes walk L = 48 k-mers (three van Herk blocks of 16), which
// spreads the w-1 extra m-mer hashes, z extra s-mers and the shard load at a
// lane's start over more k-mers than L = 32.  Answers are kept as one bit per
// k-mer and spread to bytes for 16-byte stores at the end.
// ---------------------------------------------------------------------------
template <int K, int S, int M, int H, int L, int WG, int D, bool REPAIR = false>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4))) void query_lane_kernel(const uint8_t *__restrict__ seq, uint64_t len,
                                                        const uint32_t *__restrict__ starts, int aligned16,
                                                        typename std::conditional<REPAIR, uint64_t, const uint64_t>::type *words,
                                                        uint32_t shard_mask,
                                                        uint8_t *__restrict__ out, uint64_t n_out,
                                                        int out_aligned16, int out_packed, TileQueue tq) {
  constexpr int W = K - M + 1;
  constexpr int Z = K - S;
  constexpr int GPL = L / 16;
  constexpr int NGW = lane_granules<K, L>();
  constexpr int NGRAN = (WG - 1) * GPL + NGW;
  static_assert(D >= 1 && D < L, "test distance");
  static_assert(L % 16 == 0 && L <= 64, "a lane's answer bits are whole 16-bit words of one 64-bit value");

  __shared__ uint32_t s_codes[NGRAN];
  __shared__ uint32_t s_vb[NGRAN];
  // van Herk state of each lane in LDS (structure of arrays, lane-minor):
  // slot i holds the suffix minimum i of the current block until step i has
  // used it, then the hash of position i of the next block.  Keeping these 32
  // 64-bit values out of registers lets the kernel run four waves per SIMD
  // (at most 128 VGPRs; 38 KB of LDS per workgroup at L = 48, four
  // workgroups in the 160 KB of a CU).
  __shared__ uint64_t s_vh[W][WG];

  __shared__ uint32_t s_next_tile;
  acquire_device();
  uint64_t tile;
  for (bool first = true; next_tile(tq, &s_next_tile, first, tile); first = false) {
  const uint64_t base = (uint64_t)tile * (uint64_t)(WG * L);
    stage_granules<WG>(seq, len, base, starts, aligned16 != 0, NGRAN, s_codes, s_vb);
    __syncthreads();

    const int g0 = threadIdx.x * GPL;
    uint32_t a[NGW];
#pragma unroll
    for (int i = 0; i < NGW; ++i) a[i] = s_codes[g0 + i];
    const uint64_t kv = lane_kmer_valid<K, L>(s_vb, g0);
    // lost[i]: one bit per k-mer 32i .. 32i+31, set where some bit of the
    // k-mer is missing from its shard, shifted in from the right (k-mer 32i+j
    // ends at bit n-1-j of the word's n k-mers); reversed, inverted and
    // masked by validity at the end into ans.
    uint32_t lost[(L + 31) / 32];
#pragma unroll
    for (int i = 0; i < (L + 31) / 32; ++i) lost[i] = 0;

    if (kv != 0) {
      uint64_t oh[L + Z][4];
      uint64_t pr[L + Z][4];
      uint64_t need[L][4];     // A(r), kept D k-mers (z != 3)
      uint64_t ldw[L][4];      // words loaded for k-mer r (its shard, or shard 0)
      bool fresh_at[L];        // k-mer r loaded its own shard
      uint32_t sh_at[L];       // shard of k-mer r (repair)
      uint64_t got[4];         // shard words of the last tested k-mer
      uint32_t prev_sh = 0;
      // 32 bytes per shard, as an operand the compiler cannot fold: the
      // shard's address is then one 32x32+64 multiply-add instead of a 64-bit
      // shift and add
      uint32_t shard_bytes = 32;
      asm("" : "+s"(shard_bytes));
#pragma unroll
      for (int j = 0; j < Z; ++j) smer_onehots<H>(smer_hash(smer_at<S>(a, j)), oh[j]);
      if constexpr (Z == 3) {
#pragma unroll
        for (int j = 0; j + 1 < Z; ++j)
#pragma unroll
          for (int w = 0; w < 4; ++w) pr[j][w] = oh[j][w] | oh[j + 1][w];
      }
      const int t = threadIdx.x;
      {
        // suffix minima of block 0
        uint64_t m = mmer_hash<M, true>(a, W - 1);
        s_vh[W - 1][t] = m;
#pragma unroll
        for (int i = W - 2; i >= 0; --i) {
          m = umin64(mmer_hash<M, true>(a, i), m);
          s_vh[i][t] = m;
        }
      }
      auto test = [&](int r) {
        // Select the shard words here, D k-mers after the load was issued,
        // so that the wait for the load does not follow the load at once.
#pragma unroll
        for (int w = 0; w < 4; ++w) got[w] = (r == 0 || fresh_at[r]) ? ldw[r][w] : got[w];
        // Bits of A(r) missing from the shard.  With z = 3, A(r) is the OR of
        // two pair masks and each 32-bit half of the missing bits is one
        // three-input operation (a | b) & ~c (truth table 0x54 over the
        // operand tables 0xF0, 0xCC, 0xAA).
        uint32_t m[8];
#pragma unroll
        for (int w = 0; w < 4; ++w) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const uint32_t g = (uint32_t)(got[w] >> (32 * h));
            if constexpr (Z == 3)
              m[2 * w + h] = __builtin_amdgcn_bitop3_b32((uint32_t)(pr[r][w] >> (32 * h)),
                                                         (uint32_t)(pr[r + 2][w] >> (32 * h)), g, 0x54);
            else
              m[2 * w + h] = (uint32_t)(need[r][w] >> (32 * h)) & ~g;
          }
        }
        const uint32_t miss = (m[0] | m[1] | m[2]) | (m[3] | m[4] | m[5]) | (m[6] | m[7]);
        if constexpr (REPAIR) {
          // Insert repair: OR the missing bits of a valid k-mer into its
          // shard and into the cached words, so that later k-mers of the run
          // do not repeat them.
          if (miss != 0 && ((kv >> r) & 1ull)) {
            uint64_t *p = words + 4ull * (uint64_t)sh_at[r];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
              const uint64_t mw = ((uint64_t)m[2 * w + 1] << 32) | m[2 * w];
              if (mw) atomic_or64(p + w, mw);
              got[w] |= mw;
            }
          }
        } else {
          // lost = 2 lost + (miss != 0): a compare and an add with carry (the
          // compiler's form, a select of the bit and an OR, takes a third
          // instruction and often a fourth to move the bit's constant)
          asm("v_cmp_ne_u32_e32 vcc, 0, %1\n\tv_addc_co_u32_e32 %0, vcc, %0, %0, vcc"
              : "+v"(lost[r >> 5])
              : "v"(miss)
              : "vcc");
        }
      };
#pragma unroll
      for (int q = 0; q * W < L; ++q) {
        uint64_t pre = ~0ull;
#pragma unroll
        for (int i = 0; i < W; ++i) {
          const int r = q * W + i;
          if (r < L) {
            uint64_t mu;
            if (i == 0) {
              mu = s_vh[0][t];
            } else {
              const uint64_t h = mmer_hash<M, true>(a, r + W - 1);  // position i-1 of block q+1
              pre = umin64(pre, h);
              mu = umin64(s_vh[i][t], pre);
              s_vh[i - 1][t] = h;  // slot i-1 was last read at step i-1
            }
            // A lane loads its shard only where the shard changes (about once
            // per super-k-mer); elsewhere it reads shard 0, one line shared by
            // every such lane, and keeps the previous k-mer's words.  Straight-
            // line code keeps the register footprint of the plain load.
            const uint32_t sh = (uint32_t)mu & shard_mask;
            const bool fresh = r == 0 || sh != prev_sh;
            prev_sh = sh;
            // the select on the 32-bit index (the asm operand keeps the
            // compiler from moving it past the widening to a byte offset,
            // where it takes a 64-bit shift and two selects)
            uint32_t lsh = fresh ? sh : 0u;
            asm("" : "+v"(lsh));
            const uint4 *p = reinterpret_cast<const uint4 *>(reinterpret_cast<const uint8_t *>(words) +
                                                             (uint64_t)lsh * (uint64_t)shard_bytes);
            const uint4 lo = p[0], hi = p[1];
            ldw[r][0] = ((uint64_t)lo.y << 32) | lo.x;
            ldw[r][1] = ((uint64_t)lo.w << 32) | lo.z;
            ldw[r][2] = ((uint64_t)hi.y << 32) | hi.x;
            ldw[r][3] = ((uint64_t)hi.w << 32) | hi.z;
            fresh_at[r] = fresh;
            sh_at[r] = sh;
            smer_onehots<H>(smer_hash(smer_at<S>(a, r + Z)), oh[r + Z]);
            if constexpr (Z == 3) {
#pragma unroll
              for (int w = 0; w < 4; ++w) {
                pr[r + 2][w] = oh[r + 2][w] | oh[r + 3][w];
              }
            } else {
#pragma unroll
              for (int w = 0; w < 4; ++w) {
                uint64_t x = oh[r][w];
#pragma unroll
                for (int j = 1; j <= Z; ++j) x |= oh[r + j][w];
                need[r][w] = x;
              }
            }
            if (r >= D) test(r - D);
          }
        }
        if ((q + 1) * W < L) {
          // suffix minima of block q+1, in place over its hashes
          uint64_t m = mmer_hash<M, true>(a, (q + 1) * W + W - 1);
          s_vh[W - 1][t] = m;
#pragma unroll
          for (int i = W - 2; i >= 0; --i) {
            m = umin64(s_vh[i][t], m);
            s_vh[i][t] = m;
          }
        }
      }
#pragma unroll
      for (int r = L - D; r < L; ++r) test(r);
    }
    if constexpr (REPAIR) continue;  // no answers
    uint32_t ans[(L + 31) / 32];
#pragma unroll
    for (int i = 0; i < (L + 31) / 32; ++i) {
      constexpr int kFull = 32;
      const int n = L - kFull * i < kFull ? L - kFull * i : kFull;
      ans[i] = ~(__builtin_bitreverse32(lost[i]) >> (kFull - n)) & (uint32_t)(kv >> (kFull * i));
    }
    if (out_packed) {
      // One answer bit per k-mer: the lane's L bits start at bit base +
      // lane_off, a multiple of 16, so they are L/16 aligned 16-bit words;
      // bits at or past n_out are cleared and bytes past them not written.
      const uint64_t pos0 = base + (uint64_t)threadIdx.x * L;
      if (pos0 < n_out) {
        uint64_t bits = ans[0];
        if constexpr (L > 32) bits |= (uint64_t)ans[(L + 31) / 32 - 1] << 32;
        const uint64_t left = n_out - pos0;
        if (left < (uint64_t)L) bits &= (1ull << left) - 1;
        uint8_t *ob = out + pos0 / 8;
        if (left >= (uint64_t)L) {
#pragma unroll
          for (int c = 0; c < L / 16; ++c) reinterpret_cast<uint16_t *>(ob)[c] = (uint16_t)(bits >> (16 * c));
        } else {
          for (uint64_t j = 0; j < (left + 7) / 8; ++j) ob[j] = (uint8_t)(bits >> (8 * j));
        }
      }
      continue;
    }
    // One answer byte per k-mer: four bits x of ans spread to bytes by
    // x * 0x204081 (x, x<<7, x<<14, x<<21 do not overlap), 16 k-mers per
    // 16-byte store from a workgroup-uniform base plus a 32-bit lane offset;
    // byte stores for a lane that ends past n_out or an unaligned output.
    auto bytes4 = [&](int r) { return (((ans[r >> 5] >> (r & 31)) & 0xFu) * 0x204081u) & 0x01010101u; };
    uint8_t *const out_tile = out + base;
    const uint32_t lane_off = (uint32_t)threadIdx.x * (uint32_t)L;
    if (out_aligned16 && base + lane_off + L <= n_out) {
#pragma unroll
      for (int c = 0; c < L / 16; ++c)
        *reinterpret_cast<uint4 *>(out_tile + lane_off + 16 * c) =
            make_uint4(bytes4(16 * c), bytes4(16 * c + 4), bytes4(16 * c + 8), bytes4(16 * c + 12));
    } else {
      const uint64_t pos0 = base + lane_off;
#pragma unroll
      for (int r = 0; r < L; ++r)
        if (pos0 + r < n_out) out[pos0 + r] = (uint8_t)((ans[r >> 5] >> (r & 31)) & 1u);
    }
  }
}

constexpr int kInsertL = 32;
constexpr int kInsertWG = 256;
constexpr int kQueryWG = 256;
constexpr int kQueryLaneL = 48;
constexpr int kQueryLaneWG = 256;
constexpr int kQueryLaneD = 1;

// Compiled lane lengths: the insert's store pass walks 32 k-mers per lane,
// and for the paper's default parameter set also 64, its default there for
// inserts of at least kLongInsertKmers k-mers (1.7% faster out of cache, the
// walk held in registers; a smaller insert has too few 16384-k-mer tiles for
// the 1024 resident workgroups and keeps 32); the query and the insert's
// repair walk 48 (default) or 32.  The second lengths exist for the paper's
// default parameter set only.
template <int K, int S, int M, int H>
constexpr bool lane_len_variants() { return K == 31 && S == 28 && M == 16 && H == 4; }
constexpr uint64_t kLongInsertKmers = 1ull << 24;

template <int K, int S, int M, int H, int QL>
hipError_t query_lane_launch(const uint64_t *words, uint32_t shard_mask, const SeqArgs &a, const LaunchShape &ls,
                             hipStream_t st, int aligned) {
  const uint64_t tile = (uint64_t)QL * kQueryLaneWG;
  SBF_LAUNCH_TILES((query_lane_kernel<K, S, M, H, QL, kQueryLaneWG, kQueryLaneD>), kQueryLaneWG,
                   (a.n_out + tile - 1) / tile, 2, a.seq, a.len, a.starts, aligned, words, shard_mask, a.out,
                   a.n_out, (int)(((uintptr_t)a.out & 15u) == 0), a.packed);
  return hipSuccess;
}

template <int K, int S, int M, int H, int QL>
hipError_t repair_launch(uint64_t *words, uint32_t shard_mask, const SeqArgs &a, uint64_t nk, const LaunchShape &ls,
                         hipStream_t st, int aligned) {
  const uint64_t qtile = (uint64_t)QL * kQueryLaneWG;
  SBF_LAUNCH_TILES((query_lane_kernel<K, S, M, H, QL, kQueryLaneWG, kQueryLaneD, true>), kQueryLaneWG,
                   (nk + qtile - 1) / qtile, 1, a.seq, a.len, a.starts, aligned, words, shard_mask,
                   (uint8_t *)nullptr, nk, 0, 0);
  return hipSuccess;
}

template <int K, int S, int M, int H, int IL>
hipError_t store_launch(uint64_t *words, uint32_t shard_mask, const SeqArgs &a, uint64_t nk, int mode,
                        const LaunchShape &ls, hipStream_t st, int aligned) {
  const uint64_t tile = (uint64_t)IL * kInsertWG;
  const uint64_t ntiles = (nk + tile - 1) / tile;
  if (mode == kInsertAtomicMode)
    SBF_LAUNCH_TILES((insert_rolling_kernel<K, S, M, H, IL, kInsertWG, kAtomic>), kInsertWG, ntiles, 0, a.seq,
                     a.len, a.starts, aligned, words, shard_mask);
  else
    SBF_LAUNCH_TILES((insert_rolling_kernel<K, S, M, H, IL, kInsertWG, kStore>), kInsertWG, ntiles, 0, a.seq, a.len,
                     a.starts, aligned, words, shard_mask);
  return hipSuccess;
}

template <int K, int S, int M, int H>
hipError_t insert_rolling(uint64_t *words, uint32_t shard_mask, const SeqArgs &a, int mode, const LaunchShape &ls,
                          hipStream_t st) {
  if (a.len < (uint64_t)K) return hipSuccess;
  const uint64_t nk = a.len - K + 1;
  const int aligned = ((uintptr_t)a.seq & 15u) == 0;
  hipError_t e;
  if constexpr (lane_len_variants<K, S, M, H>()) {
    if (ls.insert_lane_len == 64 || (ls.insert_lane_len == 0 && nk >= kLongInsertKmers))
      e = store_launch<K, S, M, H, 64>(words, shard_mask, a, nk, mode, ls, st, aligned);
    else
      e = store_launch<K, S, M, H, kInsertL>(words, shard_mask, a, nk, mode, ls, st, aligned);
  } else {
    e = store_launch<K, S, M, H, kInsertL>(words, shard_mask, a, nk, mode, ls, st, aligned);
  }
  if (e != hipSuccess || mode == kInsertAtomicMode) return e;
  // Repair pass: the lane query walk, OR-ing the bits the store pass lost.
  if constexpr (lane_len_variants<K, S, M, H>()) {
    if (ls.query_lane_len == 32) return repair_launch<K, S, M, H, 32>(words, shard_mask, a, nk, ls, st, aligned);
  }
  return repair_launch<K, S, M, H, kQueryLaneL>(words, shard_mask, a, nk, ls, st, aligned);
}

template <int K, int S, int M, int H>
hipError_t query_rolling(const uint64_t *words, uint32_t shard_mask, const SeqArgs &a, int mode,
                         const LaunchShape &ls, hipStream_t st) {
  if (a.n_out == 0) return hipSuccess;
  const int aligned = ((uintptr_t)a.seq & 15u) == 0;
  if (mode == kQueryLaneMode) {
    if constexpr (lane_len_variants<K, S, M, H>()) {
      if (ls.query_lane_len == 32) return query_lane_launch<K, S, M, H, 32>(words, shard_mask, a, ls, st, aligned);
    }
    return query_lane_launch<K, S, M, H, kQueryLaneL>(words, shard_mask, a, ls, st, aligned);
  }
  if (a.packed) return hipErrorInvalidValue;  // bits only from the lane organisation
  const uint64_t tile = 16ull * kQueryWG;
  if (mode == kQueryLeaderMode)
    SBF_LAUNCH_TILES((query_rolling_kernel<K, S, M, H, kQueryWG, true>), kQueryWG, (a.n_out + tile - 1) / tile, 2,
                     a.seq, a.len, a.starts, aligned, words, shard_mask, a.out, a.n_out);
  else
    SBF_LAUNCH_TILES((query_rolling_kernel<K, S, M, H, kQueryWG, false>), kQueryWG, (a.n_out + tile - 1) / tile, 2,
                     a.seq, a.len, a.starts, aligned, words, shard_mask, a.out, a.n_out);
  return hipSuccess;
}

}  // namespace

// Parameter sets (k, s, m, H) with compiled rolling kernels: the paper's
// default and the neighbours its parameter study reports (Section
// "Parameter Selection"); every other set runs the generic kernels.
#define SBF_ROLLING_SETS(X) \
  X(31, 28, 16, 4)          \
  X(31, 27, 16, 4)          \
  X(31, 30, 16, 4)          \
  X(31, 31, 16, 4)          \
  X(31, 28, 18, 4)          \
  X(31, 28, 16, 8)

bool rolling_supported(const Geometry &g) {
  if (g.shard_words != 4 || g.nshards > (1ull << 32)) return false;
#define SBF_MATCH(K_, S_, M_, H_) \
  if (g.k == K_ && g.s == S_ && g.m == M_ && g.H == H_) return true;
  SBF_ROLLING_SETS(SBF_MATCH)
#undef SBF_MATCH
  return false;
}

hipError_t launch_insert_rolling(const Geometry &g, uint64_t *words, const SeqArgs &a, int mode,
                                 const LaunchShape &ls, hipStream_t st) {
  const uint32_t mask = (uint32_t)(g.nshards - 1);
#define SBF_CALL(K_, S_, M_, H_)                            \
  if (g.k == K_ && g.s == S_ && g.m == M_ && g.H == H_) \
    return insert_rolling<K_, S_, M_, H_>(words, mask, a, mode, ls, st);
  SBF_ROLLING_SETS(SBF_CALL)
#undef SBF_CALL
  return hipErrorInvalidValue;
}

hipError_t launch_query_rolling(const Geometry &g, const uint64_t *words, const SeqArgs &a, int mode,
                                const LaunchShape &ls, hipStream_t st) {
  const uint32_t mask = (uint32_t)(g.nshards - 1);
#define SBF_CALL(K_, S_, M_, H_)                            \
  if (g.k == K_ && g.s == S_ && g.m == M_ && g.H == H_) \
    return query_rolling<K_, S_, M_, H_>(words, mask, a, mode, ls, st);
  SBF_ROLLING_SETS(SBF_CALL)
#undef SBF_CALL
  return hipErrorInvalidValue;
}

}  // namespace sbf
