// Wide-shard super-k-mer kernels for gfx950: insert and query of filters whose
// shards are SW = 4, 8 or 16 64-bit words (32, 64 or 128 bytes).  The paper
// sizes a shard to the load width of its GPU (Section "Data Layout"); on this
// GPU a 16-word shard is exactly one 128-byte cache line, the unit every
// random access moves anyway.  Hash index t of an s-mer sets a bit of sector
// t mod 4 in the word group picked by the hash bits just above its 6-bit
// address, so a super-k-mer's bits spread over all SW words.
//
// A segment's mask of SW words does not fit the registers the 4-word kernels
// keep it in, so these kernels work in two phases per tile of WG x LP k-mers:
//   phase 1 (as in the two-phase query): lane t stages LP consecutive
//     k-mers, hashes every m-mer and s-mer position once (van Herk sliding
//     minimum over the m-mer hashes) and writes each k-mer's shard and each
//     s-mer's packed bit addresses to LDS;
//   phase 2: each wave walks its own contiguous quarter of the tile, 64
//     consecutive k-mers per step, one per lane.  Runs of valid k-mers with
//     equal shard (super-k-mers, Section "Minimizers and Super-k-mers") are
//     found with a ballot, and each run's shard is moved by SW/2 lanes
//     together, one 16-byte piece of the line each, so a wave instruction
//     covers whole lines (the paper's leader load and shard sharing,
//     Algorithms 1 and 2, with the line split across lanes instead of
//     broadcast from one).
// Insert: the lanes of a run's line OR the run's s-mer bits into an LDS copy
//   of the line, then each ORs its two words into its piece and writes it
//   back if it changed (a read-modify-write whose store writes through to the
//   device's coherence point; a second launch of the same kernel reads each
//   run's line again and atomically ORs in any bit a concurrent write
//   dropped) or, in atomic mode, issues 64-bit atomic ORs.  A run that
//   continues into the wave's next step is written once.
// Query: the lanes of a run stage its line in LDS; each k-mer lane then tests
//   its (k-s+1)*H bits there (Algorithm 2, Contains).
// Results are bit-identical to the per-k-mer definition: OR is commutative
// and idempotent, and every k-mer is tested in its own shard.
#include "sbf_tiles.h"

#include <type_traits>

namespace sbf {
namespace {

// log2(SW / 4): group bits above each 6-bit address
template <int SW>
constexpr int group_bits() { return SW == 16 ? 2 : SW == 8 ? 1 : 0; }

template <int H>
using wide_pack_t = typename std::conditional<(H <= 4), uint32_t, uint64_t>::type;

// Byte t of the result: (group << 6) | bit for hash index t of s-mer hash g,
// i.e. the low 6 + log2(SW/4) bits of slice t.  The bit lands in word
// (t mod 4) + 4 * group of the shard.
template <int H, int SW>
__device__ __forceinline__ wide_pack_t<H> wide_addresses(uint64_t g) {
  constexpr int W = 64 / H;
  constexpr int GB = group_bits<SW>();
  static_assert(H % 4 == 0 && H <= 8, "one or two sets of four sectors, eight address bytes");
  static_assert(W >= 6 + GB, "the group bits lie inside each hash index's slice");
  wide_pack_t<H> p = 0;
#pragma unroll
  for (int t = 0; t < H; ++t)
    p |= (wide_pack_t<H>)((uint32_t)(g >> (t * W)) & ((64u << GB) - 1u)) << (8 * t);
  return p;
}

// LDS of one tile: the staged sequence, then per k-mer its shard and
// validity and per s-mer its packed addresses.  The staged sequence is only
// read in phase 1, so phase 2 may reuse its bytes and SCR more (scratch).
template <int K, int S, int H, int LP, int WG, int SCR = 1>
struct WideTile {
  static constexpr int Z = K - S;
  static constexpr int TILE = WG * LP;
  static constexpr int GPL = LP / 16;
  static constexpr int NGW = lane_granules<K, LP>();
  static constexpr int NGRAN = (WG - 1) * GPL + NGW;
  static constexpr int KVW = (LP + 31) / 32;  // validity words per lane
  union {
    struct {
      uint32_t codes[NGRAN];
      uint32_t vb[NGRAN];
    };
    uint2 scratch[SCR];
  };
  uint32_t shard[TILE];
  wide_pack_t<H> bits[TILE + Z];
  uint32_t kv[WG * KVW];

  // k-mer q of the tile is valid
  __device__ __forceinline__ bool valid(int q) const {
    return (kv[(q / LP) * KVW + ((q % LP) >> 5)] >> ((q % LP) & 31)) & 1u;
  }
};

// Phase 1: stage the tile starting at k-mer `base` and fill shard, kv and
// bits (lane t: k-mers and s-mers t*LP .. t*LP+LP-1, the last lane also the
// z s-mers after the tile).
template <int K, int S, int M, int H, int SW, int LP, int WG, int SCR>
__device__ __forceinline__ void wide_phase1(WideTile<K, S, H, LP, WG, SCR> &T, const uint8_t *__restrict__ seq,
                                            uint64_t len, uint64_t base, const uint32_t *__restrict__ starts,
                                            bool aligned16, uint32_t shard_mask) {
  using Tl = WideTile<K, S, H, LP, WG, SCR>;
  constexpr int W = K - M + 1;
  constexpr int Z = K - S;
  stage_granules<WG>(seq, len, base, starts, aligned16, Tl::NGRAN, T.codes, T.vb);
  __syncthreads();
  const int t = threadIdx.x;
  const int g0 = t * Tl::GPL;
  uint32_t a[Tl::NGW];
#pragma unroll
  for (int i = 0; i < Tl::NGW; ++i) a[i] = T.codes[g0 + i];
  const uint64_t kv = lane_kmer_valid<K, LP>(T.vb, g0);
#pragma unroll
  for (int j = 0; j < Tl::KVW; ++j) T.kv[t * Tl::KVW + j] = (uint32_t)(kv >> (32 * j));

  // van Herk sliding minimum: suf[i] = min(h[qW+i .. qW+W-1]) of block q
  uint64_t suf[W];
  {
    uint64_t hb[W];
#pragma unroll
    for (int i = 0; i < W; ++i) hb[i] = mmer_hash<M>(a, i);
    suf[W - 1] = hb[W - 1];
#pragma unroll
    for (int i = W - 2; i >= 0; --i) suf[i] = umin64(hb[i], suf[i + 1]);
  }
#pragma unroll
  for (int q = 0; q * W < LP; ++q) {
    uint64_t hb[W];
    uint64_t pre = ~0ull;
#pragma unroll
    for (int i = 0; i < W; ++i) {
      const int r = q * W + i;
      if (r < LP) {
        uint64_t mu;
        if (i == 0) {
          mu = suf[0];
        } else {
          hb[i - 1] = mmer_hash<M>(a, r + W - 1);
          pre = umin64(pre, hb[i - 1]);
          mu = umin64(suf[i], pre);
        }
        T.shard[t * LP + r] = (uint32_t)mu & shard_mask;
      }
    }
    if ((q + 1) * W < LP) {
      hb[W - 1] = mmer_hash<M>(a, (q + 1) * W + W - 1);
      suf[W - 1] = hb[W - 1];
#pragma unroll
      for (int i = W - 2; i >= 0; --i) suf[i] = umin64(hb[i], suf[i + 1]);
    }
  }
#pragma unroll
  for (int j = 0; j < LP; ++j) T.bits[t * LP + j] = wide_addresses<H, SW>(smer_hash(smer_at<S>(a, j)));
  if (t == WG - 1) {
#pragma unroll
    for (int j = LP; j < LP + Z; ++j) T.bits[t * LP + j] = wide_addresses<H, SW>(smer_hash(smer_at<S>(a, j)));
  }
  __syncthreads();
}

// How a run's bits reach its shard: 64-bit atomic ORs; a read-modify-write
// with a coherent store (the store pass of the two-pass insert); or, after
// the store pass, a read and an atomic OR of only the bits still missing (the
// repair walk, one check per run instead of per k-mer).
enum WideInsertMode : int { kWideAtomic = 0, kWideStore = 1, kWideRepair = 2 };

// ---------------------------------------------------------------------------
// Insert.  Lane (run j, piece p) of a round owns words 2p and 2p+1 of run j's
// shard.  The run's SW/2 lanes split its s-mers between them (every SW/2-th
// one each) and OR each s-mer's H bits into the run's line buffer in LDS with
// LDS atomics; each lane then takes its two words from the buffer and applies
// them to its piece of the shard.
// ---------------------------------------------------------------------------
template <int K, int S, int M, int H, int SW, int LP, int WG, int MODE>
__global__ __launch_bounds__(WG) void insert_wide_kernel(const uint8_t *__restrict__ seq, uint64_t len,
                                                         const uint32_t *__restrict__ starts, int aligned16,
                                                         uint64_t *__restrict__ words, uint32_t shard_mask,
                                                         TileQueue tq) {
  constexpr int Z = K - S;
  constexpr int NWAVES = WG / 64;
  // line buffers of a round's runs (two words per lane, 1 KB per wave), over
  // the tile's staged sequence, which phase 2 no longer reads
  using Tl = WideTile<K, S, H, LP, WG, NWAVES * 128>;
  constexpr int PER_WAVE = Tl::TILE / NWAVES;  // 64 * LP k-mers
  constexpr int LPR = SW / 2;                  // lanes per run
  constexpr int RPR = 64 / LPR;                // runs per round
  static_assert(WG % 64 == 0 && PER_WAVE == 64 * LP, "whole waves, one k-mer per lane per step");
  static_assert(Tl::TILE <= 65536, "tile positions fit 16 bits");

  __shared__ Tl T;
  __shared__ uint32_t s_run_shard[NWAVES][64];
  __shared__ uint32_t s_run_span[NWAVES][64];  // first k-mer | last k-mer << 16 (tile positions)
  __shared__ uint32_t s_next_tile;

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int q0 = wave * PER_WAVE;
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  // this lane's piece of a run's line: words 2p, 2p+1
  const int p = lane % LPR;
  const int slot = lane / LPR;
  // word w of run slot s of this wave's round at s_mask[s * SW + w]; this
  // lane's piece is s_mask[2 lane], s_mask[2 lane + 1]
  uint64_t *const s_mask = reinterpret_cast<uint64_t *>(T.scratch) + wave * 128;

  acquire_device();
  uint64_t tile;
  for (bool first = true; next_tile(tq, &s_next_tile, first, tile); first = false) {
    const uint64_t base = tile * (uint64_t)Tl::TILE;
    wide_phase1<K, S, M, H, SW, LP, WG>(T, seq, len, base, starts, aligned16 != 0, shard_mask);

    int carry = 0;  // first k-mer of the run open at the end of the previous step
    for (int step = 0; step < LP; ++step) {
      const int s0 = q0 + step * 64;
      const int q = s0 + lane;
      const bool v = T.valid(q);
      const uint32_t sh = T.shard[q];
      const bool prev_same = q > q0 && T.valid(q - 1) && T.shard[q - 1] == sh;
      const bool next_same = q + 1 < q0 + PER_WAVE && T.valid(q + 1) && T.shard[q + 1] == sh;
      const bool head = v && !prev_same;
      const bool tail = v && !next_same;
      const uint64_t heads = __ballot(head);
      const uint64_t tails = __ballot(tail);
      if (tail) {
        // the run ending here starts at the nearest head at or below this
        // lane, or in an earlier step
        const uint64_t hb = heads & upto;
        const int a = hb ? s0 + 63 - __clzll((long long)hb) : carry;
        const int j = __popcll(tails & upto) - 1;
        s_run_shard[wave][j] = sh;
        s_run_span[wave][j] = (uint32_t)a | ((uint32_t)q << 16);
      }
      // a run still open after lane 63 continues into the next step
      if (heads) carry = s0 + 63 - __clzll((long long)heads);
      const int nruns = __popcll(tails);
      for (int r0 = 0; r0 < nruns; r0 += RPR) {
        const int j = r0 + slot;
        // The buffer words pass between the lanes of the wave, so every
        // access is atomic, and a wavefront-scope fence orders the other
        // lanes' ORs before this lane's reads (a plain read after a plain
        // clear could be taken as still zero for a lane that ORed nothing).
        __hip_atomic_store(&s_mask[2 * lane], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        __hip_atomic_store(&s_mask[2 * lane + 1], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        uint64_t *line = nullptr;
        uint64_t o0 = 0, o1 = 0;
        if (j < nruns) {
          const uint32_t rsh = s_run_shard[wave][j];
          const uint32_t span = s_run_span[wave][j];
          const int a = (int)(span & 0xFFFFu);
          const int b = (int)(span >> 16);
          line = words + (uint64_t)rsh * SW + 2 * p;
          if constexpr (MODE != kWideAtomic) {
            const uint4 piece = *reinterpret_cast<const uint4 *>(line);
            o0 = ((uint64_t)piece.y << 32) | piece.x;
            o1 = ((uint64_t)piece.w << 32) | piece.z;
          }
          uint64_t *run_words = s_mask + slot * SW;
          for (int x = a + p; x <= b + Z; x += LPR) {
            const wide_pack_t<H> pk = T.bits[x];
#pragma unroll
            for (int h = 0; h < (H + 3) / 4; ++h) {
              // byte u of o4: the offset in the run's line of word
              // (u mod 4) + 4 * group of address u (8 bytes per word, 32 per
              // group), one shift, mask and add for four addresses (the asm
              // operand keeps the compiler from splitting them again)
              constexpr uint32_t kWords = 8u << 8 | 16u << 16 | 24u << 24;
              const uint32_t p4 = (uint32_t)(pk >> (32 * h));
              uint32_t o4 = ((p4 >> 1) & 0x60606060u) + kWords;
              asm("" : "+v"(o4));
#pragma unroll
              for (int u = 0; u < 4 && 4 * h + u < H; ++u) {
                uint64_t *wp = reinterpret_cast<uint64_t *>(reinterpret_cast<uint8_t *>(run_words) +
                                                            ((o4 >> (8 * u)) & 0xFFu));
                __hip_atomic_fetch_or(wp, 1ull << ((p4 >> (8 * u)) & 63u), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WAVEFRONT);
              }
            }
          }
        }
        // (a wave's LDS operations take effect in order) the piece now holds
        // the bits of every s-mer of the run
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (j < nruns) {
          const uint64_t m[2] = {
              __hip_atomic_load(&s_mask[2 * lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT),
              __hip_atomic_load(&s_mask[2 * lane + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT)};
          if constexpr (MODE == kWideStore) {
            // coherent store of the piece (see store_pair_coherent)
            if ((o0 | m[0]) != o0 || (o1 | m[1]) != o1) store_pair_coherent(line, o0 | m[0], o1 | m[1]);
          } else if constexpr (MODE == kWideRepair) {
            // the bits a racing store dropped
            if (m[0] & ~o0) atomic_or64(line, m[0] & ~o0);
            if (m[1] & ~o1) atomic_or64(line + 1, m[1] & ~o1);
          } else {
            if (m[0]) atomic_or64(line, m[0]);
            if (m[1]) atomic_or64(line + 1, m[1]);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Query.  Runs restart at every step; the
// lines of up to PASS runs of the step are staged in LDS at once.  A line is
// stored sector-major: dword (t mod 4) * SW/2 + 2 * group + half holds half
// `half` of word (t mod 4) + 4 * group, so the dword of an address byte b of
// hash index t is (t mod 4) * SW/2 + (b >> 5) and its bit is b & 31.
// ---------------------------------------------------------------------------
template <int K, int S, int M, int H, int SW, int LP, int WG>
__global__ __launch_bounds__(WG) void query_wide_kernel(const uint8_t *__restrict__ seq, uint64_t len,
                                                        const uint32_t *__restrict__ starts, int aligned16,
                                                        const uint64_t *__restrict__ words,
                                                        uint32_t shard_mask, uint8_t *__restrict__ out,
                                                        uint64_t n_out, TileQueue tq) {
  constexpr int Z = K - S;
  constexpr int NWAVES = WG / 64;
  constexpr int LPR = SW / 2;
  constexpr int RPR = 64 / LPR;
  // run lines staged at once per wave: 8 for 16-word shards, so that the
  // tile (38.9 KB with 256 lanes x 16 k-mers) leaves LDS for four
  // workgroups per CU (with 16 lines, three fit; the query and repair walk
  // ran 19% slower)
  constexpr int PASS = SW == 16 ? 8 : 16;
  constexpr int HALF = SW / 2;
  // one staged line per run (SW words as dword pairs), over the staged
  // sequence, which phase 1 no longer needs
  using Tl = WideTile<K, S, H, LP, WG, NWAVES * PASS * SW>;
  constexpr int PER_WAVE = Tl::TILE / NWAVES;

  __shared__ Tl T;
  __shared__ uint32_t s_run_shard[NWAVES][64];
  __shared__ uint32_t s_next_tile;
  uint2 (*s_line)[PASS][SW] = reinterpret_cast<uint2 (*)[PASS][SW]>(T.scratch);

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int q0 = wave * PER_WAVE;
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int p = lane % LPR;
  // where this lane's piece (words 2p, 2p+1) goes in a staged line
  const int e = (2 * p) & 3;
  const int grp = p >> 1;
  const int d0 = (e * HALF + 2 * grp) / 2;  // dword pair index of word 2p
  const int d1 = ((e + 1) * HALF + 2 * grp) / 2;

  acquire_device();
  uint64_t tile;
  for (bool first = true; next_tile(tq, &s_next_tile, first, tile); first = false) {
    const uint64_t base = tile * (uint64_t)Tl::TILE;
    wide_phase1<K, S, M, H, SW, LP, WG>(T, seq, len, base, starts, aligned16 != 0, shard_mask);

    for (int step = 0; step < LP; ++step) {
      const int q = q0 + step * 64 + lane;
      const bool v = T.valid(q);
      const uint32_t sh = T.shard[q];
      const bool prev_same = lane > 0 && T.valid(q - 1) && T.shard[q - 1] == sh;
      const bool head = v && !prev_same;
      const uint64_t heads = __ballot(head);
      const int ri = __popcll(heads & upto) - 1;  // run of this lane (valid lanes)
      if (head) s_run_shard[wave][ri] = sh;
      const int nruns = __popcll(heads);
      uint32_t ok = 0;
      for (int r0 = 0; r0 < nruns; r0 += PASS) {
#pragma unroll
        for (int c = 0; c < PASS; c += RPR) {
          const int slot = c + lane / LPR;
          const int j = r0 + slot;
          if (slot < PASS && j < nruns) {
            const uint32_t rsh = s_run_shard[wave][j];
            const uint64_t *src = words + (uint64_t)rsh * SW + 2 * p;
            const uint4 piece = *reinterpret_cast<const uint4 *>(src);
            const uint64_t w0 = ((uint64_t)piece.y << 32) | piece.x;
            const uint64_t w1 = ((uint64_t)piece.w << 32) | piece.z;
            s_line[wave][slot][d0] = make_uint2((uint32_t)w0, (uint32_t)(w0 >> 32));
            s_line[wave][slot][d1] = make_uint2((uint32_t)w1, (uint32_t)(w1 >> 32));
          }
        }
        if (v && ri >= r0 && ri < r0 + PASS) {
          const uint8_t *Lb = reinterpret_cast<const uint8_t *>(s_line[wave][ri - r0]);
          uint32_t acc = 1;
#pragma unroll
          for (int o = 0; o <= Z; ++o) {
            const wide_pack_t<H> pk = T.bits[q + o];
#pragma unroll
            for (int h = 0; h < (H + 3) / 4; ++h) {
              // four addresses at once: byte u of o4 is the offset in the
              // staged line of the dword holding address u (its sector's
              // u * HALF dwords plus (address >> 5)), one shift, mask and
              // add for the four; each read is then the line base plus one
              // byte of o4 (the asm operand keeps the compiler from splitting
              // the shared computation back into four)
              constexpr uint32_t kSectors = (4u * HALF) << 8 | (8u * HALF) << 16 | (12u * HALF) << 24;
              const uint32_t p4 = (uint32_t)(pk >> (32 * h));
              uint32_t o4 = ((p4 >> 3) & 0x1C1C1C1Cu) + kSectors;
              asm("" : "+v"(o4));
#pragma unroll
              for (int u = 0; u < 4 && 4 * h + u < H; ++u) {
                const uint32_t d = *reinterpret_cast<const uint32_t *>(Lb + ((o4 >> (8 * u)) & 0xFFu));
                acc &= (d >> ((p4 >> (8 * u)) & 31u)) & 1u;
              }
            }
          }
          ok = acc;
        }
      }
      const uint64_t pos = base + (uint64_t)q;
      if (pos < n_out) out[pos] = (uint8_t)(v ? ok : 0u);
    }
  }
}

constexpr int kWideWG = 256;

template <int K, int S, int M, int H, int SW, int LP>
hipError_t insert_wide(uint64_t *words, uint32_t shard_mask, const SeqArgs &a, int mode, const LaunchShape &ls,
                       hipStream_t st) {
  if (a.len < (uint64_t)K) return hipSuccess;
  const uint64_t nk = a.len - K + 1;
  const uint64_t tile = (uint64_t)LP * kWideWG;
  const uint64_t ntiles = (nk + tile - 1) / tile;
  const int aligned = ((uintptr_t)a.seq & 15u) == 0;
  if (mode == kInsertAtomicMode) {
    SBF_LAUNCH_TILES((insert_wide_kernel<K, S, M, H, SW, LP, kWideWG, kWideAtomic>), kWideWG, ntiles, 0, a.seq,
                     a.len, a.starts, aligned, words, shard_mask);
    return hipSuccess;
  }
  SBF_LAUNCH_TILES((insert_wide_kernel<K, S, M, H, SW, LP, kWideWG, kWideStore>), kWideWG, ntiles, 0, a.seq, a.len,
                   a.starts, aligned, words, shard_mask);
  SBF_LAUNCH_TILES((insert_wide_kernel<K, S, M, H, SW, LP, kWideWG, kWideRepair>), kWideWG, ntiles, 1, a.seq,
                   a.len, a.starts, aligned, words, shard_mask);
  return hipSuccess;
}

template <int K, int S, int M, int H, int SW, int LP>
hipError_t query_wide(const uint64_t *words, uint32_t shard_mask, const SeqArgs &a, const LaunchShape &ls,
                      hipStream_t st) {
  if (a.n_out == 0) return hipSuccess;
  if (a.packed) return hipErrorInvalidValue;  // answers as bytes only
  const uint64_t tile = (uint64_t)LP * kWideWG;
  const int aligned = ((uintptr_t)a.seq & 15u) == 0;
  SBF_LAUNCH_TILES((query_wide_kernel<K, S, M, H, SW, LP, kWideWG>), kWideWG, (a.n_out + tile - 1) / tile,
                   2, a.seq, a.len, a.starts, aligned, words, shard_mask, a.out, a.n_out);
  return hipSuccess;
}

// k-mers per lane in phase 1 (the tile is 256 lanes x LP k-mers)
template <int K, int S, int M, int H, int SW>
hipError_t insert_wide_lp(uint64_t *words, uint32_t shard_mask, const SeqArgs &a, int mode, const LaunchShape &ls,
                          hipStream_t st) {
  if (ls.insert_lane_len == 32) return insert_wide<K, S, M, H, SW, 32>(words, shard_mask, a, mode, ls, st);
  return insert_wide<K, S, M, H, SW, 16>(words, shard_mask, a, mode, ls, st);
}

template <int K, int S, int M, int H, int SW>
hipError_t query_wide_lp(const uint64_t *words, uint32_t shard_mask, const SeqArgs &a, const LaunchShape &ls,
                         hipStream_t st) {
  if (ls.query_lane_len == 32) return query_wide<K, S, M, H, SW, 32>(words, shard_mask, a, ls, st);
  return query_wide<K, S, M, H, SW, 16>(words, shard_mask, a, ls, st);
}

}  // namespace

// Parameter sets (k, s, m, H) with compiled wide-shard kernels, each for
// shards of 4, 8 and 16 words: the paper's default and its H = 8 neighbour.
#define SBF_WIDE_SETS(X) \
  X(31, 28, 16, 4)       \
  X(31, 28, 16, 8)

bool wide_supported(const Geometry &g) {
  if (g.nshards > (1ull << 32)) return false;
  if (g.shard_words != 4 && g.shard_words != 8 && g.shard_words != 16) return false;
  if (g.shard_words == 16 && 64 / g.H < 8) return false;
#define SBF_MATCH(K_, S_, M_, H_) \
  if (g.k == K_ && g.s == S_ && g.m == M_ && g.H == H_) return true;
  SBF_WIDE_SETS(SBF_MATCH)
#undef SBF_MATCH
  return false;
}

bool wide_lane_len_supported(uint32_t n) { return n == 0 || n == 16 || n == 32; }

hipError_t launch_insert_wide(const Geometry &g, uint64_t *words, const SeqArgs &a, int mode, const LaunchShape &ls,
                              hipStream_t st) {
  const uint32_t mask = (uint32_t)(g.nshards - 1);
#define SBF_CALL(K_, S_, M_, H_)                                                              \
  if (g.k == K_ && g.s == S_ && g.m == M_ && g.H == H_) {                                     \
    switch (g.shard_words) {                                                                  \
      case 4: return insert_wide_lp<K_, S_, M_, H_, 4>(words, mask, a, mode, ls, st);         \
      case 8: return insert_wide_lp<K_, S_, M_, H_, 8>(words, mask, a, mode, ls, st);         \
      case 16: return insert_wide_lp<K_, S_, M_, H_, 16>(words, mask, a, mode, ls, st);       \
      default: return hipErrorInvalidValue;                                                   \
    }                                                                                         \
  }
  SBF_WIDE_SETS(SBF_CALL)
#undef SBF_CALL
  return hipErrorInvalidValue;
}

hipError_t launch_query_wide(const Geometry &g, const uint64_t *words, const SeqArgs &a, const LaunchShape &ls,
                             hipStream_t st) {
  const uint32_t mask = (uint32_t)(g.nshards - 1);
#define SBF_CALL(K_, S_, M_, H_)                                                     \
  if (g.k == K_ && g.s == S_ && g.m == M_ && g.H == H_) {                            \
    switch (g.shard_words) {                                                         \
      case 4: return query_wide_lp<K_, S_, M_, H_, 4>(words, mask, a, ls, st);       \
      case 8: return query_wide_lp<K_, S_, M_, H_, 8>(words, mask, a, ls, st);       \
      case 16: return query_wide_lp<K_, S_, M_, H_, 16>(words, mask, a, ls, st);     \
      default: return hipErrorInvalidValue;                                          \
    }                                                                                \
  }
  SBF_WIDE_SETS(SBF_CALL)
#undef SBF_CALL
  return hipErrorInvalidValue;
}

}  // namespace sbf
