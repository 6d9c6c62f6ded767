// Run-time parameter super-k-mer kernels for gfx950: insert and query for any
// (k, s, m, H) with m <= k <= 32, s <= k and H <= 8, and shards of 4, 8 or 16
// words.  The lane and wide-shard kernels unroll their sliding minimum and
// s-mer windows for a few compiled parameter sets; the paper's parameter
// study (Section "Parameter Selection") spans hundreds of sets, so these
// kernels take k, s, m and H at run time and keep the super-k-mer work:
//   phase 1, per tile of WG x LP k-mers:
//     * each k-mer's validity (one ballot per 64 k-mers) and the minimizer
//       hash h_M of every m-mer position of the tile, once, into LDS, each
//       from a 64-bit base window of the staged codes (one position per lane
//       at a time: consecutive lanes, consecutive positions);
//     * then, per lane over its own LP consecutive k-mers, the minimum of
//       each k-mer's w = k-m+1 m-mer hashes: for w >= LP the LP windows
//       share positions LP-1 .. w-1, so one minimum over those, suffix
//       minima of the positions before and prefix minima of those after
//       give all LP windows (about (w + 3 LP) / LP compares per k-mer), and
//       the k-mer's shard;
//     * then, over the same LDS, the H bit addresses of every s-mer position
//       (the bit slicing of Section "Optimizations"), one byte each: bit in
//       the low 6 bits, word group above them;
//   phase 2 for 4-word shards, as in the lane kernels: lane t walks its LP
//     k-mers in order.  Insert: each run of valid k-mers with one shard (the
//     super-k-mers of Section "Minimizers and Super-k-mers") is written once,
//     by the lane holding its first k-mer, whose mask starts with that
//     k-mer's (k-s+1)*H bits and adds one s-mer per following k-mer, also
//     past the lane's own k-mers; finished runs are buffered and applied as
//     read-modify-writes by lane pairs (completed by the repair walk) or as
//     atomic ORs (Algorithm 1).  Query: a lane loads a shard where it changes
//     and tests each k-mer's mask against it (Algorithm 2);
//   phase 2 for 8- and 16-word shards, as in the wide-shard kernels: each
//     wave walks 64 consecutive k-mers per step, finds the runs of valid
//     k-mers with equal shard by ballot and moves each run's shard with SW/2
//     lanes, one 16-byte piece each: insert ORs the run's s-mer bits into
//     the pieces, query stages the run's shard in LDS and tests each k-mer's
//     bits there.
// Results are bit-identical to the per-k-mer definition for every parameter
// set these kernels accept.
#include "sbf_segments.h"
#include "sbf_tiles.h"

#include <type_traits>

namespace sbf {
namespace {

constexpr int kParamKMax = 32;

// Run-time parameters of a launch.
struct ParamGeo {
  int k;       // k-mer length (<= 32)
  int z;       // k - s: s-mers per k-mer minus one
  int w;       // k - m + 1: m-mers per k-mer
  int H;       // hash indices per s-mer (<= 8)
  int slice;   // 64 / H: hash bits per index
  int m_shift; // 64 - 2m: an m-mer from a 64-bit base window
  int s_shift; // 64 - 2s: an s-mer from a 64-bit base window
  uint32_t shard_mask;
};

// LDS of one tile: the staged sequence, one 64-bit slot per m-mer / s-mer
// position (m-mer hashes, then the s-mers' packed bit addresses), and per
// k-mer its shard and validity.  The m-mer hashes are stored one slot apart
// every LP positions (hpos), so that lanes reading their own LP consecutive
// positions hit different banks.
template <int LP, int WG>
struct ParamTile {
  static constexpr int TILE = WG * LP;
  static constexpr int NPOS = TILE + kParamKMax;  // w - 1 and z are below 32
  static constexpr int NSLOT = NPOS + NPOS / LP + 1;
  static constexpr int NGRAN = TILE / 16 + 4;      // windows reach base TILE + 62
  uint32_t codes[NGRAN];
  uint32_t vb[NGRAN];
  uint64_t pos[NSLOT];
  uint32_t shard[TILE];
  uint64_t kv[TILE / 64];  // bit q % 64 of word q / 64: k-mer q is valid

  __device__ __forceinline__ bool valid(int q) const { return (kv[q >> 6] >> (q & 63)) & 1ull; }
  // slot of the m-mer hash of position j
  static __device__ __forceinline__ int hpos(int j) { return j + j / LP; }
};

// Bases j .. j+31 of the staged tile as one 64-bit value, first base most
// significant (granules g .. g+2 hold bases 16g .. 16g+47).
__device__ __forceinline__ uint64_t base_window(const uint32_t *codes, int j) {
  const int g = j >> 4, sh = (j & 15) * 2;
  const uint32_t a = codes[g], b = codes[g + 1], c = codes[g + 2];
  const uint32_t hi = sh ? __builtin_amdgcn_alignbit(a, b, 32 - sh) : a;
  const uint32_t lo = sh ? __builtin_amdgcn_alignbit(b, c, 32 - sh) : b;
  return ((uint64_t)hi << 32) | lo;
}

// k-mer q of the tile: bases q .. q+k-1 valid and no record starting at
// q+1 .. q+k-1 (k-mers never span records).  The 48 bases from granule q/16
// cover it for k <= 32.
__device__ __forceinline__ bool kmer_ok(const uint32_t *vb, int q, int k) {
  const int g = q >> 4, off = q & 15;
  const uint32_t a = vb[g], b = vb[g + 1], c = vb[g + 2];
  const uint64_t valid = (uint64_t)(a & 0xFFFFu) | ((uint64_t)(b & 0xFFFFu) << 16) | ((uint64_t)(c & 0xFFFFu) << 32);
  const uint64_t start = (uint64_t)(a >> 16) | ((uint64_t)(b >> 16) << 16) | ((uint64_t)(c >> 16) << 32);
  const uint64_t need = (1ull << k) - 1ull;
  return ((valid >> off) & need) == need && ((start >> (off + 1)) & (need >> 1)) == 0;
}

template <int SW, int LP, int WG>
__device__ __forceinline__ void param_phase1(ParamTile<LP, WG> &T, const ParamGeo &P,
                                             const uint8_t *__restrict__ seq, uint64_t len, uint64_t base,
                                             const uint32_t *__restrict__ starts, bool aligned16) {
  using Tl = ParamTile<LP, WG>;
  // address byte: bit (6 bits), then log2(SW/4) bits of word group
  constexpr uint32_t AMASK = 16u * SW - 1u;
  stage_granules<WG>(seq, len, base, starts, aligned16, Tl::NGRAN, T.codes, T.vb);
  __syncthreads();
  const int t = threadIdx.x;
  // validity: a wave judges 64 consecutive k-mers per ballot
  for (int q = t; q < Tl::TILE; q += WG) {
    const uint64_t b = __ballot(kmer_ok(T.vb, q, P.k));
    if ((t & 63) == 0) T.kv[q >> 6] = b;
  }
  // m-mer hashes of positions 0 .. TILE + w - 2
  for (int j = t; j < Tl::TILE + P.w - 1; j += WG) T.pos[Tl::hpos(j)] = minimizer_hash(base_window(T.codes, j) >> P.m_shift);
  __syncthreads();
  // minimizer of each of the lane's k-mers q0 .. q0+LP-1 (window of
  // positions q .. q+w-1)
  {
    const int q0 = t * LP;
    const uint64_t *H = T.pos;
    uint64_t win[LP];
    if (P.w >= LP) {
      // positions q0+LP-1 .. q0+w-1 lie in every window
      uint64_t mid = H[Tl::hpos(q0 + LP - 1)];
      for (int j = q0 + LP; j < q0 + P.w; ++j) mid = umin64(mid, H[Tl::hpos(j)]);
      // window r adds positions q0+r .. q0+LP-2 (suffix) and q0+w .. q0+w+r-1 (prefix)
      uint64_t suf = ~0ull, pre = ~0ull;
#pragma unroll
      for (int r = LP - 1; r >= 0; --r) {
        if (r < LP - 1) suf = umin64(suf, H[Tl::hpos(q0 + r)]);
        win[r] = umin64(suf, mid);
      }
#pragma unroll
      for (int r = 1; r < LP; ++r) {
        pre = umin64(pre, H[Tl::hpos(q0 + P.w + r - 1)]);
        win[r] = umin64(win[r], pre);
      }
    } else {
#pragma unroll
      for (int r = 0; r < LP; ++r) {
        uint64_t m = ~0ull;
        for (int j = q0 + r; j < q0 + r + P.w; ++j) m = umin64(m, H[Tl::hpos(j)]);
        win[r] = m;
      }
    }
#pragma unroll
    for (int r = 0; r < LP; ++r) T.shard[q0 + r] = (uint32_t)win[r] & P.shard_mask;
  }
  __syncthreads();
  // packed bit addresses of s-mer positions 0 .. TILE + z - 1, over the hashes
  for (int j = t; j < Tl::TILE + P.z; j += WG) {
    const uint64_t g = smer_hash(base_window(T.codes, j) >> P.s_shift);
    uint64_t pk = 0;
    for (int h = 0; h < P.H; ++h) pk |= (uint64_t)((uint32_t)(g >> (h * P.slice)) & AMASK) << (8 * h);
    T.pos[j] = pk;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// 4-word shards: phase 2 as a lane walk over the lane's LP k-mers.  The bits
// of a k-mer are those of its s-mers q .. q+z, so consecutive k-mers of one
// shard share all but one s-mer, and a segment's mask grows by one s-mer per
// k-mer.
// ---------------------------------------------------------------------------

// Bits of the s-mer with packed addresses pk over the four words of a 4-word
// shard: bit b of word t mod 4 for the address byte b of hash index t < H.
// HMAX (4 or 8) bounds H at compile time; one[t] is 1 for t < H and 0 beyond,
// so hash indices past H add nothing.
template <int HMAX>
__device__ __forceinline__ void smer_bits4(uint64_t pk, const uint32_t (&one)[HMAX], uint64_t (&oh)[4]) {
  oh[0] = oh[1] = oh[2] = oh[3] = 0;
#pragma unroll
  for (int h = 0; h < HMAX; ++h) oh[h & 3] |= (uint64_t)one[h] << ((uint32_t)(pk >> (8 * h)) & 63u);
}

// Mask of k-mer q: the bits of its s-mers q .. q+z.
template <int HMAX>
__device__ __forceinline__ void kmer_mask4(const uint64_t *pos, int q, int z, const uint32_t (&one)[HMAX],
                                           uint64_t (&A)[4]) {
  A[0] = A[1] = A[2] = A[3] = 0;
  for (int j = 0; j <= z; ++j) {
    uint64_t oh[4];
    smer_bits4<HMAX>(pos[q + j], one, oh);
#pragma unroll
    for (int w = 0; w < 4; ++w) A[w] |= oh[w];
  }
}

// Insert: every run of the tile (consecutive valid k-mers with one shard) is
// written once, by the lane that holds its first k-mer; that lane follows
// the run past its own k-mers to the run's end in the tile, and the lanes
// whose first k-mers continue a run from an earlier lane skip them.  With
// about one run per lane, two buffer slots per lane suffice (and leave LDS
// for three workgroups per CU).
template <int LP, int WG, int MODE, int HMAX>
__global__ __launch_bounds__(WG) void insert_param4_kernel(const uint8_t *__restrict__ seq, uint64_t len,
                                                           const uint32_t *__restrict__ starts, int aligned16,
                                                           uint64_t *__restrict__ words, ParamGeo P, TileQueue tq) {
  using Tl = ParamTile<LP, WG>;
  __shared__ Tl T;
  __shared__ SegmentBuffer<(MODE == kAtomic ? 1 : WG), 2> s_buf;
  __shared__ uint32_t s_next_tile;
  uint32_t one[HMAX];
#pragma unroll
  for (int h = 0; h < HMAX; ++h) one[h] = h < P.H ? 1u : 0u;

  acquire_device();
  uint64_t tile;
  for (bool first = true; next_tile(tq, &s_next_tile, first, tile); first = false) {
    const uint64_t base = tile * (uint64_t)Tl::TILE;
    param_phase1<4, LP, WG>(T, P, seq, len, base, starts, aligned16 != 0);

    const int q0 = threadIdx.x * LP;
    uint64_t seg[4] = {0, 0, 0, 0};  // the open segment's masks
    uint32_t cur = 0;                // and its shard
    bool open = false;
    int nbuf = 0;
    // k-mers continuing a run that started in an earlier lane
    bool skip = q0 > 0 && T.valid(q0 - 1);
    uint32_t prev_sh = q0 > 0 ? T.shard[q0 - 1] : 0u;
#pragma unroll
    for (int r = 0; r < LP; ++r) {
      const int q = q0 + r;
      const bool v = T.valid(q);
      const uint32_t sh = T.shard[q];
      skip = skip && v && sh == prev_sh;
      prev_sh = sh;
      if (!skip) {
        if (open && v && sh == cur) {
          uint64_t oh[4];
          smer_bits4<HMAX>(T.pos[q + P.z], one, oh);
#pragma unroll
          for (int w = 0; w < 4; ++w) seg[w] |= oh[w];
        } else {
          if (open) push_segment<4, MODE>(s_buf, nbuf, words, cur, seg);
          if (v) {
            kmer_mask4<HMAX>(T.pos, q, P.z, one, seg);
            cur = sh;
          }
          open = v;
        }
      }
    }
    if (open) {
      // the lane's last run may go on into the next lanes' k-mers
      for (int q = q0 + LP; q < Tl::TILE && T.valid(q) && T.shard[q] == cur; ++q) {
        uint64_t oh[4];
        smer_bits4<HMAX>(T.pos[q + P.z], one, oh);
#pragma unroll
        for (int w = 0; w < 4; ++w) seg[w] |= oh[w];
      }
      push_segment<4, MODE>(s_buf, nbuf, words, cur, seg);
    }
    drain_segments<MODE>(s_buf, nbuf, words);
  }
}

// Query (and the insert's repair walk): a lane loads a shard where the shard
// changes along its k-mers and keeps the words for the k-mers after it; each
// k-mer's mask is built whole (the same work in every lane, where testing
// each s-mer once would make the lanes that start a segment wait for z more
// tests at nearly every step).
template <int LP, int WG, int HMAX, bool REPAIR>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(4))) void query_param4_kernel(const uint8_t *__restrict__ seq, uint64_t len,
                                                          const uint32_t *__restrict__ starts, int aligned16,
                                                          typename std::conditional<REPAIR, uint64_t, const uint64_t>::type *words,
                                                          ParamGeo P, uint8_t *__restrict__ out, uint64_t n_out,
                                                          int out_aligned8, TileQueue tq) {
  using Tl = ParamTile<LP, WG>;
  static_assert(LP % 8 == 0 && LP <= 32, "whole 8-byte answer groups, answer bits in one 32-bit word");
  __shared__ Tl T;
  __shared__ uint32_t s_next_tile;
  uint32_t one[HMAX];
#pragma unroll
  for (int h = 0; h < HMAX; ++h) one[h] = h < P.H ? 1u : 0u;

  acquire_device();
  uint64_t tile;
  for (bool first = true; next_tile(tq, &s_next_tile, first, tile); first = false) {
    const uint64_t base = tile * (uint64_t)Tl::TILE;
    param_phase1<4, LP, WG>(T, P, seq, len, base, starts, aligned16 != 0);

    const int q0 = threadIdx.x * LP;
    uint32_t ans = 0;
    uint64_t got[4] = {0, 0, 0, 0};
    uint32_t cur = 0;
    bool have = false;
#pragma unroll
    for (int r = 0; r < LP; ++r) {
      const int q = q0 + r;
      const uint32_t sh = T.shard[q];
      if (T.valid(q)) {
        if (!have || sh != cur) {
          const uint4 *p = reinterpret_cast<const uint4 *>(words + 4ull * (uint64_t)sh);
          const uint4 lo = p[0], hi = p[1];
          got[0] = ((uint64_t)lo.y << 32) | lo.x;
          got[1] = ((uint64_t)lo.w << 32) | lo.z;
          got[2] = ((uint64_t)hi.y << 32) | hi.x;
          got[3] = ((uint64_t)hi.w << 32) | hi.z;
          cur = sh;
          have = true;
        }
        uint64_t A[4];
        kmer_mask4<HMAX>(T.pos, q, P.z, one, A);
        uint64_t miss[4];
#pragma unroll
        for (int w = 0; w < 4; ++w) miss[w] = A[w] & ~got[w];
        if constexpr (REPAIR) {
          // OR the bits a racing store dropped into the shard and into the
          // cached words, so that later k-mers of the lane do not repeat them
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            if (miss[w]) atomic_or64(words + 4ull * (uint64_t)sh + w, miss[w]);
            got[w] |= miss[w];
          }
        } else {
          if ((miss[0] | miss[1] | miss[2] | miss[3]) == 0) ans |= 1u << r;
        }
      }
    }
    if constexpr (!REPAIR) {
      // answer bytes: four bits x spread to bytes by x * 0x204081
      const uint64_t pos0 = base + (uint64_t)q0;
      if (out_aligned8 && pos0 + LP <= n_out) {
#pragma unroll
        for (int c = 0; c < LP / 8; ++c) {
          const uint32_t b = ans >> (8 * c);
          *reinterpret_cast<uint2 *>(out + pos0 + 8 * c) =
              make_uint2(((b & 0xFu) * 0x204081u) & 0x01010101u, (((b >> 4) & 0xFu) * 0x204081u) & 0x01010101u);
        }
      } else {
        for (int r = 0; r < LP; ++r)
          if (pos0 + r < n_out) out[pos0 + r] = (uint8_t)((ans >> r) & 1u);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Insert.  Lane (run j, piece p) of a round owns words 2p and 2p+1 of run j's
// shard: sectors e = 2p mod 4 and e+1 of word group p / 2, reached by hash
// indices e, e+4 (word 2p) and e+1, e+5 (word 2p+1).
// ---------------------------------------------------------------------------
template <int SW, int LP, int WG, int MODE>
__global__ __launch_bounds__(WG) void insert_param_kernel(const uint8_t *__restrict__ seq, uint64_t len,
                                                          const uint32_t *__restrict__ starts, int aligned16,
                                                          uint64_t *__restrict__ words, ParamGeo P, TileQueue tq) {
  using Tl = ParamTile<LP, WG>;
  constexpr int NWAVES = WG / 64;
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
  const int p = lane % LPR;
  const int e = (2 * p) & 3;
  const uint32_t grp = (uint32_t)(p >> 1);

  acquire_device();
  uint64_t tile;
  for (bool first = true; next_tile(tq, &s_next_tile, first, tile); first = false) {
    const uint64_t base = tile * (uint64_t)Tl::TILE;
    param_phase1<SW, LP, WG>(T, P, seq, len, base, starts, aligned16 != 0);

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
        const uint64_t hb = heads & upto;
        const int a = hb ? s0 + 63 - __clzll((long long)hb) : carry;
        const int j = __popcll(tails & upto) - 1;
        s_run_shard[wave][j] = sh;
        s_run_span[wave][j] = (uint32_t)a | ((uint32_t)q << 16);
      }
      if (heads) carry = s0 + 63 - __clzll((long long)heads);
      const int nruns = __popcll(tails);
      for (int r0 = 0; r0 < nruns; r0 += RPR) {
        const int j = r0 + lane / LPR;
        if (j < nruns) {
          const uint32_t rsh = s_run_shard[wave][j];
          const uint32_t span = s_run_span[wave][j];
          const int a = (int)(span & 0xFFFFu);
          const int b = (int)(span >> 16);
          uint64_t *line = words + (uint64_t)rsh * SW + 2 * p;
          uint64_t o0 = 0, o1 = 0;
          if constexpr (MODE == kStore) {
            const uint4 piece = *reinterpret_cast<const uint4 *>(line);
            o0 = ((uint64_t)piece.y << 32) | piece.x;
            o1 = ((uint64_t)piece.w << 32) | piece.z;
          }
          uint64_t m0 = 0, m1 = 0;
          for (int x = a; x <= b + P.z; ++x) {
            const uint64_t pk = T.pos[x];
            for (int h = e; h < P.H; h += 4) {
              const uint32_t b0 = (uint32_t)(pk >> (8 * h)) & 0xFFu;
              uint64_t one = 1ull << (b0 & 63u);
              if constexpr (SW > 4) one = (b0 >> 6) == grp ? one : 0ull;
              m0 |= one;
              if (h + 1 < P.H) {
                const uint32_t b1 = (uint32_t)(pk >> (8 * h + 8)) & 0xFFu;
                uint64_t one1 = 1ull << (b1 & 63u);
                if constexpr (SW > 4) one1 = (b1 >> 6) == grp ? one1 : 0ull;
                m1 |= one1;
              }
            }
          }
          if constexpr (MODE == kStore) {
            if ((o0 | m0) != o0 || (o1 | m1) != o1) store_pair_coherent(line, o0 | m0, o1 | m1);
          } else {
            if (m0) atomic_or64(line, m0);
            if (m1) atomic_or64(line + 1, m1);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Query (and the insert's repair walk): the lines of up to PASS runs of a
// step are staged in LDS sector-major (dword (t mod 4) * SW/2 + (byte >> 5)
// holds the bit of address byte `byte` of hash index t).
// ---------------------------------------------------------------------------
template <int SW, int LP, int WG, bool REPAIR>
__global__ __launch_bounds__(WG) void query_param_kernel(const uint8_t *__restrict__ seq, uint64_t len,
                                                         const uint32_t *__restrict__ starts, int aligned16,
                                                         typename std::conditional<REPAIR, uint64_t, const uint64_t>::type *words,
                                                         ParamGeo P, uint8_t *__restrict__ out, uint64_t n_out,
                                                         TileQueue tq) {
  using Tl = ParamTile<LP, WG>;
  constexpr int NWAVES = WG / 64;
  constexpr int PER_WAVE = Tl::TILE / NWAVES;
  constexpr int LPR = SW / 2;
  constexpr int RPR = 64 / LPR;
  constexpr int PASS = 16;
  constexpr int HALF = SW / 2;

  __shared__ Tl T;
  __shared__ uint32_t s_run_shard[NWAVES][64];
  __shared__ uint2 s_line[NWAVES][PASS][SW];
  __shared__ uint32_t s_next_tile;

  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int q0 = wave * PER_WAVE;
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int p = lane % LPR;
  const int e = (2 * p) & 3;
  const int grp = p >> 1;
  const int d0 = (e * HALF + 2 * grp) / 2;  // dword pair of word 2p in a staged line
  const int d1 = ((e + 1) * HALF + 2 * grp) / 2;

  acquire_device();
  uint64_t tile;
  for (bool first = true; next_tile(tq, &s_next_tile, first, tile); first = false) {
    const uint64_t base = tile * (uint64_t)Tl::TILE;
    param_phase1<SW, LP, WG>(T, P, seq, len, base, starts, aligned16 != 0);

    for (int step = 0; step < LP; ++step) {
      const int q = q0 + step * 64 + lane;
      const bool v = T.valid(q);
      const uint32_t sh = T.shard[q];
      const bool prev_same = lane > 0 && T.valid(q - 1) && T.shard[q - 1] == sh;
      const bool head = v && !prev_same;
      const uint64_t heads = __ballot(head);
      const int ri = __popcll(heads & upto) - 1;
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
            const uint4 piece = *reinterpret_cast<const uint4 *>(words + (uint64_t)rsh * SW + 2 * p);
            s_line[wave][slot][d0] = make_uint2(piece.x, piece.y);
            s_line[wave][slot][d1] = make_uint2(piece.z, piece.w);
          }
        }
        if (v && ri >= r0 && ri < r0 + PASS) {
          const uint32_t *L = reinterpret_cast<const uint32_t *>(s_line[wave][ri - r0]);
          uint32_t acc = 1;
          for (int o = 0; o <= P.z; ++o) {
            const uint64_t pk = T.pos[q + o];
            for (int h = 0; h < P.H; ++h) {
              const uint32_t byte = (uint32_t)(pk >> (8 * h)) & 0xFFu;
              const uint32_t hit = (L[(h & 3) * HALF + (byte >> 5)] >> (byte & 31u)) & 1u;
              if constexpr (REPAIR) {
                if (!hit) {
                  const int wd = (h & 3) + 4 * (int)(byte >> 6);
                  atomic_or64(words + (uint64_t)sh * SW + wd, 1ull << (byte & 63u));
                }
              } else {
                acc &= hit;
              }
            }
          }
          ok = acc;
        }
      }
      if constexpr (!REPAIR) {
        const uint64_t pos = base + (uint64_t)q;
        if (pos < n_out) out[pos] = (uint8_t)(v ? ok : 0u);
      }
    }
  }
}

constexpr int kParamWG = 256;

ParamGeo param_geo(const Geometry &g) {
  ParamGeo P;
  P.k = (int)g.k;
  P.z = (int)(g.k - g.s);
  P.w = (int)(g.k - g.m + 1);
  P.H = (int)g.H;
  P.slice = 64 / (int)g.H;
  P.m_shift = 64 - 2 * (int)g.m;
  P.s_shift = 64 - 2 * (int)g.s;
  P.shard_mask = (uint32_t)(g.nshards - 1);
  return P;
}

template <int LP, int HMAX>
hipError_t insert_param4(const ParamGeo &P, uint64_t *words, const SeqArgs &a, int mode, const LaunchShape &ls,
                         hipStream_t st) {
  const uint64_t nk = a.len - P.k + 1;
  const uint64_t tile = (uint64_t)LP * kParamWG;
  const uint64_t ntiles = (nk + tile - 1) / tile;
  const int aligned = ((uintptr_t)a.seq & 15u) == 0;
  if (mode == kInsertAtomicMode) {
    SBF_LAUNCH_TILES((insert_param4_kernel<LP, kParamWG, kAtomic, HMAX>), kParamWG, ntiles, 0, a.seq, a.len,
                     a.starts, aligned, words, P);
    return hipSuccess;
  }
  SBF_LAUNCH_TILES((insert_param4_kernel<LP, kParamWG, kStore, HMAX>), kParamWG, ntiles, 0, a.seq, a.len, a.starts,
                   aligned, words, P);
  SBF_LAUNCH_TILES((query_param4_kernel<LP, kParamWG, HMAX, true>), kParamWG, ntiles, 1, a.seq, a.len, a.starts,
                   aligned, words, P, (uint8_t *)nullptr, nk, 0);
  return hipSuccess;
}

template <int LP, int HMAX>
hipError_t query_param4(const ParamGeo &P, const uint64_t *words, const SeqArgs &a, const LaunchShape &ls,
                        hipStream_t st) {
  const uint64_t tile = (uint64_t)LP * kParamWG;
  const int aligned = ((uintptr_t)a.seq & 15u) == 0;
  SBF_LAUNCH_TILES((query_param4_kernel<LP, kParamWG, HMAX, false>), kParamWG, (a.n_out + tile - 1) / tile, 2, a.seq,
                   a.len, a.starts, aligned, words, P, a.out, a.n_out, (int)(((uintptr_t)a.out & 7u) == 0));
  return hipSuccess;
}

template <int SW, int LP>
hipError_t insert_param(const ParamGeo &P, uint64_t *words, const SeqArgs &a, int mode, const LaunchShape &ls,
                        hipStream_t st) {
  if (a.len < (uint64_t)P.k) return hipSuccess;
  if constexpr (SW == 4) {
    return P.H <= 4 ? insert_param4<LP, 4>(P, words, a, mode, ls, st) : insert_param4<LP, 8>(P, words, a, mode, ls, st);
  } else {
    const uint64_t nk = a.len - P.k + 1;
    const uint64_t tile = (uint64_t)LP * kParamWG;
    const uint64_t ntiles = (nk + tile - 1) / tile;
    const int aligned = ((uintptr_t)a.seq & 15u) == 0;
    if (mode == kInsertAtomicMode) {
      SBF_LAUNCH_TILES((insert_param_kernel<SW, LP, kParamWG, kAtomic>), kParamWG, ntiles, 0, a.seq, a.len, a.starts,
                       aligned, words, P);
      return hipSuccess;
    }
    SBF_LAUNCH_TILES((insert_param_kernel<SW, LP, kParamWG, kStore>), kParamWG, ntiles, 0, a.seq, a.len, a.starts,
                     aligned, words, P);
    SBF_LAUNCH_TILES((query_param_kernel<SW, LP, kParamWG, true>), kParamWG, ntiles, 1, a.seq, a.len, a.starts,
                     aligned, words, P, (uint8_t *)nullptr, nk);
    return hipSuccess;
  }
}

template <int SW, int LP>
hipError_t query_param(const ParamGeo &P, const uint64_t *words, const SeqArgs &a, const LaunchShape &ls,
                       hipStream_t st) {
  if (a.n_out == 0) return hipSuccess;
  if (a.packed) return hipErrorInvalidValue;  // answers as bytes only
  if constexpr (SW == 4) {
    return P.H <= 4 ? query_param4<LP, 4>(P, words, a, ls, st) : query_param4<LP, 8>(P, words, a, ls, st);
  } else {
    const uint64_t tile = (uint64_t)LP * kParamWG;
    const int aligned = ((uintptr_t)a.seq & 15u) == 0;
    SBF_LAUNCH_TILES((query_param_kernel<SW, LP, kParamWG, false>), kParamWG, (a.n_out + tile - 1) / tile, 2, a.seq,
                     a.len, a.starts, aligned, words, P, a.out, a.n_out);
    return hipSuccess;
  }
}

template <int SW>
hipError_t insert_param_lp(const ParamGeo &P, uint64_t *words, const SeqArgs &a, int mode, const LaunchShape &ls,
                           hipStream_t st) {
  if (ls.insert_lane_len == 16) return insert_param<SW, 16>(P, words, a, mode, ls, st);
  return insert_param<SW, 8>(P, words, a, mode, ls, st);
}

template <int SW>
hipError_t query_param_lp(const ParamGeo &P, const uint64_t *words, const SeqArgs &a, const LaunchShape &ls,
                          hipStream_t st) {
  if (ls.query_lane_len == 16) return query_param<SW, 16>(P, words, a, ls, st);
  return query_param<SW, 8>(P, words, a, ls, st);
}

}  // namespace

bool param_supported(const Geometry &g) {
  if (g.nshards > (1ull << 32)) return false;
  if (g.shard_words != 4 && g.shard_words != 8 && g.shard_words != 16) return false;
  return g.k >= 1 && g.k <= (uint32_t)kParamKMax && g.m >= 1 && g.m <= g.k && g.s >= 1 && g.s <= g.k && g.H >= 1 &&
         g.H <= 8;
}

hipError_t launch_insert_param(const Geometry &g, uint64_t *words, const SeqArgs &a, int mode, const LaunchShape &ls,
                               hipStream_t st) {
  if (!param_supported(g)) return hipErrorInvalidValue;
  const ParamGeo P = param_geo(g);
  switch (g.shard_words) {
    case 4: return insert_param_lp<4>(P, words, a, mode, ls, st);
    case 8: return insert_param_lp<8>(P, words, a, mode, ls, st);
    default: return insert_param_lp<16>(P, words, a, mode, ls, st);
  }
}

hipError_t launch_query_param(const Geometry &g, const uint64_t *words, const SeqArgs &a, const LaunchShape &ls,
                              hipStream_t st) {
  if (!param_supported(g)) return hipErrorInvalidValue;
  const ParamGeo P = param_geo(g);
  switch (g.shard_words) {
    case 4: return query_param_lp<4>(P, words, a, ls, st);
    case 8: return query_param_lp<8>(P, words, a, ls, st);
    default: return query_param_lp<16>(P, words, a, ls, st);
  }
}

}  // namespace sbf
