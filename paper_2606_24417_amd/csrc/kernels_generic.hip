// Generic insert and query kernels: one k-mer per lane, k, s, m and H known
// only at run time (any 1 <= m, s <= k <= 32, 1 <= H <= 16).  This is the
// paper's per-k-mer scheme (Algorithms 1 and 2) written for wave64:
//   insert: each lane packs its k-mer, takes the minimum m-mer hash, ORs the
//   bits of its k-s+1 s-mers into per-word masks; lanes with equal shard in a
//   contiguous run of the wave merge their masks with a segmented OR scan
//   (ds_bpermute shifts of 1, 2, 4, .., 32 lanes) and the run's last lane
//   issues the atomics;
//   query: each lane loads its shard and tests every bit.
// Also the small utility kernels of the library.
#include "sbf_device.h"
#include "sbf_internal.h"

namespace sbf {
namespace {

constexpr int kGenericWG = 256;
constexpr int kGenericRounds = 4;                         // k-mers per lane
constexpr int kGenericTile = kGenericWG * kGenericRounds;  // k-mers per workgroup
constexpr int kGenericGran = kGenericTile / 16 + 4;

struct RtParams {
  int k, s, m, H;
  uint64_t shard_mask;
};

// k-mer starting at tile position q (packed, first base most significant)
// and its validity.
__device__ __forceinline__ bool load_kmer(const uint32_t *s_codes, const uint32_t *s_vb, int q, int k,
                                          uint64_t &kmer) {
  const int g = q >> 4;
  const int sh = (q & 15) * 2;
  const uint32_t a0 = s_codes[g], a1 = s_codes[g + 1], a2 = s_codes[g + 2];
  const uint32_t hi = sh ? __builtin_amdgcn_alignbit(a0, a1, 32 - sh) : a0;
  const uint32_t lo = sh ? __builtin_amdgcn_alignbit(a1, a2, 32 - sh) : a1;
  const uint64_t win = ((uint64_t)hi << 32) | lo;
  kmer = k == 32 ? win : (win >> (64 - 2 * k));
  uint64_t vbits = 0, sbits = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t vb = s_vb[g + i];
    vbits |= (uint64_t)(vb & 0xFFFFu) << (16 * i);
    sbits |= (uint64_t)(vb >> 16) << (16 * i);
  }
  vbits >>= (q & 15);
  sbits >>= (q & 15);
  const uint64_t kmask = k == 64 ? ~0ull : ((1ull << k) - 1ull);
  const bool all_valid = (vbits & kmask) == kmask;
  const bool no_start = ((sbits >> 1) & (kmask >> 1)) == 0;
  return all_valid && no_start;
}

__device__ __forceinline__ uint64_t sub_window(uint64_t kmer, int k, int L, int j) {
  const uint64_t x = kmer >> (2 * (k - L - j));
  return L == 32 ? x : (x & ((1ull << (2 * L)) - 1ull));
}

__device__ __forceinline__ uint64_t min_hash(uint64_t kmer, const RtParams &p) {
  uint64_t best = ~0ull;
  for (int j = 0; j + p.m <= p.k; ++j) best = umin64(best, minimizer_hash(sub_window(kmer, p.k, p.m, j)));
  return best;
}

template <int SW>
__device__ __forceinline__ void kmer_masks(uint64_t kmer, const RtParams &p, uint64_t (&msk)[SW]) {
#pragma unroll
  for (int w = 0; w < SW; ++w) msk[w] = 0;
  const int W = 64 / p.H;
  for (int j = 0; j + p.s <= p.k; ++j) {
    const uint64_t g = smer_hash(sub_window(kmer, p.k, p.s, j));
    for (int t = 0; t < p.H; ++t) {
      const uint64_t bit = 1ull << bit_address_rt(g, t, p.H);
      int word = t & 3;
      if (SW > 4) word += 4 * (int)((g >> (t * W + 6)) & (uint64_t)(SW / 4 - 1));
#pragma unroll
      for (int w = 0; w < SW; ++w) msk[w] |= (word == w) ? bit : 0ull;
    }
  }
}

template <int SW>
__global__ __launch_bounds__(kGenericWG) void insert_generic_kernel(const uint8_t *__restrict__ seq, uint64_t len,
                                                                    const uint32_t *__restrict__ starts,
                                                                    int aligned16, uint64_t *__restrict__ words,
                                                                    RtParams p) {
  __shared__ uint32_t s_codes[kGenericGran];
  __shared__ uint32_t s_vb[kGenericGran];
  const uint64_t base = (uint64_t)blockIdx.x * kGenericTile;
  stage_granules<kGenericWG>(seq, len, base, starts, aligned16 != 0, kGenericGran, s_codes, s_vb);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  for (int round = 0; round < kGenericRounds; ++round) {
    const int q = round * kGenericWG + threadIdx.x;
    uint64_t kmer;
    const bool v = load_kmer(s_codes, s_vb, q, p.k, kmer);
    uint64_t shard = 0;
    uint64_t msk[SW];
    if (v) {
      shard = min_hash(kmer, p) & p.shard_mask;
      kmer_masks<SW>(kmer, p, msk);
    } else {
#pragma unroll
      for (int w = 0; w < SW; ++w) msk[w] = 0;
    }
    // run heads: first lane, or previous lane invalid or in another shard
    const uint64_t prev_shard = __shfl_up(shard, 1);
    const int prev_v = __shfl_up((int)v, 1);
    const bool head = v && (lane == 0 || !prev_v || prev_shard != shard);
    // segmented inclusive OR scan towards higher lanes; a run ends at a lane
    // whose successor starts a new run (or is invalid)
    bool stop = head || !v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int ostop = __shfl_up((int)stop, d);
      uint64_t o[SW];
#pragma unroll
      for (int w = 0; w < SW; ++w) o[w] = __shfl_up(msk[w], d);
      if (lane >= d && !stop) {
#pragma unroll
        for (int w = 0; w < SW; ++w) msk[w] |= o[w];
        stop = ostop != 0;
      }
    }
    const int next_begins = __shfl_down((int)(head || !v), 1);
    const bool tail = v && (lane == 63 || next_begins);
    if (tail) {
      uint64_t *dst = words + shard * (uint64_t)SW;
#pragma unroll
      for (int w = 0; w < SW; ++w)
        if (msk[w]) atomic_or64(dst + w, msk[w]);
    }
  }
}

template <int SW>
__global__ __launch_bounds__(kGenericWG) void query_generic_kernel(const uint8_t *__restrict__ seq, uint64_t len,
                                                                   const uint32_t *__restrict__ starts,
                                                                   int aligned16,
                                                                   const uint64_t *__restrict__ words, RtParams p,
                                                                   uint8_t *__restrict__ out, uint64_t n_out) {
  acquire_device();  // no filter line cached before this launch is read
  __shared__ uint32_t s_codes[kGenericGran];
  __shared__ uint32_t s_vb[kGenericGran];
  const uint64_t base = (uint64_t)blockIdx.x * kGenericTile;
  stage_granules<kGenericWG>(seq, len, base, starts, aligned16 != 0, kGenericGran, s_codes, s_vb);
  __syncthreads();
  for (int round = 0; round < kGenericRounds; ++round) {
    const int q = round * kGenericWG + threadIdx.x;
    const uint64_t pos = base + (uint64_t)q;
    uint64_t kmer;
    const bool v = load_kmer(s_codes, s_vb, q, p.k, kmer);
    uint8_t present = 0;
    if (v) {
      const uint64_t shard = min_hash(kmer, p) & p.shard_mask;
      uint64_t msk[SW];
      kmer_masks<SW>(kmer, p, msk);
      const uint64_t *src = words + shard * (uint64_t)SW;
      bool all = true;
#pragma unroll
      for (int w = 0; w < SW; ++w) all = all && ((src[w] & msk[w]) == msk[w]);
      present = all ? 1 : 0;
    }
    if (pos < n_out) out[pos] = present;
  }
}

template <int SW>
hipError_t launch_generic_insert_sw(const Geometry &g, uint64_t *words, const SeqArgs &a, hipStream_t st) {
  if (a.len < g.k) return hipSuccess;
  const uint64_t nk = a.len - g.k + 1;
  const uint64_t grid = (nk + kGenericTile - 1) / kGenericTile;
  const RtParams p{(int)g.k, (int)g.s, (int)g.m, (int)g.H, g.nshards - 1};
  const int aligned = ((uintptr_t)a.seq & 15u) == 0;
  hipLaunchKernelGGL(insert_generic_kernel<SW>, dim3((unsigned)grid), dim3(kGenericWG), 0, st, a.seq, a.len,
                     a.starts, aligned, words, p);
  return hipGetLastError();
}

template <int SW>
hipError_t launch_generic_query_sw(const Geometry &g, const uint64_t *words, const SeqArgs &a, hipStream_t st) {
  if (a.n_out == 0) return hipSuccess;
  const uint64_t grid = (a.n_out + kGenericTile - 1) / kGenericTile;
  const RtParams p{(int)g.k, (int)g.s, (int)g.m, (int)g.H, g.nshards - 1};
  const int aligned = ((uintptr_t)a.seq & 15u) == 0;
  hipLaunchKernelGGL(query_generic_kernel<SW>, dim3((unsigned)grid), dim3(kGenericWG), 0, st, a.seq, a.len,
                     a.starts, aligned, words, p, a.out, a.n_out);
  return hipGetLastError();
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_u64_kernel(uint64_t *p, uint64_t n, uint64_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void mark_starts_kernel(const uint64_t *__restrict__ off, uint64_t nrec, uint64_t len,
                                   uint32_t *__restrict__ starts) {
  for (uint64_t r = 1 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nrec;
       r += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t p = off[r];
    if (p < len) atomicOr(starts + (p >> 5), 1u << (uint32_t)(p & 31u));
  }
}

// Add the number of nonzero bytes of p[0, n) to *count: 16 bytes per lane
// per step where aligned, a wave reduction, one atomic per wave.
__global__ void count_nonzero_u8_kernel(const uint8_t *__restrict__ p, uint64_t n, unsigned long long *count) {
  uint64_t c = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t head = ((16u - ((uintptr_t)p & 15u)) & 15u) < n ? ((16u - ((uintptr_t)p & 15u)) & 15u) : n;
  const uint64_t nvec = (n - head) / 16;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid < head) c += p[tid] != 0;
  const uint4 *v = reinterpret_cast<const uint4 *>(p + head);
  for (uint64_t i = tid; i < nvec; i += stride) {
    const uint4 x = v[i];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const uint32_t y = w == 0 ? x.x : w == 1 ? x.y : w == 2 ? x.z : x.w;
      // a byte is nonzero when any of its bits is set
      const uint32_t z = (((y & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | y) & 0x80808080u;
      c += (uint64_t)__popc(z);
    }
  }
  for (uint64_t i = head + nvec * 16 + tid; i < n; i += stride) c += p[i] != 0;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, (unsigned long long)c);
}

// x^e for a small non-negative integer e (square and multiply).
__device__ __forceinline__ double ipow(double x, int e) {
  double r = 1.0;
  while (e) {
    if (e & 1) r *= x;
    x *= x;
    e >>= 1;
  }
  return r;
}

// Load statistics of a filter: *sum += over shards of the probability that a
// k-mer sent to that shard with k-s+1 s-mers of independent ideal hashes finds
// all its bits set, i.e. the product over sectors c of p_c^((k-s+1) n_c), where
// p_c is the fraction of set bits among the sector's words (the word of a hash
// index is uniform among its sector's S/4 words) and n_c the number of hash
// indices t < H with t mod 4 = c (Eq. 1 per sector, Eq. 2 across s-mers);
// *bits += the set bits.  One shard per lane, a wave reduction, one atomic
// per wave.
template <int SW>
__global__ void estimate_fpr_kernel(const uint64_t *__restrict__ words, uint64_t nshards, int H, int z1, double *sum,
                                    unsigned long long *bits) {
  constexpr int G = SW / 4;
  int expo[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) expo[c] = z1 * ((H - c + 3) / 4);  // hash indices t < H with t mod 4 = c
  double acc = 0.0;
  uint64_t ones = 0;
  for (uint64_t sh = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; sh < nshards;
       sh += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t *w = words + sh * SW;
    double prob = 1.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int pop = 0;
#pragma unroll
      for (int g = 0; g < G; ++g) pop += __popcll(w[c + 4 * g]);
      ones += (uint64_t)pop;
      prob *= ipow((double)pop / (64.0 * G), expo[c]);
    }
    acc += prob;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    acc += __shfl_xor(acc, d, 64);
    ones += __shfl_xor(ones, d, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (acc != 0.0) atomicAdd(sum, acc);
    if (ones) atomicAdd(bits, (unsigned long long)ones);
  }
}

unsigned grid_for(uint64_t n, unsigned block) {
  uint64_t g = (n + block - 1) / block;
  if (g > 65536u) g = 65536u;
  if (g == 0) g = 1;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_insert_generic(const Geometry &g, uint64_t *words, const SeqArgs &a, hipStream_t st) {
  switch (g.shard_words) {
    case 4: return launch_generic_insert_sw<4>(g, words, a, st);
    case 8: return launch_generic_insert_sw<8>(g, words, a, st);
    case 16: return launch_generic_insert_sw<16>(g, words, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_query_generic(const Geometry &g, const uint64_t *words, const SeqArgs &a, hipStream_t st) {
  if (a.packed) return hipErrorInvalidValue;  // answers as bits come from the lane query only
  switch (g.shard_words) {
    case 4: return launch_generic_query_sw<4>(g, words, a, st);
    case 8: return launch_generic_query_sw<8>(g, words, a, st);
    case 16: return launch_generic_query_sw<16>(g, words, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, value);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t value, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, value);
  return hipGetLastError();
}

hipError_t launch_count_nonzero_u8(const uint8_t *p, uint64_t n, uint64_t *count, hipStream_t st) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(count_nonzero_u8_kernel, dim3(grid_for((n + 15) / 16, 256)), dim3(256), 0, st, p, n,
                     (unsigned long long *)count);
  return hipGetLastError();
}

hipError_t launch_estimate_fpr(const Geometry &g, const uint64_t *words, double *sum, uint64_t *bits,
                               hipStream_t st) {
  const unsigned grid = grid_for(g.nshards, 256);
  const int z1 = (int)(g.k - g.s + 1);
  switch (g.shard_words) {
    case 4:
      hipLaunchKernelGGL(estimate_fpr_kernel<4>, dim3(grid), dim3(256), 0, st, words, g.nshards, (int)g.H, z1, sum,
                         (unsigned long long *)bits);
      break;
    case 8:
      hipLaunchKernelGGL(estimate_fpr_kernel<8>, dim3(grid), dim3(256), 0, st, words, g.nshards, (int)g.H, z1, sum,
                         (unsigned long long *)bits);
      break;
    case 16:
      hipLaunchKernelGGL(estimate_fpr_kernel<16>, dim3(grid), dim3(256), 0, st, words, g.nshards, (int)g.H, z1, sum,
                         (unsigned long long *)bits);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_mark_record_starts(const uint64_t *off, uint64_t nrec, uint64_t len, uint32_t *starts,
                                     hipStream_t st) {
  if (nrec < 2) return hipSuccess;
  hipLaunchKernelGGL(mark_starts_kernel, dim3(grid_for(nrec - 1, 256)), dim3(256), 0, st, off, nrec, len, starts);
  return hipGetLastError();
}

}  // namespace sbf
