// Device helpers shared by the SBF kernels (gfx950, wave64).
//
// Sequence staging: a workgroup copies its tile of ASCII bases from HBM with
// 16-byte loads and stores it in LDS as "granules" of 16 bases:
//   codes[g]: 2 bits per base, the first base in bits 31:30 (the packing
//             order of the paper's PackKmer: first base most significant);
//   vb[g]:    bits 0..15 = base valid, bits 16..31 = a record starts at
//             this base (record batches).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sbf {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Minimizer hash multiplier: floor(2^64 / golden ratio) (Fibonacci hashing;
// Section "Optimizations": a single multiplicative mix).
constexpr uint64_t kMinimizerMul = 0x9E3779B97F4A7C15ull;
// s-mer hash multiplier of the SplitMix64 finaliser's first round (Section
// "Optimizations": a stronger mix with an additional xorshift).
constexpr uint64_t kSmerMul = 0xBF58476D1CE4E5B9ull;

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

// h_M of a (zero-extended) m-mer of at most 16 bases.
__device__ __forceinline__ uint64_t minimizer_hash32(uint32_t y) { return (uint64_t)y * kMinimizerMul; }
// The same low 64 bits of y * kMinimizerMul as one 32x32->64 multiply plus
// the high word's 32-bit partial product.  The empty asm operand keeps that
// partial product a plain multiply and add: fused into a second 64-bit
// multiply-add it needs its addend in a register pair, which costs two moves
// per hash.  Measured faster in the lane kernels and slower in the wide-shard
// kernels, whose m-mer loop the compiler schedules better in the fused form.
__device__ __forceinline__ uint64_t minimizer_hash32_split(uint32_t y) {
  const uint64_t p = (uint64_t)y * (uint32_t)kMinimizerMul;
  uint32_t t = y * (uint32_t)(kMinimizerMul >> 32);
  asm("" : "+v"(t));
  return ((uint64_t)((uint32_t)(p >> 32) + t) << 32) | (uint32_t)p;
}
__device__ __forceinline__ uint64_t minimizer_hash(uint64_t y) { return y * kMinimizerMul; }

// h_S: xorshift 30, multiply, xorshift 31.
__device__ __forceinline__ uint64_t smer_hash(uint64_t v) {
  v ^= v >> 30;
  v *= kSmerMul;
  return v ^ (v >> 31);
}

// Bit address of hash index t (Section "Optimizations", bit-slicing; narrow
// slices fall back to a golden-ratio salt and the top 6 bits).
template <int H>
__device__ __forceinline__ uint32_t bit_address(uint64_t g, int t) {
  constexpr int W = 64 / H;
  if constexpr (W >= 6) {
    return (uint32_t)(g >> (t * W)) & 63u;
  } else {
    const uint64_t salt = kMinimizerMul * (2ull * (uint64_t)t + 1ull);
    return (uint32_t)((g * salt) >> 58);
  }
}

__device__ __forceinline__ uint32_t bit_address_rt(uint64_t g, int t, int H) {
  const int W = 64 / H;
  if (W >= 6) return (uint32_t)(g >> (t * W)) & 63u;
  const uint64_t salt = kMinimizerMul * (2ull * (uint64_t)t + 1ull);
  return (uint32_t)((g * salt) >> 58);
}

// Four ASCII bytes (little-endian in x, byte 0 = first base) -> 8 bits of
// codes (first base in bits 7:6) and a 4-bit valid mask (bit j = byte j).
// Code: ((c >> 1) ^ (c >> 2)) & 3 maps A/a C/c G/g T/t to 0 1 2 3; a byte is
// valid when its lower-case form equals the letter of its code.
__device__ __forceinline__ void encode4(uint32_t x, uint32_t &code8, uint32_t &valid4) {
  const uint32_t c = ((x >> 1) ^ (x >> 2)) & 0x03030303u;
  const uint32_t lower = x | 0x20202020u;
  const uint32_t expect = __builtin_amdgcn_perm(0u, 0x74676361u, c);  // 'a','c','g','t' by code
  const uint32_t diff = lower ^ expect;
  const uint32_t nz = (((diff & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | diff) & 0x80808080u;  // bit 7 per nonzero byte
  // gather bytes' bit 7 into bits 28..31, then invert
  valid4 = (~(((nz >> 7) * 0x10204080u) >> 28)) & 0xFu;
  // c0<<6 | c1<<4 | c2<<2 | c3, from the four byte-aligned codes
  code8 = (c * 0x40100401u) >> 24;
}

// Stage granules [0, ngran) of the bases starting at `base` (a multiple of
// 32).  Bytes at or beyond len read as 0, which is invalid.  brk, if not
// null, holds one bit per base (bit p%32 of word p/32) set where a record
// starts; it has ceil(len/32) words.
template <int WG>
__device__ __forceinline__ void stage_granules(const uint8_t *__restrict__ seq, uint64_t len, uint64_t base,
                                               const uint32_t *__restrict__ brk, bool aligned16, int ngran,
                                               uint32_t *__restrict__ s_codes, uint32_t *__restrict__ s_vb) {
  for (int g = threadIdx.x; g < ngran; g += WG) {
    const uint64_t p = base + 16ull * (uint64_t)g;
    uint32_t x[4];
    if (aligned16 && p + 16 <= len) {
      const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(seq + p));
      x[0] = v[0]; x[1] = v[1]; x[2] = v[2]; x[3] = v[3];
    } else {
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        uint32_t acc = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const uint64_t q = p + (uint64_t)(4 * w + b);
          const uint32_t byte = q < len ? (uint32_t)seq[q] : 0u;
          acc |= byte << (8 * b);
        }
        x[w] = acc;
      }
    }
    uint32_t code = 0, valid = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      uint32_t c8, v4;
      encode4(x[w], c8, v4);
      code = (code << 8) | c8;
      valid |= v4 << (4 * w);
    }
    uint32_t rs = 0;
    if (brk != nullptr && p < len) rs = (brk[p >> 5] >> (uint32_t)(p & 16u)) & 0xFFFFu;
    s_codes[g] = code;
    s_vb[g] = valid | (rs << 16);
  }
}

// 32-bit window of bases j .. j+15 of a lane's granule array a[] (first base
// most significant); j is a compile-time constant in the rolling kernels.
__device__ __forceinline__ uint32_t win32(const uint32_t *a, int j) {
  const int w = j >> 4, sh = (j & 15) * 2;
  return sh == 0 ? a[w] : __builtin_amdgcn_alignbit(a[w], a[w + 1], 32 - sh);
}

// Bit r = AND of x bits r .. r+n-1 (n >= 1, compile-time), bits past 63 read 0.
template <int N>
__device__ __forceinline__ uint64_t window_and(uint64_t x) {
  if constexpr (N <= 1) {
    return x;
  } else {
    constexpr int P = (N >= 32) ? 32 : (N >= 16) ? 16 : (N >= 8) ? 8 : (N >= 4) ? 4 : 2;
    uint64_t a = x;
#pragma unroll
    for (int d = 1; d < P; d <<= 1) a &= a >> d;
    return a & (a >> (N - P));
  }
}

// Bit r = OR of x bits r .. r+n-1 (n >= 0; n = 0 gives 0).
template <int N>
__device__ __forceinline__ uint64_t window_or(uint64_t x) {
  if constexpr (N <= 0) {
    return 0;
  } else if constexpr (N == 1) {
    return x;
  } else {
    constexpr int P = (N >= 32) ? 32 : (N >= 16) ? 16 : (N >= 8) ? 8 : (N >= 4) ? 4 : 2;
    uint64_t a = x;
#pragma unroll
    for (int d = 1; d < P; d <<= 1) a |= a >> d;
    return a | (a >> (N - P));
  }
}

// k-mer validity over a 64-base lane window: bit r set iff bases r .. r+K-1
// are valid and no record starts at r+1 .. r+K-1 (k-mers never span records).
template <int K>
__device__ __forceinline__ uint64_t kmer_valid_mask(uint64_t valid, uint64_t starts) {
  uint64_t kv = window_and<K>(valid);
  if (starts) kv &= ~window_or<K - 1>(starts >> 1);
  return kv;
}

// Agent-scope relaxed 64-bit atomic OR (the paper's atomicOr on shard words).
__device__ __forceinline__ void atomic_or64(uint64_t *p, uint64_t v) {
  __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Filter accesses of the two-pass insert.  The store pass's read-OR-writes
// of one shard race between workgroups on different XCDs, each with its own
// write-back L2.  Measured on the MI355X: with plain stores the racing dirty
// lines can reach memory after the repair walk's atomic ORs and overwrite
// them (bits went missing in filters that fit the caches), while stores that
// write through to the coherence point leave every word with one order of
// values, each a superset of the word at launch, which the repair walk then
// completes with agent-scope atomic ORs.  So the store pass writes each
// 16-byte half of its shard update with a system-coherent store (a volatile
// global access: global_store_dwordx4 with sc0 sc1).
typedef __attribute__((address_space(1))) volatile u32x4 coherent_u32x4;

__device__ __forceinline__ void store_pair_coherent(uint64_t *p, uint64_t a, uint64_t b) {
  u32x4 v;
  v[0] = (uint32_t)a;
  v[1] = (uint32_t)(a >> 32);
  v[2] = (uint32_t)b;
  v[3] = (uint32_t)(b >> 32);
  *(coherent_u32x4 *)p = v;
}

// Value of the other lane of an aligned lane pair (lane ^ 1), by a DPP quad
// permutation [1, 0, 3, 2]; every lane of the wave must be active.
__device__ __forceinline__ uint32_t pair_swap(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ uint64_t pair_swap64(uint64_t x) {
  return ((uint64_t)pair_swap((uint32_t)(x >> 32)) << 32) | pair_swap((uint32_t)x);
}

// Every workgroup of the insert, repair and query kernels starts with an
// agent-scope acquire (buffer_inv sc1: its XCD's L2 drops its lines), so
// that no load of the launch returns a copy cached before it.  Within a
// launch a plain load may then only miss bits that other workgroups are
// adding at the same time: the store pass loses them to a racing update and
// the repair walk restores them, and the repair walk, whose plain loads race
// only with its own atomic ORs, at worst repeats an OR.
__device__ __forceinline__ void acquire_device() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

}  // namespace sbf
