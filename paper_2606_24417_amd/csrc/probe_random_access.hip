// Random shard-access, streaming-copy and integer VALU probes (include/sbf_probe.h).
#include "sbf_probe.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint64_t scramble(uint64_t x) {
  // MurmurHash3 64-bit finaliser: spreads thread/iteration ids over the buffer
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

// Random shard accesses with many memory operations in flight per lane: each
// lane draws `D` independent shard indices, issues every load of the batch
// (D shards of SB bytes = D * SB/16 16-byte loads) before it uses any of them,
// then consumes them (read: fold into a checksum; read-modify-write: OR one
// bit and store the shard back; atomics: fire-and-forget 64-bit atomic ORs).
// The grid is num_CUs * wgs_per_cu workgroups that each run `batches` batches,
// so occupancy (waves per SIMD) is a sweep parameter of the caller.  The
// register budget allows two waves per SIMD, so that the compiler keeps every
// load of a batch in its own registers instead of reusing them (which would
// serialise the loads on waits).
//
// With COOP (the _LINE modes) the SB/16 consecutive lanes of a group share
// each shard: lane c of the group loads and stores 16-byte piece c, so one
// wave instruction covers 64 * 16 / SB whole shards (the access pattern of
// the wide-shard kernels, which move a super-k-mer's line with SB/16 lanes).
// Store of a 16-byte chunk that writes through to the device's coherence
// point (a volatile global access: global_store_dwordx4 with sc0 sc1), the
// store the filter's insert kernels use for their racing read-modify-writes.
typedef uint32_t probe_u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) volatile probe_u32x4 probe_coherent_u32x4;
__device__ __forceinline__ void store_coherent(uint4 *q, const uint4 &v) {
  probe_u32x4 x;
  x[0] = v.x;
  x[1] = v.y;
  x[2] = v.z;
  x[3] = v.w;
  *(probe_coherent_u32x4 *)q = x;
}

template <int MODE, int SB, int D, bool COOP = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void random_shards(uint64_t *__restrict__ buf, uint64_t shard_mask,
                                                        uint64_t seed, uint32_t batches,
                                                        uint64_t *__restrict__ sink) {
  constexpr int P = COOP ? SB / 16 : 1;  // lanes per shard
  constexpr int C = SB / 16 / P;         // 16-byte chunks per lane and shard
  const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t nthreads = (uint64_t)gridDim.x * kBlock;
  const uint64_t group = tid / P, ngroups = nthreads / P;
  const int piece = (int)(tid % P);
  uint64_t acc = 0;
  for (uint32_t it = 0; it < batches; ++it) {
    uint64_t idx[D];
    uint64_t bit[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const uint64_t op = ((uint64_t)it * ngroups + group) * D + (uint64_t)d;
      const uint64_t h = scramble(op * 0x9E3779B97F4A7C15ull + seed);
      idx[d] = h & shard_mask;
      bit[d] = 1ull << (h >> 58);
    }
    if constexpr (MODE == SBF_PROBE_READ || MODE == SBF_PROBE_RMW || MODE == SBF_PROBE_READ_LINE ||
                  MODE == SBF_PROBE_RMW_LINE || MODE == SBF_PROBE_RMW_COHERENT || MODE == SBF_PROBE_RMW_LINE_COHERENT) {
      uint4 v[D][C];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const uint4 *q = reinterpret_cast<const uint4 *>(buf + idx[d] * (SB / 8)) + piece;
#pragma unroll
        for (int c = 0; c < C; ++c) v[d][c] = q[c];
      }
      // Every load of the batch is issued before the first wait: the barrier
      // keeps the machine scheduler from moving uses up between the loads, and
      // the empty asm statements (which stay below the barrier) keep the IR
      // optimiser from folding loaded values early.
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int d = 0; d < D; ++d)
#pragma unroll
        for (int c = 0; c < C; ++c) asm volatile("" : "+v"(v[d][c].x), "+v"(v[d][c].y), "+v"(v[d][c].z), "+v"(v[d][c].w));
      if constexpr (MODE == SBF_PROBE_READ || MODE == SBF_PROBE_READ_LINE) {
#pragma unroll
        for (int d = 0; d < D; ++d)
#pragma unroll
          for (int c = 0; c < C; ++c) acc ^= (uint64_t)(v[d][c].x ^ v[d][c].y ^ v[d][c].z ^ v[d][c].w) + (uint64_t)c;
      } else {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          v[d][0].x |= (uint32_t)bit[d];
          v[d][C - 1].w |= (uint32_t)(bit[d] >> 32);
          uint4 *q = reinterpret_cast<uint4 *>(buf + idx[d] * (SB / 8)) + piece;
#pragma unroll
          for (int c = 0; c < C; ++c) {
            if constexpr (MODE == SBF_PROBE_RMW_COHERENT || MODE == SBF_PROBE_RMW_LINE_COHERENT)
              store_coherent(q + c, v[d][c]);
            else
              q[c] = v[d][c];
          }
        }
      }
    } else {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        uint64_t *p = buf + idx[d] * (SB / 8);
        if constexpr (MODE == SBF_PROBE_ATOMIC4) {
#pragma unroll
          for (int w = 0; w < 4; ++w) __hip_atomic_fetch_or(p + w, bit[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
          __hip_atomic_fetch_or(p, bit[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  }
  if ((MODE == SBF_PROBE_READ || MODE == SBF_PROBE_READ_LINE) && acc == 0x5bd1e995ull) sink[0] = acc;  // keeps the loads
}

__global__ __launch_bounds__(kBlock) void stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                      uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock)
    dst[i] = src[i];
}

// In-flight depths compiled per shard size: at most 32 loads of 16 bytes
// (128 registers of data) per lane.
bool depth_supported(uint32_t sb, uint32_t d) {
  switch (sb) {
    case 32: return d == 1 || d == 4 || d == 8 || d == 16;
    case 64: return d == 1 || d == 4 || d == 8;
    case 128: return d == 1 || d == 2 || d == 4;
    default: return false;
  }
}

template <int MODE>
hipError_t launch_random(uint64_t *buf, uint64_t bytes, uint32_t sb, uint32_t d, unsigned grid, uint32_t batches,
                         uint64_t seed, uint64_t *sink) {
  const uint64_t mask = bytes / sb - 1;
  constexpr bool coop =
      MODE == SBF_PROBE_READ_LINE || MODE == SBF_PROBE_RMW_LINE || MODE == SBF_PROBE_RMW_LINE_COHERENT;
#define SBF_PROBE_CASE(SB_, D_)                                                                              \
  if (sb == SB_ && d == D_) {                                                                                \
    hipLaunchKernelGGL((random_shards<MODE, SB_, D_, coop>), dim3(grid), dim3(kBlock), 0, 0, buf, mask, seed,    \
                       batches, sink);                                                                       \
    return hipGetLastError();                                                                                \
  }
  SBF_PROBE_CASE(32, 1) SBF_PROBE_CASE(32, 4) SBF_PROBE_CASE(32, 8) SBF_PROBE_CASE(32, 16)
  SBF_PROBE_CASE(64, 1) SBF_PROBE_CASE(64, 4) SBF_PROBE_CASE(64, 8)
  SBF_PROBE_CASE(128, 1) SBF_PROBE_CASE(128, 2) SBF_PROBE_CASE(128, 4)
#undef SBF_PROBE_CASE
  return hipErrorInvalidValue;
}

hipError_t launch(int mode, uint64_t *buf, uint64_t bytes, uint32_t sb, uint32_t d, unsigned grid, uint32_t batches,
                  uint64_t seed, uint64_t *sink) {
  if (mode == SBF_PROBE_COPY) {
    const uint64_t n = bytes / 2 / 16;
    hipLaunchKernelGGL(stream_copy, dim3(8192), dim3(kBlock), 0, 0, (const uint4 *)buf,
                       (uint4 *)(buf + bytes / 2 / 8), n);
    return hipGetLastError();
  }
  switch (mode) {
    case SBF_PROBE_READ: return launch_random<SBF_PROBE_READ>(buf, bytes, sb, d, grid, batches, seed, sink);
    case SBF_PROBE_RMW: return launch_random<SBF_PROBE_RMW>(buf, bytes, sb, d, grid, batches, seed, sink);
    case SBF_PROBE_ATOMIC4: return launch_random<SBF_PROBE_ATOMIC4>(buf, bytes, sb, d, grid, batches, seed, sink);
    case SBF_PROBE_READ_LINE: return launch_random<SBF_PROBE_READ_LINE>(buf, bytes, sb, d, grid, batches, seed, sink);
    case SBF_PROBE_RMW_LINE: return launch_random<SBF_PROBE_RMW_LINE>(buf, bytes, sb, d, grid, batches, seed, sink);
    case SBF_PROBE_RMW_COHERENT:
      return launch_random<SBF_PROBE_RMW_COHERENT>(buf, bytes, sb, d, grid, batches, seed, sink);
    case SBF_PROBE_RMW_LINE_COHERENT:
      return launch_random<SBF_PROBE_RMW_LINE_COHERENT>(buf, bytes, sb, d, grid, batches, seed, sink);
    default: return launch_random<SBF_PROBE_ATOMIC1>(buf, bytes, sb, d, grid, batches, seed, sink);
  }
}

// Integer VALU issue-rate probe: eight independent chains of one instruction
// kind per lane, written as inline assembly so that the compiler neither
// folds nor substitutes them.
constexpr int kValuBlocks = 2048;   // 8192 waves: eight per SIMD on 256 CUs
constexpr uint32_t kValuIters = 32768;

template <int OP>
__global__ __launch_bounds__(kBlock) void valu_chains(uint32_t iters, uint64_t *__restrict__ sink) {
  uint32_t a[8];
  uint64_t d[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = threadIdx.x * (uint32_t)(2 * j + 1) + blockIdx.x;
    d[j] = ((uint64_t)a[j] << 32) | (a[j] ^ 0x5bd1e995u);
  }
  const uint32_t c = 0x9E3779B9u + (blockIdx.x & 1u);
  const uint32_t sh = 3u + (threadIdx.x & 1u);
  uint64_t q[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // scalar results, one register pair per chain
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if constexpr (OP == SBF_PROBE_VALU_ADD32) {
        asm volatile("v_add_u32_e32 %0, %1, %0" : "+v"(a[j]) : "v"(c));
      } else if constexpr (OP == SBF_PROBE_VALU_MUL32) {
        asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[j]) : "v"(c));
      } else if constexpr (OP == SBF_PROBE_VALU_MAD64) {
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(d[j]), "=s"(q[j]) : "v"(a[j]), "v"(c));
      } else if constexpr (OP == SBF_PROBE_VALU_SHL64) {
        asm volatile("v_lshlrev_b64 %0, %1, %0" : "+v"(d[j]) : "v"(sh));
      } else if constexpr (OP == SBF_PROBE_VALU_BITOP3) {
        asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[j]) : "v"(c), "v"(sh));
      } else {
        asm volatile("v_cmp_lt_u64_e64 %0, %1, %2" : "=s"(q[j]) : "v"(d[j]), "v"(d[(j + 1) & 7]));
      }
    }
  }
  uint64_t x = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) x ^= d[j] ^ a[j] ^ q[j];
  if (x == 0x5bd1e9955bd1e995ull) sink[0] = x;  // keeps the chains' results live
}

hipError_t launch_valu(int op, uint64_t *sink) {
  const dim3 grid(kValuBlocks), block(kBlock);
  switch (op) {
    case SBF_PROBE_VALU_ADD32: hipLaunchKernelGGL(valu_chains<SBF_PROBE_VALU_ADD32>, grid, block, 0, 0, kValuIters, sink); break;
    case SBF_PROBE_VALU_MUL32: hipLaunchKernelGGL(valu_chains<SBF_PROBE_VALU_MUL32>, grid, block, 0, 0, kValuIters, sink); break;
    case SBF_PROBE_VALU_MAD64: hipLaunchKernelGGL(valu_chains<SBF_PROBE_VALU_MAD64>, grid, block, 0, 0, kValuIters, sink); break;
    case SBF_PROBE_VALU_SHL64: hipLaunchKernelGGL(valu_chains<SBF_PROBE_VALU_SHL64>, grid, block, 0, 0, kValuIters, sink); break;
    case SBF_PROBE_VALU_BITOP3: hipLaunchKernelGGL(valu_chains<SBF_PROBE_VALU_BITOP3>, grid, block, 0, 0, kValuIters, sink); break;
    default: hipLaunchKernelGGL(valu_chains<SBF_PROBE_VALU_CMP64>, grid, block, 0, 0, kValuIters, sink); break;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" int sbf_probe_valu(int op, double *wave_instr_per_second, double *ms) {
  if (!wave_instr_per_second || !ms || op < SBF_PROBE_VALU_ADD32 || op > SBF_PROBE_VALU_CMP64) return -1;
  uint64_t *sink = nullptr;
  if (hipMalloc((void **)&sink, 64) != hipSuccess) return -2;
  int rc = 0;
  hipEvent_t a = nullptr, b = nullptr;
  float t = 0.f;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess || launch_valu(op, sink) != hipSuccess ||
      hipEventRecord(a, 0) != hipSuccess) {
    rc = -3;
  } else {
    for (int r = 0; r < 3 && rc == 0; ++r)
      if (launch_valu(op, sink) != hipSuccess) rc = -3;
    if (rc == 0 && (hipEventRecord(b, 0) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                    hipEventElapsedTime(&t, a, b) != hipSuccess))
      rc = -3;
  }
  if (rc == 0) {
    *ms = t / 3.0;
    const double waves = (double)kValuBlocks * (kBlock / 64);
    *wave_instr_per_second = waves * 8.0 * kValuIters / (*ms * 1e-3);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(sink);
  return rc;
}

extern "C" int sbf_probe_random_access(uint64_t bytes, int mode, uint32_t shard_bytes, uint32_t inflight,
                                       uint32_t wgs_per_cu, uint64_t ops, double *per_second, double *ms) {
  if (!per_second || !ms || mode < SBF_PROBE_READ || mode > SBF_PROBE_RMW_LINE_COHERENT) return -1;
  if (bytes < (1ull << 16) || bytes > (1ull << 36) || (bytes & (bytes - 1))) return -1;
  if (mode != SBF_PROBE_COPY && (!depth_supported(shard_bytes, inflight) || wgs_per_cu < 1 || wgs_per_cu > 16))
    return -1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return -3;
  const unsigned grid = (unsigned)cus * wgs_per_cu;
  // shard operations per batch of the grid (a shard per SB/16 lanes in the _LINE modes)
  const uint64_t lanes_per_shard =
      (mode == SBF_PROBE_READ_LINE || mode == SBF_PROBE_RMW_LINE || mode == SBF_PROBE_RMW_LINE_COHERENT)
          ? (uint64_t)shard_bytes / 16
          : 1;
  const uint64_t per_batch = (uint64_t)grid * kBlock * (mode == SBF_PROBE_COPY ? 1 : inflight) / lanes_per_shard;
  if (ops < (1ull << 20)) ops = 1ull << 20;
  const uint64_t nb = (ops + per_batch - 1) / per_batch;
  if (nb > 0xffffffffull) return -1;
  const uint32_t batches = (uint32_t)nb;
  uint64_t *buf = nullptr, *sink = nullptr;
  if (hipMalloc((void **)&buf, bytes) != hipSuccess) return -2;
  if (hipMalloc((void **)&sink, 64) != hipSuccess) {
    (void)hipFree(buf);
    return -2;
  }
  int rc = 0;
  hipEvent_t a = nullptr, b = nullptr;
  float t = 0.f;
  if (hipMemset(buf, 0, bytes) != hipSuccess || hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess ||
      launch(mode, buf, bytes, shard_bytes, inflight, grid, batches, 1, sink) != hipSuccess ||
      hipEventRecord(a, 0) != hipSuccess) {
    rc = -3;
  } else {
    for (int r = 0; r < 3 && rc == 0; ++r)
      if (launch(mode, buf, bytes, shard_bytes, inflight, grid, batches, 7 + r, sink) != hipSuccess) rc = -3;
    if (rc == 0 && (hipEventRecord(b, 0) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                    hipEventElapsedTime(&t, a, b) != hipSuccess))
      rc = -3;
  }
  if (rc == 0) {
    *ms = t / 3.0;
    const double work =
        mode == SBF_PROBE_COPY ? (double)(bytes / 2 / 16 * 16) * 2.0 : (double)per_batch * (double)batches;
    *per_second = work / (*ms * 1e-3);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(sink);
  (void)hipFree(buf);
  return rc;
}
