// Random shard-access and streaming-copy probes (include/sbf_probe.h).
#include "sbf_probe.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kBlock = 256;
constexpr int kIters = 64;

__device__ __forceinline__ uint64_t scramble(uint64_t x) {
  // MurmurHash3 64-bit finaliser: spreads thread/iteration ids over the buffer
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdull;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ull;
  x ^= x >> 33;
  return x;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void random_shards(uint64_t *__restrict__ buf, uint64_t shard_mask,
                                                        uint64_t seed, uint64_t *__restrict__ sink) {
  const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  uint64_t acc = 0;
  for (int i = 0; i < kIters; ++i) {
    const uint64_t h = scramble(tid * 0x9E3779B97F4A7C15ull + (uint64_t)i + seed);
    uint64_t *p = buf + 4ull * (h & shard_mask);
    const uint64_t bit = 1ull << (h >> 58);
    if constexpr (MODE == SBF_PROBE_READ32) {
      const uint4 *q = reinterpret_cast<const uint4 *>(p);
      const uint4 a = q[0], b = q[1];
      acc ^= (uint64_t)(a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w);
    } else if constexpr (MODE == SBF_PROBE_RMW32) {
      uint4 *q = reinterpret_cast<uint4 *>(p);
      uint4 a = q[0], b = q[1];
      a.x |= (uint32_t)bit;
      b.w |= (uint32_t)(bit >> 32);
      q[0] = a;
      q[1] = b;
    } else if constexpr (MODE == SBF_PROBE_ATOMIC4) {
#pragma unroll
      for (int w = 0; w < 4; ++w) __hip_atomic_fetch_or(p + w, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __hip_atomic_fetch_or(p, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (MODE == SBF_PROBE_READ32 && acc == 0x5bd1e995ull) sink[0] = acc;  // keeps the loads
}

__global__ __launch_bounds__(kBlock) void stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                      uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock)
    dst[i] = src[i];
}

hipError_t launch(int mode, uint64_t *buf, uint64_t bytes, uint64_t ops, uint64_t seed, uint64_t *sink) {
  if (mode == SBF_PROBE_COPY) {
    const uint64_t n = bytes / 2 / 16;
    hipLaunchKernelGGL(stream_copy, dim3(8192), dim3(kBlock), 0, 0, (const uint4 *)buf,
                       (uint4 *)(buf + bytes / 2 / 8), n);
    return hipGetLastError();
  }
  const uint64_t mask = bytes / 32 - 1;
  const unsigned grid = (unsigned)(ops / ((uint64_t)kBlock * kIters));
  switch (mode) {
    case SBF_PROBE_READ32:
      hipLaunchKernelGGL(random_shards<SBF_PROBE_READ32>, dim3(grid), dim3(kBlock), 0, 0, buf, mask, seed, sink);
      break;
    case SBF_PROBE_RMW32:
      hipLaunchKernelGGL(random_shards<SBF_PROBE_RMW32>, dim3(grid), dim3(kBlock), 0, 0, buf, mask, seed, sink);
      break;
    case SBF_PROBE_ATOMIC4:
      hipLaunchKernelGGL(random_shards<SBF_PROBE_ATOMIC4>, dim3(grid), dim3(kBlock), 0, 0, buf, mask, seed, sink);
      break;
    default:
      hipLaunchKernelGGL(random_shards<SBF_PROBE_ATOMIC1>, dim3(grid), dim3(kBlock), 0, 0, buf, mask, seed, sink);
      break;
  }
  return hipGetLastError();
}

}  // namespace

extern "C" int sbf_probe_random_access(uint64_t bytes, int mode, uint64_t ops, double *per_second, double *ms) {
  if (!per_second || !ms || mode < SBF_PROBE_READ32 || mode > SBF_PROBE_COPY) return -1;
  if (bytes < (1ull << 16) || bytes > (1ull << 36) || (bytes & (bytes - 1))) return -1;
  const uint64_t chunk = (uint64_t)kBlock * kIters;
  if (ops < (1ull << 20)) ops = 1ull << 20;
  ops = (ops + chunk - 1) / chunk * chunk;
  if (ops / chunk > 0x7fffffffull) return -1;
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
      launch(mode, buf, bytes, ops, 1, sink) != hipSuccess || hipEventRecord(a, 0) != hipSuccess) {
    rc = -3;
  } else {
    for (int r = 0; r < 3 && rc == 0; ++r)
      if (launch(mode, buf, bytes, ops, 7 + r, sink) != hipSuccess) rc = -3;
    if (rc == 0 && (hipEventRecord(b, 0) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                    hipEventElapsedTime(&t, a, b) != hipSuccess))
      rc = -3;
  }
  if (rc == 0) {
    *ms = t / 3.0;
    const double work = mode == SBF_PROBE_COPY ? (double)(bytes / 2 / 16 * 16) * 2.0 : (double)ops;
    *per_second = work / (*ms * 1e-3);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(sink);
  (void)hipFree(buf);
  return rc;
}
