// Host runtime behind the C ABI of include/sbf.h: filter objects, parameter
// validation, staging of host input, record-start scratch per stream, and
// dispatch to the rolling or generic kernels.
#include "sbf.h"
#include "sbf_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using sbf::Geometry;
using sbf::SeqArgs;

namespace {

thread_local int g_err = SBF_OK;
thread_local std::string g_msg;

int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int set_error(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = code;
  g_msg = buf;
  return code;
}

int ok() {
  g_err = SBF_OK;
  g_msg.clear();
  return SBF_OK;
}

}  // namespace

int sbf::record_error(int code, const char *msg) {
  g_err = code;
  g_msg = msg ? msg : "";
  return code;
}

namespace {

int hip_error(hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory) return set_error(SBF_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
  return set_error(SBF_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define SBF_HIP(call, what)                  \
  do {                                       \
    hipError_t e_ = (call);                  \
    if (e_ != hipSuccess) return hip_error(e_, what); \
  } while (0)

constexpr uint64_t kMaxBits = 1ull << 40;
constexpr uint64_t kDefaultStaging = 64ull << 20;

struct Scratch {
  void *ptr = nullptr;
  size_t bytes = 0;
};

// Pinned host memory (hipHostMalloc), so that copies from and to it run
// asynchronously with the kernels.
struct Pinned {
  void *ptr = nullptr;
  size_t bytes = 0;
};

// One stage of the host pipeline: a stream with the device and pinned host
// buffers of one chunk.  Two stages alternate, so that the host-side copy or
// answer unpacking of one chunk overlaps the transfers and kernel of the
// other.
struct PipeSlot {
  hipStream_t stream = nullptr;
  hipEvent_t kernel_done = nullptr;  // the stage's last kernel has finished
  hipEvent_t done = nullptr;         // the stage's last chunk has finished, answers included
  Scratch d_seq, d_out, d_off;
  Pinned h_seq, h_out, h_off;
  uint8_t *flush_dst = nullptr;  // caller buffer for the answers waiting in h_out
  uint64_t flush_len = 0;        // answers (bytes in the caller's buffer)
  bool flush_packed = false;     // h_out holds them as bits
  bool pending = false;
};
constexpr int kPipeSlots = 2;

}  // namespace

struct sbf_filter {
  Geometry g{};
  uint64_t *words = nullptr;  // device, 4 * nshards
  hipStream_t stream = nullptr;
  int device = 0;
  int variant = SBF_VARIANT_AUTO;
  int insert_mode = SBF_INSERT_TWO_PASS;
  int query_mode = SBF_QUERY_LANE;
  // 0: one workgroup per tile; n: persistent grid of n workgroups per CU
  // (4 measured best for both kernels on MI355X)
  uint32_t insert_wgs_per_cu = 4;
  uint32_t query_wgs_per_cu = 4;
  // k-mers per lane of the insert and query tiles (0: the family's default)
  uint32_t insert_lane_len = 0;
  uint32_t query_lane_len = 0;
  int num_cus = 1;
  uint64_t staging = kDefaultStaging;
  // host entry points: chunk pipeline (created on first use)
  PipeSlot pipe[kPipeSlots];
  // record-start bits, one buffer per stream
  std::mutex mu;
  std::unordered_map<hipStream_t, Scratch> starts;
  // work-queue counters of persistent launches, one set per stream
  std::unordered_map<hipStream_t, Scratch> queues;
};

namespace {

uint64_t next_pow2(uint64_t x) {
  uint64_t n = 1;
  while (n < x) n <<= 1;
  return n;
}

// Kernel family a filter's launches use: the 4-word lane kernels, the
// wide-shard kernels (any of 4, 8, 16 words), the run-time parameter
// super-k-mer kernels or the generic kernels.
enum Family { kGenericFamily, kLaneFamily, kWideFamily, kParamFamily };

Family family(const sbf_filter *f) {
  switch (f->variant) {
    case SBF_VARIANT_GENERIC:
      return kGenericFamily;
    case SBF_VARIANT_WIDE:
      return sbf::wide_supported(f->g) ? kWideFamily : kGenericFamily;
    case SBF_VARIANT_PARAM:
      return sbf::param_supported(f->g) ? kParamFamily : kGenericFamily;
    default:  // AUTO and ROLLING: the fastest super-k-mer kernels for the filter
      if (sbf::rolling_supported(f->g)) return kLaneFamily;
      if (sbf::wide_supported(f->g)) return kWideFamily;
      if (sbf::param_supported(f->g)) return kParamFamily;
      return kGenericFamily;
  }
}

bool use_rolling(const sbf_filter *f) { return family(f) != kGenericFamily; }

// Compiled k-mers per lane of each family (0 stands for the default).
bool lane_len_ok(const sbf_filter *f, uint32_t n, bool insert) {
  if (n == 0) return true;
  switch (family(f)) {
    case kLaneFamily: {
      const Geometry &g = f->g;
      if (!(g.k == 31 && g.s == 28 && g.m == 16 && g.H == 4)) return false;
      return insert ? (n == 32 || n == 64) : (n == 32 || n == 48);
    }
    case kWideFamily:
      return n == 16 || n == 32;
    case kParamFamily:
      return n == 8 || n == 16;
    default:
      return false;
  }
}

uint32_t lane_len_effective(const sbf_filter *f, uint32_t n, bool insert) {
  if (n) return n;
  switch (family(f)) {
    case kLaneFamily: {
      const Geometry &g = f->g;
      const bool variants = g.k == 31 && g.s == 28 && g.m == 16 && g.H == 4;
      return insert ? (variants ? 64 : 32) : 48;
    }
    case kWideFamily: return 16;
    case kParamFamily: return 8;
    default: return 0;
  }
}

// stream-ordered entry points run on the caller's stream; NULL is HIP's null stream
hipStream_t pick(const sbf_filter *, void *stream) { return (hipStream_t)stream; }

int grow(Scratch &s, size_t bytes, const char *what) {
  if (s.bytes >= bytes) return SBF_OK;
  if (s.ptr) {
    hipError_t e = hipFree(s.ptr);
    s.ptr = nullptr;
    s.bytes = 0;
    if (e != hipSuccess) return hip_error(e, what);
  }
  size_t want = std::max<size_t>(bytes, 4096);
  hipError_t e = hipMalloc(&s.ptr, want);
  if (e != hipSuccess) {
    s.ptr = nullptr;
    return hip_error(e, what);
  }
  s.bytes = want;
  return SBF_OK;
}

// Launch shape for a pass on stream st (queue counters allocated on first use
// of a stream), unless the caller supplies its own (graph capture).
int launch_shape(sbf_filter *f, uint32_t wgs_per_cu, hipStream_t st, sbf::LaunchShape &ls) {
  ls.queue = nullptr;
  ls.persistent_wgs = 0;
  if (wgs_per_cu == 0) return SBF_OK;
  Scratch *s;
  {
    std::lock_guard<std::mutex> lk(f->mu);
    s = &f->queues[st];
  }
  int rc = grow(*s, 256, "work-queue counters");
  if (rc) return rc;
  ls.queue = (uint32_t *)s->ptr;
  ls.persistent_wgs = wgs_per_cu * (uint32_t)f->num_cus;
  return SBF_OK;
}

}  // namespace

int sbf::prepare_stream(sbf_filter *f, hipStream_t st) {
  sbf::LaunchShape ls;
  int rc = launch_shape(f, f->query_wgs_per_cu, st, ls);
  if (rc == SBF_OK) rc = launch_shape(f, f->insert_wgs_per_cu, st, ls);
  return rc;
}

void sbf::release_stream(sbf_filter *f, hipStream_t st) {
  std::lock_guard<std::mutex> lk(f->mu);
  for (auto *m : {&f->queues, &f->starts}) {
    auto it = m->find(st);
    if (it == m->end()) continue;
    if (it->second.ptr) (void)hipFree(it->second.ptr);
    m->erase(it);
  }
}

namespace {

int run_insert(sbf_filter *f, const SeqArgs &a, hipStream_t st, const sbf::LaunchShape *given = nullptr) {
  const int mode = f->insert_mode == SBF_INSERT_ATOMIC ? sbf::kInsertAtomicMode : sbf::kInsertTwoPassMode;
  hipError_t e;
  if (use_rolling(f)) {
    sbf::LaunchShape ls;
    if (given) {
      ls = *given;
      ls.persistent_wgs = f->insert_wgs_per_cu * (uint32_t)f->num_cus;
    } else {
      int rc = launch_shape(f, f->insert_wgs_per_cu, st, ls);
      if (rc) return rc;
    }
    ls.insert_lane_len = f->insert_lane_len;
    ls.query_lane_len = f->query_lane_len;
    switch (family(f)) {
      case kWideFamily: e = sbf::launch_insert_wide(f->g, f->words, a, mode, ls, st); break;
      case kParamFamily: e = sbf::launch_insert_param(f->g, f->words, a, mode, ls, st); break;
      default: e = sbf::launch_insert_rolling(f->g, f->words, a, mode, ls, st); break;
    }
  } else {
    e = sbf::launch_insert_generic(f->g, f->words, a, st);
  }
  if (e != hipSuccess) return hip_error(e, "insert kernel launch");
  return SBF_OK;
}

int query_kernel_mode(const sbf_filter *f) {
  return f->query_mode == SBF_QUERY_DIRECT   ? sbf::kQueryDirectMode
         : f->query_mode == SBF_QUERY_LEADER ? sbf::kQueryLeaderMode
                                             : sbf::kQueryLaneMode;
}

int run_query(sbf_filter *f, const SeqArgs &a, hipStream_t st, const sbf::LaunchShape *given = nullptr) {
  const int mode = query_kernel_mode(f);
  hipError_t e;
  if (use_rolling(f)) {
    sbf::LaunchShape ls;
    if (given) {
      ls = *given;
      ls.persistent_wgs = f->query_wgs_per_cu * (uint32_t)f->num_cus;
    } else {
      int rc = launch_shape(f, f->query_wgs_per_cu, st, ls);
      if (rc) return rc;
    }
    ls.insert_lane_len = f->insert_lane_len;
    ls.query_lane_len = f->query_lane_len;
    switch (family(f)) {
      case kWideFamily: e = sbf::launch_query_wide(f->g, f->words, a, ls, st); break;
      case kParamFamily: e = sbf::launch_query_param(f->g, f->words, a, ls, st); break;
      default: e = sbf::launch_query_rolling(f->g, f->words, a, mode, ls, st); break;
    }
  } else {
    e = sbf::launch_query_generic(f->g, f->words, a, st);
  }
  if (e != hipSuccess) return hip_error(e, "query kernel launch");
  return SBF_OK;
}

// record-start bits for a batch on stream st; returns null when not needed
int record_starts(sbf_filter *f, const uint64_t *d_off, uint64_t nrec, uint64_t len, hipStream_t st,
                  const uint32_t **out) {
  *out = nullptr;
  if (nrec < 2 || len == 0) return SBF_OK;
  const uint64_t nw = (len + 31) / 32;
  Scratch *s;
  {
    std::lock_guard<std::mutex> lk(f->mu);
    s = &f->starts[st];
  }
  if (s->bytes < nw * 4) {
    // the old buffer may still be in use by earlier work on this stream
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_error(e, "record-start scratch");
    int rc = grow(*s, nw * 4, "record-start scratch");
    if (rc) return rc;
  }
  uint32_t *w = (uint32_t *)s->ptr;
  hipError_t e = sbf::launch_fill_u32(w, nw, 0u, st);
  if (e == hipSuccess) e = sbf::launch_mark_record_starts(d_off, nrec, len, w, st);
  if (e != hipSuccess) return hip_error(e, "record-start marking");
  *out = w;
  return SBF_OK;
}

int check_filter(const sbf_filter *f) {
  if (!f) return set_error(SBF_E_INVAL, "filter is NULL");
  return SBF_OK;
}

// Scratch of the allocation-free query (sbf_query_batch_dev_noalloc): the
// work-queue counters of a persistent launch, then the record-start bits of
// up to kNoAllocMaxBases bases.  A file-scope device array, one copy per GPU
// for the life of the process; every call on a GPU shares it.  Host code uses
// the address hipGetSymbolAddress returns for the current device (kept per
// device in g_noalloc), never the array's name.
constexpr uint64_t kNoAllocQueueWords = 64;  // 256 bytes: the counters, at the array's 256-byte alignment
constexpr uint64_t kNoAllocStartWords = 1ull << 21;
constexpr uint64_t kNoAllocMaxBases = kNoAllocStartWords * 32;  // 2^26 bases, 8 MiB of scratch
__device__ __align__(256) uint32_t scratch[kNoAllocQueueWords + kNoAllocStartWords];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
uint32_t *g_noalloc[kMaxDevices];

// Device address of `scratch` on device dev, which must be current; looked up
// once per device.
int noalloc_scratch(int dev, uint32_t **out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(SBF_E_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_error(e, "address of the allocation-free scratch");
    if (p == nullptr) return set_error(SBF_E_DEVICE, "address of the allocation-free scratch is NULL");
    g_noalloc[dev] = (uint32_t *)p;
  }
  *out = g_noalloc[dev];
  return SBF_OK;
}

int set_device(const sbf_filter *f) {
  SBF_HIP(hipSetDevice(f->device), "hipSetDevice");
  return SBF_OK;
}

int grow_pinned(Pinned &p, size_t bytes, const char *what) {
  if (p.bytes >= bytes) return SBF_OK;
  if (p.ptr) {
    hipError_t e = hipHostFree(p.ptr);
    p.ptr = nullptr;
    p.bytes = 0;
    if (e != hipSuccess) return hip_error(e, what);
  }
  size_t want = std::max<size_t>(bytes, 4096);
  hipError_t e = hipHostMalloc(&p.ptr, want, hipHostMallocDefault);
  if (e != hipSuccess) {
    p.ptr = nullptr;
    return hip_error(e, what);
  }
  p.bytes = want;
  return SBF_OK;
}

// True when p lies in page-locked host memory the device can copy from
// asynchronously (hipHostMalloc, torch pin_memory).
bool host_pinned(const void *p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();  // pageable memory: clear the recorded error
    return false;
  }
  return at.type == hipMemoryTypeHost;
}

int ensure_pipe(sbf_filter *f) {
  for (PipeSlot &ps : f->pipe) {
    hipError_t e = hipSuccess;
    if (!ps.stream) e = hipStreamCreateWithFlags(&ps.stream, hipStreamNonBlocking);
    if (e == hipSuccess && !ps.kernel_done) e = hipEventCreateWithFlags(&ps.kernel_done, hipEventDisableTiming);
    if (e == hipSuccess && !ps.done) e = hipEventCreateWithFlags(&ps.done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_error(e, "host pipeline set-up");
  }
  return SBF_OK;
}

// Host copy between pageable and pinned memory, split over up to 8 threads
// for large buffers (one thread copies at well under the host link's rate).
void host_copy(void *dst, const void *src, size_t n) {
  constexpr size_t kPerThread = 8ull << 20;
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t parts = std::min<size_t>(std::min<size_t>(8, hw), n / kPerThread);
  if (parts < 2) {
    memcpy(dst, src, n);
    return;
  }
  std::vector<std::thread> th;
  const size_t step = (n / parts + 4095) & ~size_t(4095);
  try {
    for (size_t i = 1; i < parts && i * step < n; ++i) {
      const size_t a = i * step, b = std::min(n, a + step);
      th.emplace_back([=] { memcpy((char *)dst + a, (const char *)src + a, b - a); });
    }
  } catch (...) {
    // no thread available: the remaining parts are copied below
  }
  const size_t done_by_threads = th.size();
  memcpy(dst, src, std::min(n, step));
  for (size_t i = done_by_threads + 1; i < parts && i * step < n; ++i) {
    const size_t a = i * step, b = std::min(n, a + step);
    memcpy((char *)dst + a, (const char *)src + a, b - a);
  }
  for (auto &t : th) t.join();
}

// Byte b of table entry x is bit b of x: one answer byte per answer bit.
struct BitBytes {
  uint64_t v[256];
  BitBytes() {
    for (int x = 0; x < 256; ++x) {
      uint64_t e = 0;
      for (int b = 0; b < 8; ++b) e |= (uint64_t)((x >> b) & 1) << (8 * b);
      v[x] = e;
    }
  }
};
const BitBytes kBitBytes;

void unpack_range(uint8_t *dst, const uint8_t *bits, size_t a, size_t b) {
  // a is a multiple of 8
  size_t i = a;
  for (; i + 8 <= b; i += 8) memcpy(dst + i, &kBitBytes.v[bits[i / 8]], 8);
  for (; i < b; ++i) dst[i] = (uint8_t)((bits[i / 8] >> (i % 8)) & 1u);
}

// Answer bytes dst[0, n) from answer bits (bit i%8 of bits[i/8]), split over
// up to 8 host threads for large chunks like host_copy.
void unpack_bits(uint8_t *dst, const uint8_t *bits, size_t n) {
  constexpr size_t kPerThread = 8ull << 20;
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t parts = std::min<size_t>(std::min<size_t>(8, hw), n / kPerThread);
  if (parts < 2) {
    unpack_range(dst, bits, 0, n);
    return;
  }
  const size_t step = (n / parts + 4095) & ~size_t(4095);
  std::vector<std::thread> th;
  try {
    for (size_t i = 1; i < parts && i * step < n; ++i)
      th.emplace_back([=] { unpack_range(dst, bits, i * step, std::min(n, (i + 1) * step)); });
  } catch (...) {
    // no thread available: the remaining parts are unpacked below
  }
  unpack_range(dst, bits, 0, std::min(n, step));
  for (size_t i = th.size() + 1; i < parts && i * step < n; ++i)
    unpack_range(dst, bits, i * step, std::min(n, (i + 1) * step));
  for (auto &t : th) t.join();
}

// Wait for a stage's last chunk and move its answers to the caller's buffer.
int finish_slot(PipeSlot &ps) {
  if (!ps.pending) return SBF_OK;
  ps.pending = false;
  SBF_HIP(hipEventSynchronize(ps.done), "kernel execution");
  if (ps.flush_dst && ps.flush_len) {
    if (ps.flush_packed)
      unpack_bits(ps.flush_dst, (const uint8_t *)ps.h_out.ptr, ps.flush_len);
    else
      host_copy(ps.flush_dst, ps.h_out.ptr, ps.flush_len);
  }
  ps.flush_dst = nullptr;
  ps.flush_len = 0;
  ps.flush_packed = false;
  return SBF_OK;
}

// After a failure: let the queued work end so that no copy still reads or
// writes the caller's buffers, and keep the first error.
int drain_pipe(sbf_filter *f, int rc) {
  for (PipeSlot &ps : f->pipe) {
    if (ps.stream) (void)hipStreamSynchronize(ps.stream);
    ps.pending = false;
    ps.flush_dst = nullptr;
    ps.flush_packed = false;
  }
  (void)hipGetLastError();
  return rc;
}

// Host-sequence insert or query of one record batch, in chunks of at most
// `staging` bases whose k-mer starts partition [0, total); a chunk carries
// k-1 extra bases.  Chunk c runs on pipeline stage c mod 2: the caller's bases
// are copied into pinned memory (or sent directly when the caller's buffer is
// pinned), sent to the device, marked, and inserted or queried.  With the
// lane query, answers come back as bits (an eighth of the bytes over the host
// link) and are spread to bytes on the host; otherwise as bytes, copied like
// the input.  The kernels of successive chunks are ordered by events, so
// inserts never overlap one another.  Queries write answers for k-mer starts
// [0, n_out).
int host_batch(sbf_filter *f, const char *seq, const uint64_t *off, uint64_t nrec, uint8_t *out, uint64_t n_out,
               bool query) {
  // earlier stream-ordered work on any stream may still use the filter
  SBF_HIP(hipDeviceSynchronize(), "device synchronisation");
  int rc;
  if ((rc = ensure_pipe(f))) return rc;
  const uint64_t k = f->g.k;
  const uint64_t total = off[nrec];
  const uint64_t budget = std::max<uint64_t>(f->staging, 4096);
  const bool packed = query && family(f) == kLaneFamily && sbf::query_packed_supported(query_kernel_mode(f));
  // k-mer starts per chunk; a multiple of 64 when answers travel as bits, so
  // that every chunk's bits start on a byte
  const uint64_t span = packed ? (budget - (k - 1)) & ~63ull : budget - (k - 1);
  const bool in_direct = host_pinned(seq);
  const bool out_direct = query && !packed && host_pinned(out);
  hipEvent_t prev_kernel = nullptr;
  uint64_t r0 = 0;  // first record overlapping the chunk
  int si = 0;
  for (uint64_t c0 = 0; c0 < total; c0 += span, si = (si + 1) % kPipeSlots) {
    PipeSlot &ps = f->pipe[si];
    if ((rc = finish_slot(ps))) return drain_pipe(f, rc);
    const uint64_t c1 = std::min(total, c0 + span);       // k-mer starts [c0, c1)
    const uint64_t e1 = std::min(total, c1 + k - 1);      // bases [c0, e1)
    const uint64_t o1 = std::min(c1, n_out);              // answers wanted for starts [c0, o1)
    while (r0 + 1 < nrec && off[r0 + 1] <= c0) ++r0;
    uint64_t r1 = r0;  // last record overlapping the chunk
    while (r1 + 1 < nrec && off[r1 + 1] < e1) ++r1;
    const uint64_t nloc = r1 - r0 + 1;
    const uint64_t len = e1 - c0;
    hipStream_t st = ps.stream;
    if ((rc = grow(ps.d_seq, budget + 64, "staging buffer"))) return drain_pipe(f, rc);
    const char *src = seq + c0;
    if (!in_direct) {
      if ((rc = grow_pinned(ps.h_seq, budget + 64, "pinned staging buffer"))) return drain_pipe(f, rc);
      host_copy(ps.h_seq.ptr, src, len);
      src = (const char *)ps.h_seq.ptr;
    }
    hipError_t e = hipMemcpyAsync(ps.d_seq.ptr, src, len, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return drain_pipe(f, hip_error(e, "copy sequence to device"));
    const uint32_t *starts = nullptr;
    if (nloc > 1) {
      // local offsets: 0, each record start inside the chunk, then len
      const size_t ob = (nloc + 1) * 8;
      if ((rc = grow_pinned(ps.h_off, ob, "pinned staging buffer")) || (rc = grow(ps.d_off, ob, "staging buffer")))
        return drain_pipe(f, rc);
      uint64_t *loc = (uint64_t *)ps.h_off.ptr;
      loc[0] = 0;
      for (uint64_t r = 1; r < nloc; ++r) loc[r] = off[r0 + r] - c0;
      loc[nloc] = len;
      e = hipMemcpyAsync(ps.d_off.ptr, loc, ob, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) return drain_pipe(f, hip_error(e, "copy offsets to device"));
    }
    if (prev_kernel && (e = hipStreamWaitEvent(st, prev_kernel, 0)) != hipSuccess)
      return drain_pipe(f, hip_error(e, "pipeline ordering"));
    if (nloc > 1 && (rc = record_starts(f, (const uint64_t *)ps.d_off.ptr, nloc, len, st, &starts)))
      return drain_pipe(f, rc);
    SeqArgs a{(const uint8_t *)ps.d_seq.ptr, len, starts, nullptr, 0};
    if (query) {
      if ((rc = grow(ps.d_out, budget + 64, "staging buffer"))) return drain_pipe(f, rc);
      a.out = (uint8_t *)ps.d_out.ptr;
      a.n_out = c1 - c0;
      a.packed = packed ? 1 : 0;
      rc = run_query(f, a, st);
    } else {
      rc = run_insert(f, a, st);
    }
    if (rc) return drain_pipe(f, rc);
    if ((e = hipEventRecord(ps.kernel_done, st)) != hipSuccess) return drain_pipe(f, hip_error(e, "event record"));
    prev_kernel = ps.kernel_done;
    if (query && o1 > c0) {
      uint8_t *dst = out + c0;
      uint64_t nbytes = o1 - c0;
      if (!out_direct) {
        if ((rc = grow_pinned(ps.h_out, (packed ? budget / 8 : budget) + 64, "pinned staging buffer")))
          return drain_pipe(f, rc);
        ps.flush_dst = dst;
        ps.flush_len = o1 - c0;
        ps.flush_packed = packed;
        dst = (uint8_t *)ps.h_out.ptr;
        if (packed) nbytes = (o1 - c0 + 7) / 8;
      }
      e = hipMemcpyAsync(dst, ps.d_out.ptr, nbytes, hipMemcpyDeviceToHost, st);
      if (e != hipSuccess) return drain_pipe(f, hip_error(e, "copy answers to host"));
    }
    if ((e = hipEventRecord(ps.done, st)) != hipSuccess) return drain_pipe(f, hip_error(e, "event record"));
    ps.pending = true;
  }
  for (PipeSlot &ps : f->pipe)
    if ((rc = finish_slot(ps))) return drain_pipe(f, rc);
  return SBF_OK;
}

int validate_offsets(const uint64_t *off, uint64_t nrec) {
  if (!off) return set_error(SBF_E_INVAL, "offsets are NULL");
  if (off[0] != 0) return set_error(SBF_E_INVAL, "off[0] must be 0");
  for (uint64_t r = 0; r < nrec; ++r)
    if (off[r + 1] < off[r]) return set_error(SBF_E_INVAL, "offsets decrease at record %llu", (unsigned long long)r);
  return SBF_OK;
}

}  // namespace

extern "C" {

sbf_filter *sbf_create(uint32_t k, uint32_t s, uint32_t m, uint32_t H, uint64_t bits) {
  return sbf_create_ex(k, s, m, H, bits, 4);
}

sbf_filter *sbf_create_ex(uint32_t k, uint32_t s, uint32_t m, uint32_t H, uint64_t bits, uint32_t shard_words) {
  if (k < 1 || k > 32 || s < 1 || s > k || m < 1 || m > k || H < 1 || H > 16 || bits < 1 || bits > kMaxBits) {
    set_error(SBF_E_INVAL,
              "invalid parameters k=%u s=%u m=%u H=%u bits=%llu (need 1<=s,m<=k<=32, 1<=H<=16, 1<=bits<=2^40)", k, s,
              m, H, (unsigned long long)bits);
    return nullptr;
  }
  // shard geometry: 4, 8 or 16 words; a wider shard takes its word group from
  // the log2(S/4) bits above each 6-bit address, which must fit the slice
  const uint32_t extra = shard_words == 16 ? 2 : shard_words == 8 ? 1 : 0;
  if ((shard_words != 4 && shard_words != 8 && shard_words != 16) || (extra && 64 / H < 6 + extra)) {
    set_error(SBF_E_INVAL, "invalid shard geometry: %u words with H=%u (need 4, 8 or 16 words, and 64/H >= %u)",
              shard_words, H, 6 + extra);
    return nullptr;
  }
  sbf_filter *f = new (std::nothrow) sbf_filter;
  if (!f) {
    set_error(SBF_E_NOMEM, "host allocation of the filter object");
    return nullptr;
  }
  f->g.k = k;
  f->g.s = s;
  f->g.m = m;
  f->g.H = H;
  f->g.shard_words = shard_words;
  const uint64_t per_shard = 64ull * shard_words;
  f->g.nshards = next_pow2(std::max<uint64_t>(1, (bits + per_shard - 1) / per_shard));
  hipError_t e = hipGetDevice(&f->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&f->num_cus, hipDeviceAttributeMultiprocessorCount, f->device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&f->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    hip_error(e, "stream creation");
    delete f;
    return nullptr;
  }
  const uint64_t nwords = f->g.nshards * f->g.shard_words;
  e = hipMalloc((void **)&f->words, nwords * sizeof(uint64_t));
  if (e != hipSuccess) {
    f->words = nullptr;
    hip_error(e, "filter allocation");
    (void)hipStreamDestroy(f->stream);
    delete f;
    return nullptr;
  }
  e = sbf::launch_fill_u64(f->words, nwords, 0ull, f->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
  uint32_t *noalloc = nullptr;
  if (e != hipSuccess || noalloc_scratch(f->device, &noalloc) != SBF_OK) {
    if (e != hipSuccess) hip_error(e, "filter initialisation");
    (void)hipFree(f->words);
    (void)hipStreamDestroy(f->stream);
    delete f;
    return nullptr;
  }
  ok();
  return f;
}

void sbf_destroy(sbf_filter *f) {
  if (!f) return;
  (void)hipSetDevice(f->device);
  (void)hipDeviceSynchronize();
  for (auto &kv : f->starts)
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
  for (auto &kv : f->queues)
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
  for (PipeSlot &ps : f->pipe) {
    for (Scratch *d : {&ps.d_seq, &ps.d_out, &ps.d_off})
      if (d->ptr) (void)hipFree(d->ptr);
    for (Pinned *h : {&ps.h_seq, &ps.h_out, &ps.h_off})
      if (h->ptr) (void)hipHostFree(h->ptr);
    if (ps.kernel_done) (void)hipEventDestroy(ps.kernel_done);
    if (ps.done) (void)hipEventDestroy(ps.done);
    if (ps.stream) (void)hipStreamDestroy(ps.stream);
  }
  if (f->words) (void)hipFree(f->words);
  if (f->stream) (void)hipStreamDestroy(f->stream);
  delete f;
}

int sbf_last_error(const char **msg) {
  if (msg) *msg = g_msg.c_str();
  return g_err;
}

uint64_t sbf_num_shards(const sbf_filter *f) { return f ? f->g.nshards : 0; }
uint64_t sbf_num_bits(const sbf_filter *f) { return f ? f->g.nshards * f->g.shard_words * 64ull : 0; }
uint64_t sbf_num_words(const sbf_filter *f) { return f ? f->g.nshards * f->g.shard_words : 0; }
const uint64_t *sbf_device_words(const sbf_filter *f) { return f ? f->words : nullptr; }

int sbf_get_bits(const sbf_filter *f, uint64_t *host_dst, uint64_t nwords) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (!host_dst || nwords != sbf_num_words(f)) return set_error(SBF_E_INVAL, "need %llu words", (unsigned long long)sbf_num_words(f));
  if ((rc = set_device(f))) return rc;
  SBF_HIP(hipDeviceSynchronize(), "device synchronisation");
  SBF_HIP(hipMemcpy(host_dst, f->words, nwords * 8, hipMemcpyDeviceToHost), "copy filter to host");
  return ok();
}

int sbf_set_bits(sbf_filter *f, const uint64_t *host_src, uint64_t nwords) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (!host_src || nwords != sbf_num_words(f)) return set_error(SBF_E_INVAL, "need %llu words", (unsigned long long)sbf_num_words(f));
  if ((rc = set_device(f))) return rc;
  SBF_HIP(hipDeviceSynchronize(), "device synchronisation");
  SBF_HIP(hipMemcpy(f->words, host_src, nwords * 8, hipMemcpyHostToDevice), "copy filter to device");
  return ok();
}

int sbf_clear(sbf_filter *f, void *stream) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if ((rc = set_device(f))) return rc;
  hipError_t e = sbf::launch_fill_u64(f->words, sbf_num_words(f), 0ull, pick(f, stream));
  if (e != hipSuccess) return hip_error(e, "clear kernel launch");
  return ok();
}

int sbf_estimate_fpr(const sbf_filter *f, double *fpr, uint64_t *set_bits) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (!fpr && !set_bits) return set_error(SBF_E_INVAL, "no output");
  if ((rc = set_device(f))) return rc;
  SBF_HIP(hipDeviceSynchronize(), "device synchronisation");
  Scratch acc;
  if ((rc = grow(acc, 16, "statistics accumulators"))) return rc;
  double *d_sum = (double *)acc.ptr;
  uint64_t *d_bits = (uint64_t *)acc.ptr + 1;
  hipError_t e = sbf::launch_fill_u64((uint64_t *)acc.ptr, 2, 0ull, f->stream);
  if (e == hipSuccess) e = sbf::launch_estimate_fpr(f->g, f->words, d_sum, d_bits, f->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
  uint64_t host[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpy(host, acc.ptr, 16, hipMemcpyDeviceToHost);
  (void)hipFree(acc.ptr);
  if (e != hipSuccess) return hip_error(e, "filter statistics");
  double sum;
  memcpy(&sum, &host[0], sizeof sum);
  if (fpr) *fpr = sum / (double)f->g.nshards;
  if (set_bits) *set_bits = host[1];
  return ok();
}

int sbf_insert_seq_dev(sbf_filter *f, const char *d_seq, uint64_t len, void *stream) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (len == 0) return ok();
  if (!d_seq) return set_error(SBF_E_INVAL, "sequence is NULL");
  if ((rc = set_device(f))) return rc;
  SeqArgs a{(const uint8_t *)d_seq, len, nullptr, nullptr, 0};
  if ((rc = run_insert(f, a, pick(f, stream)))) return rc;
  return ok();
}

int sbf_query_seq_dev(sbf_filter *f, const char *d_seq, uint64_t len, uint8_t *d_out, void *stream) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (len < f->g.k) return ok();
  if (!d_seq || !d_out) return set_error(SBF_E_INVAL, "sequence or output is NULL");
  if ((rc = set_device(f))) return rc;
  SeqArgs a{(const uint8_t *)d_seq, len, nullptr, d_out, len - f->g.k + 1};
  if ((rc = run_query(f, a, pick(f, stream)))) return rc;
  return ok();
}

int sbf_insert_batch_dev(sbf_filter *f, const char *d_seq, uint64_t len, const uint64_t *d_off, uint64_t nrec,
                         void *stream) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (len == 0 || nrec == 0) return ok();
  if (!d_seq || !d_off) return set_error(SBF_E_INVAL, "sequence or offsets are NULL");
  if ((rc = set_device(f))) return rc;
  hipStream_t st = pick(f, stream);
  const uint32_t *starts = nullptr;
  if ((rc = record_starts(f, d_off, nrec, len, st, &starts))) return rc;
  SeqArgs a{(const uint8_t *)d_seq, len, starts, nullptr, 0};
  if ((rc = run_insert(f, a, st))) return rc;
  return ok();
}

int sbf_query_batch_dev(sbf_filter *f, const char *d_seq, uint64_t len, const uint64_t *d_off, uint64_t nrec,
                        uint8_t *d_out, void *stream) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (len == 0 || nrec == 0) return ok();
  if (!d_seq || !d_off || !d_out) return set_error(SBF_E_INVAL, "sequence, offsets or output is NULL");
  if ((rc = set_device(f))) return rc;
  hipStream_t st = pick(f, stream);
  const uint32_t *starts = nullptr;
  if ((rc = record_starts(f, d_off, nrec, len, st, &starts))) return rc;
  SeqArgs a{(const uint8_t *)d_seq, len, starts, d_out, len};
  if ((rc = run_query(f, a, st))) return rc;
  return ok();
}

int sbf_query_batch_dev_noalloc(sbf_filter *f, const char *d_seq, uint64_t len, const uint64_t *d_off,
                                uint64_t nrec, uint8_t *d_out, void *stream) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (len == 0 || nrec == 0) return ok();
  if (!d_seq || !d_off || !d_out) return set_error(SBF_E_INVAL, "sequence, offsets or output is NULL");
  if (len > kNoAllocMaxBases)
    return set_error(SBF_E_INVAL, "batch of %llu bases exceeds the %llu bases of the allocation-free scratch",
                     (unsigned long long)len, (unsigned long long)kNoAllocMaxBases);
  if ((rc = set_device(f))) return rc;
  uint32_t *scr = nullptr;
  if ((rc = noalloc_scratch(f->device, &scr))) return rc;
  hipStream_t st = pick(f, stream);
  const uint32_t *starts = nullptr;
  if (nrec >= 2) {
    // the bits of this batch only: clear its words (a fill kernel), then mark
    uint32_t *w = scr + kNoAllocQueueWords;
    const uint64_t nw = (len + 31) / 32;
    hipError_t e = sbf::launch_fill_u32(w, nw, 0u, st);
    if (e == hipSuccess) e = sbf::launch_mark_record_starts(d_off, nrec, len, w, st);
    if (e != hipSuccess) return hip_error(e, "record-start marking");
    starts = w;
  }
  // persistent launches take their tile counters from the scratch as well
  sbf::LaunchShape ls{scr, 0};
  SeqArgs a{(const uint8_t *)d_seq, len, starts, d_out, len};
  if ((rc = run_query(f, a, st, &ls))) return rc;
  return ok();
}

int sbf_mark_record_starts_dev(const uint64_t *d_off, uint64_t nrec, uint64_t len, uint32_t *d_starts,
                               void *stream) {
  if (len == 0) return ok();
  if (!d_off || !d_starts) return set_error(SBF_E_INVAL, "offsets or record-start bits are NULL");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = sbf::launch_fill_u32(d_starts, (len + 31) / 32, 0u, st);
  if (e == hipSuccess) e = sbf::launch_mark_record_starts(d_off, nrec, len, d_starts, st);
  if (e != hipSuccess) return hip_error(e, "record-start marking");
  return ok();
}

int sbf_insert_marked_dev(sbf_filter *f, const char *d_seq, uint64_t len, const uint32_t *d_starts, void *stream) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (len == 0) return ok();
  if (!d_seq) return set_error(SBF_E_INVAL, "sequence is NULL");
  if ((rc = set_device(f))) return rc;
  SeqArgs a{(const uint8_t *)d_seq, len, d_starts, nullptr, 0};
  if ((rc = run_insert(f, a, pick(f, stream)))) return rc;
  return ok();
}

int sbf_query_marked_dev(sbf_filter *f, const char *d_seq, uint64_t len, const uint32_t *d_starts, uint8_t *d_out,
                         void *stream) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (len == 0) return ok();
  if (!d_seq || !d_out) return set_error(SBF_E_INVAL, "sequence or output is NULL");
  if ((rc = set_device(f))) return rc;
  SeqArgs a{(const uint8_t *)d_seq, len, d_starts, d_out, len};
  if ((rc = run_query(f, a, pick(f, stream)))) return rc;
  return ok();
}

int sbf_insert_seq(sbf_filter *f, const char *seq, uint64_t len) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (len < f->g.k) return ok();
  if (!seq) return set_error(SBF_E_INVAL, "sequence is NULL");
  if ((rc = set_device(f))) return rc;
  const uint64_t off[2] = {0, len};
  if ((rc = host_batch(f, seq, off, 1, nullptr, 0, false))) return rc;
  return ok();
}

int sbf_query_seq(sbf_filter *f, const char *seq, uint64_t len, uint8_t *out) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (len < f->g.k) return ok();
  if (!seq || !out) return set_error(SBF_E_INVAL, "sequence or output is NULL");
  if ((rc = set_device(f))) return rc;
  // one record; answers for k-mer starts [0, len-k+1)
  const uint64_t off[2] = {0, len};
  if ((rc = host_batch(f, seq, off, 1, out, len - f->g.k + 1, true))) return rc;
  return ok();
}

int sbf_insert_batch(sbf_filter *f, const char *seq, const uint64_t *off, uint64_t nrec) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (nrec == 0) return ok();
  if ((rc = validate_offsets(off, nrec))) return rc;
  if (off[nrec] == 0) return ok();
  if (!seq) return set_error(SBF_E_INVAL, "sequence is NULL");
  if ((rc = set_device(f))) return rc;
  if ((rc = host_batch(f, seq, off, nrec, nullptr, 0, false))) return rc;
  return ok();
}

int sbf_query_batch(sbf_filter *f, const char *seq, const uint64_t *off, uint64_t nrec, uint8_t *out) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (nrec == 0) return ok();
  if ((rc = validate_offsets(off, nrec))) return rc;
  if (off[nrec] == 0) return ok();
  if (!seq || !out) return set_error(SBF_E_INVAL, "sequence or output is NULL");
  if ((rc = set_device(f))) return rc;
  if ((rc = host_batch(f, seq, off, nrec, out, off[nrec], true))) return rc;
  return ok();
}

int sbf_set_variant(sbf_filter *f, int variant) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (variant != SBF_VARIANT_AUTO && variant != SBF_VARIANT_ROLLING && variant != SBF_VARIANT_GENERIC &&
      variant != SBF_VARIANT_WIDE && variant != SBF_VARIANT_PARAM)
    return set_error(SBF_E_INVAL, "unknown variant %d", variant);
  if (variant == SBF_VARIANT_ROLLING && !sbf::rolling_supported(f->g) && !sbf::wide_supported(f->g) &&
      !sbf::param_supported(f->g))
    return set_error(SBF_E_INVAL, "no super-k-mer kernel for k=%u s=%u m=%u H=%u with %u-word shards", f->g.k,
                     f->g.s, f->g.m, f->g.H, f->g.shard_words);
  if (variant == SBF_VARIANT_WIDE && !sbf::wide_supported(f->g))
    return set_error(SBF_E_INVAL, "no wide-shard kernel for k=%u s=%u m=%u H=%u", f->g.k, f->g.s, f->g.m, f->g.H);
  if (variant == SBF_VARIANT_PARAM && !sbf::param_supported(f->g))
    return set_error(SBF_E_INVAL, "no run-time parameter kernel for k=%u s=%u m=%u H=%u (needs k <= 32, H <= 8)",
                     f->g.k, f->g.s, f->g.m, f->g.H);
  f->variant = variant;
  // lane lengths belong to a family: back to the new family's defaults
  f->insert_lane_len = 0;
  f->query_lane_len = 0;
  return ok();
}

int sbf_get_variant(const sbf_filter *f) {
  if (!f) return set_error(SBF_E_INVAL, "filter is NULL");
  ok();
  switch (family(f)) {
    case kLaneFamily: return SBF_VARIANT_ROLLING;
    case kWideFamily: return SBF_VARIANT_WIDE;
    case kParamFamily: return SBF_VARIANT_PARAM;
    default: return SBF_VARIANT_GENERIC;
  }
}

int sbf_set_tile(sbf_filter *f, uint32_t insert_kmers_per_lane, uint32_t query_kmers_per_lane) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (!lane_len_ok(f, insert_kmers_per_lane, true) || !lane_len_ok(f, query_kmers_per_lane, false))
    return set_error(SBF_E_INVAL, "no compiled tile of %u (insert) / %u (query) k-mers per lane for this filter",
                     insert_kmers_per_lane, query_kmers_per_lane);
  f->insert_lane_len = insert_kmers_per_lane;
  f->query_lane_len = query_kmers_per_lane;
  return ok();
}

int sbf_get_tile(const sbf_filter *f, uint32_t *insert_kmers_per_lane, uint32_t *query_kmers_per_lane) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (insert_kmers_per_lane) *insert_kmers_per_lane = lane_len_effective(f, f->insert_lane_len, true);
  if (query_kmers_per_lane) *query_kmers_per_lane = lane_len_effective(f, f->query_lane_len, false);
  return ok();
}

int sbf_set_insert_mode(sbf_filter *f, int mode) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (mode != SBF_INSERT_TWO_PASS && mode != SBF_INSERT_ATOMIC)
    return set_error(SBF_E_INVAL, "unknown insert mode %d", mode);
  f->insert_mode = mode;
  return ok();
}

int sbf_set_query_mode(sbf_filter *f, int mode) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (mode != SBF_QUERY_LANE && mode != SBF_QUERY_LEADER && mode != SBF_QUERY_DIRECT)
    return set_error(SBF_E_INVAL, "unknown query mode %d", mode);
  f->query_mode = mode;
  return ok();
}

int sbf_set_launch(sbf_filter *f, uint32_t insert_wgs_per_cu, uint32_t query_wgs_per_cu) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (insert_wgs_per_cu > 32 || query_wgs_per_cu > 32)
    return set_error(SBF_E_INVAL, "at most 32 persistent workgroups per CU");
  f->insert_wgs_per_cu = insert_wgs_per_cu;
  f->query_wgs_per_cu = query_wgs_per_cu;
  return ok();
}

int sbf_get_launch(const sbf_filter *f, uint32_t *insert_wgs_per_cu, uint32_t *query_wgs_per_cu, int *insert_mode,
                   int *query_mode) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (insert_wgs_per_cu) *insert_wgs_per_cu = f->insert_wgs_per_cu;
  if (query_wgs_per_cu) *query_wgs_per_cu = f->query_wgs_per_cu;
  if (insert_mode) *insert_mode = f->insert_mode;
  if (query_mode) *query_mode = f->query_mode;
  return ok();
}

int sbf_set_staging_bytes(sbf_filter *f, uint64_t bytes) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  if (bytes < 4096) return set_error(SBF_E_INVAL, "staging must be at least 4096 bytes");
  f->staging = bytes;
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form: a HIP graph of one insert batch and one query batch, and the
// autotuner of launch shapes and kernel organisation.
// ---------------------------------------------------------------------------
struct sbf_graph {
  sbf_filter *f = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  Scratch starts_ins, starts_q, queue;
};

namespace {

void free_scratch(Scratch &s) {
  if (s.ptr) (void)hipFree(s.ptr);
  s.ptr = nullptr;
  s.bytes = 0;
}

void graph_release(sbf_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  free_scratch(g->starts_ins);
  free_scratch(g->starts_q);
  free_scratch(g->queue);
  delete g;
}

void appendf(std::string &out, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void appendf(std::string &out, const char *fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  out += buf;
}

// fill + mark record starts into s (allocated before any capture)
int mark_into(Scratch &s, const uint64_t *d_off, uint64_t nrec, uint64_t len, hipStream_t st, const uint32_t **out) {
  *out = nullptr;
  if (nrec < 2 || len == 0) return SBF_OK;
  const uint64_t nw = (len + 31) / 32;
  hipError_t e = sbf::launch_fill_u32((uint32_t *)s.ptr, nw, 0u, st);
  if (e == hipSuccess) e = sbf::launch_mark_record_starts(d_off, nrec, len, (uint32_t *)s.ptr, st);
  if (e != hipSuccess) return hip_error(e, "record-start marking");
  *out = (const uint32_t *)s.ptr;
  return SBF_OK;
}

}  // namespace

extern "C" {

sbf_graph *sbf_graph_create(sbf_filter *f, int clear_first, const char *d_ins, uint64_t ins_len,
                            const uint64_t *d_ins_off, uint64_t ins_nrec, const char *d_q, uint64_t q_len,
                            const uint64_t *d_q_off, uint64_t q_nrec, uint8_t *d_out) {
  if (check_filter(f)) return nullptr;
  if ((d_ins && ins_len && (!d_ins_off || ins_nrec == 0)) || (d_q && q_len && (!d_q_off || q_nrec == 0 || !d_out))) {
    set_error(SBF_E_INVAL, "batch without offsets, records or output");
    return nullptr;
  }
  if (set_device(f)) return nullptr;
  sbf_graph *g = new (std::nothrow) sbf_graph;
  if (!g) {
    set_error(SBF_E_NOMEM, "host allocation of the graph object");
    return nullptr;
  }
  g->f = f;
  const bool do_ins = d_ins && ins_len, do_q = d_q && q_len;
  int rc = grow(g->queue, 256, "work-queue counters");
  if (!rc && do_ins && ins_nrec > 1) rc = grow(g->starts_ins, (ins_len + 31) / 32 * 4, "record-start bits");
  if (!rc && do_q && q_nrec > 1) rc = grow(g->starts_q, (q_len + 31) / 32 * 4, "record-start bits");
  hipError_t e = hipSuccess;
  if (!rc) {
    e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
    if (e != hipSuccess) rc = hip_error(e, "capture stream");
  }
  if (rc) {
    graph_release(g);
    return nullptr;
  }
  e = hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    hip_error(e, "graph capture");
    graph_release(g);
    return nullptr;
  }
  sbf::LaunchShape ls{(uint32_t *)g->queue.ptr, 0};
  if (clear_first) {
    e = sbf::launch_fill_u64(f->words, sbf_num_words(f), 0ull, g->cap);
    if (e != hipSuccess) rc = hip_error(e, "clear kernel launch");
  }
  const uint32_t *st_ins = nullptr, *st_q = nullptr;
  if (!rc && do_ins) rc = mark_into(g->starts_ins, d_ins_off, ins_nrec, ins_len, g->cap, &st_ins);
  if (!rc && do_q) rc = mark_into(g->starts_q, d_q_off, q_nrec, q_len, g->cap, &st_q);
  if (!rc && do_ins) {
    SeqArgs a{(const uint8_t *)d_ins, ins_len, st_ins, nullptr, 0};
    rc = run_insert(f, a, g->cap, &ls);
  }
  if (!rc && do_q) {
    SeqArgs a{(const uint8_t *)d_q, q_len, st_q, d_out, q_len};
    rc = run_query(f, a, g->cap, &ls);
  }
  e = hipStreamEndCapture(g->cap, &g->graph);
  if (!rc && e != hipSuccess) rc = hip_error(e, "graph capture");
  if (!rc) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) rc = hip_error(e, "graph instantiation");
  }
  if (rc) {
    graph_release(g);
    return nullptr;
  }
  ok();
  return g;
}

int sbf_graph_launch(sbf_graph *g, void *stream) {
  if (!g) return set_error(SBF_E_INVAL, "graph is NULL");
  int rc;
  if ((rc = set_device(g->f))) return rc;
  SBF_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream), "graph launch");
  return ok();
}

void sbf_graph_destroy(sbf_graph *g) {
  if (!g) return;
  (void)hipSetDevice(g->f->device);
  (void)hipDeviceSynchronize();
  graph_release(g);
}

}  // extern "C"

namespace {

void copy_report(const std::string &rep, char *report, uint64_t report_len) {
  if (report && report_len) {
    const size_t n = std::min<size_t>(rep.size(), report_len - 1);
    memcpy(report, rep.data(), n);
    report[n] = 0;
  }
}

struct Batch {
  const char *seq;
  uint64_t len;
  const uint64_t *off;
  uint64_t nrec;
  bool ok() const { return seq && off && len && nrec; }
};

// Autotuner of one filter: on the insert batch `ins` and query batch `q`,
// time every insert strategy, query organisation, compiled lane length and
// launch shape of the filter's kernel family (median of three runs after a
// warm-up) on f itself, whose words are saved to a temporary device buffer
// and restored afterwards, then apply the fastest.  Generic kernels have
// nothing to tune and are timed as they are.  Appends the report to rep and
// returns the best insert and query times.
int autotune_filter(sbf_filter *f, const Batch &ins, const Batch &q, std::string &rep, float *best_ins_out,
                    float *best_q_out) {
  int rc = SBF_OK;
#define line(...) appendf(rep, __VA_ARGS__)
  // The trials run on the filter itself, so that they see its own memory (a
  // second filter-sized allocation can be mapped differently and time
  // differently out of cache); its words are saved first and put back after.
  sbf_filter *t = f;
  Scratch si, sq, out, saved;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t st = t->stream;
  const int keep_imode = f->insert_mode, keep_qmode = f->query_mode;
  const uint32_t keep_iw = f->insert_wgs_per_cu, keep_qw = f->query_wgs_per_cu;
  const uint32_t keep_il = f->insert_lane_len, keep_ql = f->query_lane_len;
  SBF_HIP(hipDeviceSynchronize(), "device synchronisation");
  bool backed_up = false;
  rc = grow(saved, sbf_num_words(f) * sizeof(uint64_t), "filter backup");
  if (!rc) {
    if (hipMemcpyAsync(saved.ptr, f->words, sbf_num_words(f) * sizeof(uint64_t), hipMemcpyDeviceToDevice, st) ==
        hipSuccess)
      backed_up = true;
    else
      rc = set_error(SBF_E_DEVICE, "filter backup copy");
  }
  if (!rc) rc = grow(si, (ins.len + 31) / 32 * 4, "record-start bits");
  if (!rc) rc = grow(sq, (q.len + 31) / 32 * 4, "record-start bits");
  if (!rc) rc = grow(out, q.len, "autotune answers");
  if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
    rc = set_error(SBF_E_DEVICE, "event creation");
  const uint32_t *st_i = nullptr, *st_q = nullptr;
  if (!rc) rc = mark_into(si, ins.off, ins.nrec, ins.len, st, &st_i);
  if (!rc) rc = mark_into(sq, q.off, q.nrec, q.len, st, &st_q);
  auto time_it = [&](bool insert, float &ms_out) -> int {
    float best[3];
    for (int rep_i = 0; rep_i < 4; ++rep_i) {
      if (insert) {
        hipError_t e = sbf::launch_fill_u64(t->words, sbf_num_words(t), 0ull, st);
        if (e != hipSuccess) return hip_error(e, "clear kernel launch");
      }
      if (hipEventRecord(e0, st) != hipSuccess) return set_error(SBF_E_DEVICE, "event record");
      int r2 = insert ? run_insert(t, SeqArgs{(const uint8_t *)ins.seq, ins.len, st_i, nullptr, 0}, st)
                      : run_query(t, SeqArgs{(const uint8_t *)q.seq, q.len, st_q, (uint8_t *)out.ptr, q.len}, st);
      if (r2) return r2;
      float ms = 0.f;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        return set_error(SBF_E_DEVICE, "event timing");
      if (rep_i > 0) best[rep_i - 1] = ms;
    }
    std::sort(best, best + 3);
    ms_out = best[1];
    return SBF_OK;
  };
  float best_ins = 1e30f, best_q = 1e30f;
  int bi_mode = f->insert_mode, bq_mode = f->query_mode;
  uint32_t bi_shape = f->insert_wgs_per_cu, bq_shape = f->query_wgs_per_cu, bi_len = 0, bq_len = 0;
  const Family fam = family(f);
  if (fam == kGenericFamily) {
    if (!rc) rc = time_it(true, best_ins);
    if (!rc) rc = time_it(false, best_q);
    if (!rc) line("generic kernels (nothing to tune): insert %.4f ms, query %.4f ms\n", best_ins, best_q);
  } else {
    // the wide-shard and run-time parameter kernels have one query
    // organisation (two phases, whole lines)
    const bool wide = fam != kLaneFamily;
    const char *wide_name = fam == kParamFamily ? "param" : "wide";
    const uint32_t shapes[] = {0, 1, 2, 4, 8};
    // compiled k-mers per lane (the tile is 256 lanes of them)
    std::vector<uint32_t> ins_lens, q_lens;
    for (uint32_t n : {8u, 16u, 32u, 48u, 64u}) {
      if (lane_len_ok(f, n, true)) ins_lens.push_back(n);
      if (lane_len_ok(f, n, false)) q_lens.push_back(n);
    }
    if (ins_lens.empty()) ins_lens.push_back(0);
    if (q_lens.empty()) q_lens.push_back(0);
    // the insert's repair walk runs at the query's default lane length here
    t->query_lane_len = 0;
    for (int mode : {SBF_INSERT_TWO_PASS, SBF_INSERT_ATOMIC}) {
      for (uint32_t len : ins_lens) {
        for (uint32_t sh : shapes) {
          if (rc) break;
          t->insert_mode = mode;
          t->insert_wgs_per_cu = sh;
          t->insert_lane_len = len;
          float ms;
          rc = time_it(true, ms);
          if (rc) break;
          line("insert %-8s %2u k-mers/lane, workgroups/CU %u%s: %.4f ms\n",
               mode == SBF_INSERT_ATOMIC ? "atomic" : "two-pass", lane_len_effective(t, len, true), sh,
               sh ? "" : " (one per tile)", ms);
          if (ms < best_ins) {
            best_ins = ms;
            bi_mode = mode;
            bi_shape = sh;
            bi_len = len;
          }
        }
      }
    }
    t->insert_lane_len = 0;
    for (int mode : {SBF_QUERY_LANE, SBF_QUERY_LEADER, SBF_QUERY_DIRECT}) {
      // the wide-shard kernels have one query organisation; lane lengths
      // apply to the lane-sequential query and to the wide kernels
      if (wide && mode != SBF_QUERY_LANE) continue;
      for (uint32_t len : q_lens) {
        if (mode != SBF_QUERY_LANE && len != q_lens[0]) continue;
        for (uint32_t sh : shapes) {
          if (rc) break;
          t->query_mode = mode;
          t->query_wgs_per_cu = sh;
          t->query_lane_len = mode == SBF_QUERY_LANE ? len : 0;
          float ms;
          rc = time_it(false, ms);
          if (rc) break;
          line("query  %-8s %2u k-mers/lane, workgroups/CU %u%s: %.4f ms\n",
               wide ? wide_name : mode == SBF_QUERY_LANE ? "lane" : mode == SBF_QUERY_LEADER ? "leader" : "direct",
               mode == SBF_QUERY_LANE ? lane_len_effective(t, len, false) : 16u, sh, sh ? "" : " (one per tile)",
               ms);
          if (ms < best_q) {
            best_q = ms;
            bq_mode = mode;
            bq_shape = sh;
            bq_len = mode == SBF_QUERY_LANE ? len : 0;
          }
        }
      }
    }
    if (!rc) {
      line("best insert: %s, %u k-mers/lane, workgroups/CU %u (%.4f ms)\n",
           bi_mode == SBF_INSERT_ATOMIC ? "atomic" : "two-pass", lane_len_effective(f, bi_len, true), bi_shape,
           best_ins);
      line("best query: %s, %u k-mers/lane, workgroups/CU %u (%.4f ms)\n",
           wide ? wide_name : bq_mode == SBF_QUERY_LANE ? "lane" : bq_mode == SBF_QUERY_LEADER ? "leader" : "direct",
           bq_mode == SBF_QUERY_LANE ? lane_len_effective(f, bq_len, false) : 16u, bq_shape, best_q);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  // put the filter's words back
  if (backed_up && hipMemcpyAsync(f->words, saved.ptr, sbf_num_words(f) * sizeof(uint64_t), hipMemcpyDeviceToDevice,
                                  st) != hipSuccess && !rc)
    rc = set_error(SBF_E_DEVICE, "filter restore copy");
  (void)hipStreamSynchronize(st);
  free_scratch(si);
  free_scratch(sq);
  free_scratch(out);
  free_scratch(saved);
  f->insert_mode = keep_imode;
  f->query_mode = keep_qmode;
  f->insert_wgs_per_cu = keep_iw;
  f->query_wgs_per_cu = keep_qw;
  f->insert_lane_len = keep_il;
  f->query_lane_len = keep_ql;
  if (rc) return rc;
  f->insert_mode = bi_mode;
  f->insert_wgs_per_cu = bi_shape;
  f->insert_lane_len = bi_len;
  f->query_mode = bq_mode;
  f->query_wgs_per_cu = bq_shape;
  f->query_lane_len = bq_len;
  if (best_ins_out) *best_ins_out = best_ins;
  if (best_q_out) *best_q_out = best_q;
#undef line
  return SBF_OK;
}

// Number of k-mers of batch q that f answers present (nonzero answer bytes,
// counted on the device); synchronous on f's stream.
int count_present(sbf_filter *f, const Batch &q, uint64_t *present) {
  hipStream_t st = f->stream;
  Scratch starts, out, cnt;
  int rc = grow(starts, (q.len + 31) / 32 * 4, "record-start bits");
  if (!rc) rc = grow(out, q.len, "answers");
  if (!rc) rc = grow(cnt, 8, "counter");
  const uint32_t *st_q = nullptr;
  if (!rc) rc = mark_into(starts, q.off, q.nrec, q.len, st, &st_q);
  hipError_t e = hipSuccess;
  if (!rc) {
    e = sbf::launch_fill_u64((uint64_t *)cnt.ptr, 1, 0ull, st);
    if (e != hipSuccess) rc = hip_error(e, "fill kernel launch");
  }
  if (!rc) rc = run_query(f, SeqArgs{(const uint8_t *)q.seq, q.len, st_q, (uint8_t *)out.ptr, q.len}, st);
  if (!rc) {
    e = sbf::launch_count_nonzero_u8((const uint8_t *)out.ptr, q.len, (uint64_t *)cnt.ptr, st);
    if (e != hipSuccess) rc = hip_error(e, "count kernel launch");
  }
  (void)hipStreamSynchronize(st);
  uint64_t host = 0;
  if (!rc && hipMemcpy(&host, cnt.ptr, 8, hipMemcpyDeviceToHost) != hipSuccess)
    rc = set_error(SBF_E_DEVICE, "counter copy");
  free_scratch(starts);
  free_scratch(out);
  free_scratch(cnt);
  *present = host;
  return rc;
}

// Insert batch b into f (cleared first); synchronous on f's stream.
int fill_filter(sbf_filter *f, const Batch &b) {
  hipStream_t st = f->stream;
  Scratch starts;
  hipError_t e = sbf::launch_fill_u64(f->words, sbf_num_words(f), 0ull, st);
  if (e != hipSuccess) return hip_error(e, "clear kernel launch");
  int rc = grow(starts, (b.len + 31) / 32 * 4, "record-start bits");
  const uint32_t *st_i = nullptr;
  if (!rc) rc = mark_into(starts, b.off, b.nrec, b.len, st, &st_i);
  if (!rc) rc = run_insert(f, SeqArgs{(const uint8_t *)b.seq, b.len, st_i, nullptr, 0}, st);
  (void)hipStreamSynchronize(st);
  free_scratch(starts);
  return rc;
}

}  // namespace

extern "C" {

int sbf_autotune(sbf_filter *f, const char *d_ins, uint64_t ins_len, const uint64_t *d_ins_off, uint64_t ins_nrec,
                 const char *d_q, uint64_t q_len, const uint64_t *d_q_off, uint64_t q_nrec, char *report,
                 uint64_t report_len) {
  int rc;
  if ((rc = check_filter(f))) return rc;
  const Batch ins{d_ins, ins_len, d_ins_off, ins_nrec}, q{d_q, q_len, d_q_off, q_nrec};
  if (!ins.ok() || !q.ok()) return set_error(SBF_E_INVAL, "autotuning needs an insert batch and a query batch");
  if ((rc = set_device(f))) return rc;
  std::string rep;
  rc = autotune_filter(f, ins, q, rep, nullptr, nullptr);
  copy_report(rep, report, report_len);
  if (rc) return rc;
  return ok();
}

int sbf_autotune_geometry(uint32_t k, uint32_t s, uint32_t m, uint32_t H, uint64_t bits, const char *d_ins,
                          uint64_t ins_len, const uint64_t *d_ins_off, uint64_t ins_nrec, const char *d_q,
                          uint64_t q_len, const uint64_t *d_q_off, uint64_t q_nrec, const char *d_neg,
                          uint64_t neg_len, const uint64_t *d_neg_off, uint64_t neg_nrec, double max_fpr,
                          uint32_t *shard_words, uint32_t *insert_kmers_per_lane, uint32_t *query_kmers_per_lane,
                          double *fpr, char *report, uint64_t report_len) {
  const Batch ins{d_ins, ins_len, d_ins_off, ins_nrec}, q{d_q, q_len, d_q_off, q_nrec},
      neg{d_neg, neg_len, d_neg_off, neg_nrec};
  if (!ins.ok() || !q.ok() || !neg.ok())
    return set_error(SBF_E_INVAL, "geometry autotuning needs insert, query and negative batches");
  if (!shard_words) return set_error(SBF_E_INVAL, "shard_words is NULL");
  std::string rep;
  struct Choice {
    uint32_t S = 0, il = 0, ql = 0;
    double fpr = 2.0, ms = 1e30;
  } best_ok, best_any;
  int rc = SBF_OK;
  for (uint32_t S : {4u, 8u, 16u}) {
    sbf_filter *f = sbf_create_ex(k, s, m, H, bits, S);
    if (!f) {
      if (g_err == SBF_E_INVAL) {  // this geometry does not exist for H
        appendf(rep, "shard %2u words: not available for H=%u\n", S, H);
        continue;
      }
      rc = g_err;
      break;
    }
    float ti = 0.f, tq = 0.f;
    std::string sub;
    rc = autotune_filter(f, ins, q, sub, &ti, &tq);
    uint64_t valid = 0, present = 0;
    // valid k-mers of the negatives: every one is present in a full filter
    if (!rc) {
      hipError_t e = sbf::launch_fill_u64(f->words, sbf_num_words(f), ~0ull, f->stream);
      rc = e == hipSuccess ? count_present(f, neg, &valid) : hip_error(e, "fill kernel launch");
    }
    if (!rc) rc = fill_filter(f, ins);
    if (!rc) rc = count_present(f, neg, &present);
    uint32_t il = 0, ql = 0;
    if (!rc) rc = sbf_get_tile(f, &il, &ql);
    const int fam = sbf_get_variant(f);
    sbf_destroy(f);
    if (rc) break;
    const double rate = valid ? (double)present / (double)valid : 0.0;
    appendf(rep, "shard %2u words (%s kernels): insert %.4f ms (%u k-mers/lane), query %.4f ms (%u k-mers/lane), "
                 "FPR %.4g (%llu of %llu negative k-mers)\n",
            S, fam == SBF_VARIANT_ROLLING ? "lane" : fam == SBF_VARIANT_WIDE ? "wide-shard" : "generic", ti, il, tq,
            ql, rate, (unsigned long long)present, (unsigned long long)valid);
    const std::string indented = "    " + sub.substr(0, sub.size() ? sub.size() - 1 : 0);
    std::string body;
    for (char c : indented) {
      body += c;
      if (c == '\n') body += "    ";
    }
    rep += body + "\n";
    const double ms = (double)ti + (double)tq;
    if (rate < best_any.fpr || (rate == best_any.fpr && ms < best_any.ms)) best_any = {S, il, ql, rate, ms};
    if (rate <= max_fpr && ms < best_ok.ms) best_ok = {S, il, ql, rate, ms};
  }
  if (!rc && best_any.S == 0) rc = set_error(SBF_E_INVAL, "no shard geometry exists for H=%u", H);
  if (!rc) {
    const Choice &c = best_ok.S ? best_ok : best_any;
    appendf(rep, "%s: %u-word shards, %u/%u k-mers per lane, FPR %.4g, insert + query %.4f ms\n",
            best_ok.S ? "fastest within the FPR bound" : "no geometry meets the FPR bound; lowest FPR", c.S, c.il,
            c.ql, c.fpr, c.ms);
    *shard_words = c.S;
    if (insert_kmers_per_lane) *insert_kmers_per_lane = c.il;
    if (query_kmers_per_lane) *query_kmers_per_lane = c.ql;
    if (fpr) *fpr = c.fpr;
  }
  copy_report(rep, report, report_len);
  if (rc) return rc;
  return ok();
}

}  // extern "C"
