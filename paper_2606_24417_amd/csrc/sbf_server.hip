// Served form: a request loop over a resident filter with continuous
// batching.  A scheduler thread owns `slots` execution slots (a HIP stream, a
// device staging area for `slot_bases` bases / `slot_records` records, and an
// event).  Whenever a slot is free it takes pending query requests in arrival
// order for as long as they fit its memory, concatenates them into one record
// batch (copies in, record-start marking, query kernel, copies out), and
// records the slot's event.  Requests that arrive while slots are busy wait
// in the queue and join the next batch of the first slot that frees up, so
// the copies and kernels of different batches overlap on the device.  The
// server uses the filter only through the public stream-ordered entry points.
//
// Requests whose sequence and answer buffers are 16-byte aligned pinned host
// memory that the device can address are moved by the server's own kernels
// (a gather of every such request's bases into the slot's device buffer, a
// scatter of answers back), reading and writing host memory directly; other
// requests use hipMemcpyAsync.  The runtime's copy engines can stall a
// host-to-device copy for milliseconds after an idle period, which is what
// the kernels avoid.
#include "sbf.h"
#include "sbf_internal.h"

#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

enum : int { kPending = 1, kRunning = 2, kDone = 0 };

struct Request {
  uint64_t id = 0;
  const char *seq = nullptr;
  const uint64_t *off = nullptr;
  uint64_t nrec = 0;
  uint8_t *out = nullptr;
  uint64_t bases = 0;
  bool direct_in = false, direct_out = false;  // moved by the server's kernels
  int64_t t_submit = 0, t_start = 0, t_done = 0;
  int state = kPending;
  int status = SBF_OK;
  std::string error;
};

// One request of a batch for the copy kernels.  The table lives in the slot's
// pinned memory and the kernels read it from there.
struct CopyDesc {
  const uint8_t *src;  // the caller's bases when they are moved by the gather, else null
  uint8_t *dst;        // the caller's answer buffer when the scatter writes it, else null
  uint64_t base;       // 16-byte aligned offset of the request in the slot's device buffers
  uint64_t n;          // bases
  uint64_t end;        // 16-byte aligned end; bytes [base + n, end) are padding
};

constexpr uint32_t kPad4 = 0x4E4E4E4Eu;  // "NNNN": padding bases are invalid

// Bases into the slot buffer: full 16-byte chunks of directly moved requests
// with 16-byte loads from host memory, the chunk holding the last bases byte
// by byte, and padding as 'N'.  Requests copied by the runtime only get their
// padding.  Block row y walks requests y, y + gridDim.y, ...
__global__ __launch_bounds__(256) void gather_kernel(const CopyDesc *desc, uint32_t nreq, uint8_t *dev) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.y; i < nreq; i += gridDim.y) {
    const CopyDesc d = desc[i];
    const uint64_t nch = (d.end - d.base) >> 4;
    const uint64_t cfull = d.n >> 4;
    const uint32_t keep = (uint32_t)(d.n & 15);
    for (uint64_t c = (d.src ? 0 : cfull) + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += stride) {
      uint8_t *o = dev + d.base + 16 * c;
      if (c < cfull) {
        *reinterpret_cast<uint4 *>(o) = *reinterpret_cast<const uint4 *>(d.src + 16 * c);
      } else if (c == cfull && keep) {
        if (d.src) {
          uint32_t w[4] = {kPad4, kPad4, kPad4, kPad4};
          for (uint32_t j = 0; j < keep; ++j) {
            const uint32_t sh = 8 * (j & 3);
            w[j >> 2] = (w[j >> 2] & ~(0xFFu << sh)) | ((uint32_t)d.src[16 * c + j] << sh);
          }
          *reinterpret_cast<uint4 *>(o) = make_uint4(w[0], w[1], w[2], w[3]);
        } else {
          for (uint32_t j = keep; j < 16; ++j) o[j] = (uint8_t)'N';
        }
      } else {
        *reinterpret_cast<uint4 *>(o) = make_uint4(kPad4, kPad4, kPad4, kPad4);
      }
    }
  }
}

// Answers back into the callers' buffers for directly moved requests:
// 16-byte stores for full chunks, byte stores for the last bytes; nothing
// outside [dst, dst + n) is written.
__global__ __launch_bounds__(256) void scatter_kernel(const CopyDesc *desc, uint32_t nreq, const uint8_t *dev) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.y; i < nreq; i += gridDim.y) {
    const CopyDesc d = desc[i];
    if (!d.dst) continue;
    const uint64_t cfull = d.n >> 4;
    const uint64_t nch = (d.n + 15) >> 4;
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nch; c += stride) {
      const uint8_t *in = dev + d.base + 16 * c;
      if (c < cfull) {
        *reinterpret_cast<uint4 *>(d.dst + 16 * c) = *reinterpret_cast<const uint4 *>(in);
      } else {
        for (uint32_t j = 0; j < (uint32_t)(d.n & 15); ++j) d.dst[16 * c + j] = in[j];
      }
    }
  }
}

hipError_t launch_copy(bool gather, const CopyDesc *desc, uint32_t nreq, uint8_t *dev, hipStream_t st) {
  if (nreq == 0) return hipSuccess;
  const dim3 grid(64, std::min<uint32_t>(nreq, 65535u));
  if (gather)
    hipLaunchKernelGGL(gather_kernel, grid, dim3(256), 0, st, desc, nreq, dev);
  else
    hipLaunchKernelGGL(scatter_kernel, grid, dim3(256), 0, st, desc, nreq, (const uint8_t *)dev);
  return hipGetLastError();
}

// True when p is 16-byte aligned pinned host memory that the device addresses
// with the same pointer.
bool device_view(const void *p) {
  if (!p || ((uintptr_t)p & 15u)) return false;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeHost && at.devicePointer == p;
}

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char *d_seq = nullptr;
  uint8_t *d_out = nullptr;
  uint64_t *d_off = nullptr;
  uint32_t *d_starts = nullptr;
  uint64_t *h_off = nullptr;  // pinned; reused once the slot's event has completed
  CopyDesc *h_desc = nullptr;  // pinned copy descriptors, one per request of a batch
  const uint64_t *dv_off = nullptr;  // device addresses of h_off and h_desc
  const CopyDesc *dv_desc = nullptr;
  std::vector<Request *> reqs;
  bool busy = false;
};

}  // namespace

struct sbf_server {
  sbf_filter *f = nullptr;
  int device = 0;
  uint64_t cap_bases = 0, cap_records = 0;
  uint32_t max_pending = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> pending;
  std::unordered_map<uint64_t, Request *> live;
  uint64_t next_id = 1;
  int64_t window_ns = 0;  // batching window (0: launch as soon as a slot is free)
  bool stop = false;
  bool ready = false;               // the scheduler has warmed every slot
  hipError_t warm_error = hipSuccess;
  std::thread thread;
  uint64_t batches = 0, requests_done = 0, bases_done = 0, max_batch_requests = 0;
};

namespace {

int fail(int code, const std::string &msg) { return sbf::record_error(code, msg.c_str()); }
int succeed() { return sbf::record_error(SBF_OK, ""); }

void release_slot(sbf_filter *f, Slot &s) {
  if (s.stream) (void)hipStreamSynchronize(s.stream);
  if (s.stream && f) sbf::release_stream(f, s.stream);
  if (s.d_seq) (void)hipFree(s.d_seq);
  if (s.d_out) (void)hipFree(s.d_out);
  if (s.d_off) (void)hipFree(s.d_off);
  if (s.d_starts) (void)hipFree(s.d_starts);
  if (s.h_off) (void)hipHostFree(s.h_off);
  if (s.h_desc) (void)hipHostFree(s.h_desc);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s = Slot();
}

// Issue one batch on a free slot.  Returns an error message or "".  Each
// request starts at a 16-byte aligned offset of the slot buffers; the padding
// before the next request ('N' bases) extends the previous request's last
// record, where it only adds invalid k-mers whose answers are not returned.
std::string launch_batch(sbf_server *sv, Slot &s, const std::vector<Request *> &batch) {
  uint64_t base = 0, rec = 0;
  uint32_t i = 0;
  hipError_t e = hipSuccess;
  for (Request *r : batch) {
    const uint64_t end = (base + r->bases + 15) & ~15ull;
    s.h_desc[i++] = CopyDesc{r->direct_in ? (const uint8_t *)r->seq : nullptr, r->direct_out ? r->out : nullptr,
                             base, r->bases, end};
    if (!r->direct_in) {
      e = hipMemcpyAsync(s.d_seq + base, r->seq, r->bases, hipMemcpyHostToDevice, s.stream);
      if (e != hipSuccess) return std::string("copy to device: ") + hipGetErrorString(e);
    }
    for (uint64_t j = 0; j < r->nrec; ++j) s.h_off[rec + j] = base + r->off[j];
    rec += r->nrec;
    base = end;
  }
  s.h_off[rec] = base;
  e = launch_copy(true, s.dv_desc, i, (uint8_t *)s.d_seq, s.stream);
  if (e != hipSuccess) return std::string("gather kernel: ") + hipGetErrorString(e);
  const char *msg = nullptr;
  // the marking kernel reads the offsets straight from the slot's pinned table
  if (sbf_mark_record_starts_dev(s.dv_off, rec, base, s.d_starts, s.stream) != SBF_OK ||
      sbf_query_marked_dev(sv->f, s.d_seq, base, s.d_starts, s.d_out, s.stream) != SBF_OK) {
    sbf_last_error(&msg);
    return std::string("query: ") + (msg ? msg : "");
  }
  e = launch_copy(false, s.dv_desc, i, s.d_out, s.stream);
  if (e != hipSuccess) return std::string("scatter kernel: ") + hipGetErrorString(e);
  for (uint32_t j = 0; j < i; ++j) {
    const Request *r = batch[j];
    if (r->direct_out) continue;
    e = hipMemcpyAsync(r->out, s.d_out + s.h_desc[j].base, r->bases, hipMemcpyDeviceToHost, s.stream);
    if (e != hipSuccess) return std::string("copy to host: ") + hipGetErrorString(e);
  }
  e = hipEventRecord(s.done, s.stream);
  if (e != hipSuccess) return std::string("event: ") + hipGetErrorString(e);
  return "";
}

void finish(sbf_server *sv, std::vector<Request *> &reqs, int status, const std::string &err) {
  const int64_t t = now_ns();
  std::lock_guard<std::mutex> lk(sv->mu);
  for (Request *r : reqs) {
    r->t_done = t;
    r->state = kDone;
    r->status = status;
    r->error = err;
    if (status == SBF_OK) {
      sv->requests_done++;
      sv->bases_done += r->bases;
    }
  }
  reqs.clear();
  sv->cv_done.notify_all();
}

// Run one tiny batch on every slot (a poly-A record of 64 bases) from the
// scheduler thread: the first HIP calls of a thread and the first copies,
// kernels and event of a new stream carry one-time costs that would otherwise
// land on the first requests.
hipError_t warm_slots(sbf_server *sv) {
  hipError_t e = hipSuccess;
  for (Slot &s : sv->slots) {
    const uint64_t n = 64, back = std::min<uint64_t>(n, (sv->cap_records + 1) * sizeof(uint64_t));
    s.h_off[0] = 0;
    s.h_off[1] = n;
    s.h_desc[0] = CopyDesc{nullptr, nullptr, 0, n, n};
    e = hipMemsetAsync(s.d_seq, 'A', n, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.d_off, s.h_off, 2 * sizeof(uint64_t), hipMemcpyHostToDevice, s.stream);
    if (e == hipSuccess) e = launch_copy(true, s.dv_desc, 1, (uint8_t *)s.d_seq, s.stream);
    if (e == hipSuccess && (sbf_mark_record_starts_dev(s.dv_off, 1, n, s.d_starts, s.stream) != SBF_OK ||
                            sbf_query_marked_dev(sv->f, s.d_seq, n, s.d_starts, s.d_out, s.stream) != SBF_OK))
      e = hipErrorLaunchFailure;
    if (e == hipSuccess) e = launch_copy(false, s.dv_desc, 1, s.d_out, s.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s.h_off, s.d_out, back, hipMemcpyDeviceToHost, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
    if (e == hipSuccess) e = hipEventSynchronize(s.done);
    if (e != hipSuccess) break;
  }
  return e;
}

void scheduler(sbf_server *sv) {
  // The loop below polls busy slots with 5 us sleeps; Linux's default 50 us
  // timer slack would stretch each to ~57 us and delay every completion.
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
  hipError_t e = hipSetDevice(sv->device);
  if (e == hipSuccess) e = warm_slots(sv);
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->warm_error = e;
    sv->ready = true;
  }
  sv->cv_done.notify_all();
  if (e != hipSuccess) return;
  for (;;) {
    bool progress = false;
    bool any_busy = false;
    for (Slot &s : sv->slots) {
      if (!s.busy) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) {
        any_busy = true;
        continue;
      }
      finish(sv, s.reqs, q == hipSuccess ? SBF_OK : SBF_E_DEVICE,
             q == hipSuccess ? "" : std::string("batch: ") + hipGetErrorString(q));
      s.busy = false;
      progress = true;
    }
    for (Slot &s : sv->slots) {
      if (s.busy) continue;
      std::vector<Request *> batch;
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->pending.empty()) continue;
        if (sv->window_ns > 0 && !sv->stop && now_ns() - sv->pending.front()->t_submit < sv->window_ns) {
          // hold the slot for more requests unless the pending ones already fill it
          uint64_t b = 0, n = 0;
          bool fills = false;
          for (const Request *r : sv->pending) {
            if (b + r->bases > sv->cap_bases || n + r->nrec > sv->cap_records) {
              fills = true;
              break;
            }
            b += r->bases;
            n += r->nrec;
          }
          if (!fills) continue;
        }
        uint64_t bases = 0, recs = 0;
        while (!sv->pending.empty()) {
          Request *r = sv->pending.front();
          if (bases + r->bases > sv->cap_bases || recs + r->nrec > sv->cap_records) break;
          sv->pending.pop_front();
          bases += r->bases;
          recs += r->nrec;
          r->state = kRunning;
          batch.push_back(r);
        }
      }
      if (batch.empty()) continue;
      const int64_t t = now_ns();
      for (Request *r : batch) r->t_start = t;
      const std::string err = launch_batch(sv, s, batch);
      if (!err.empty()) {
        (void)hipStreamSynchronize(s.stream);
        finish(sv, batch, SBF_E_DEVICE, err);
        continue;
      }
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->batches++;
        if (batch.size() > sv->max_batch_requests) sv->max_batch_requests = batch.size();
      }
      s.reqs = std::move(batch);
      s.busy = true;
      any_busy = true;
      progress = true;
    }
    std::unique_lock<std::mutex> lk(sv->mu);
    if (!any_busy && sv->pending.empty()) {
      if (sv->stop) break;
      sv->cv_work.wait(lk, [sv] { return sv->stop || !sv->pending.empty(); });
    } else if (!progress) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(5));
    }
  }
}

}  // namespace

extern "C" {

sbf_server *sbf_server_create(sbf_filter *f, uint32_t slots, uint64_t slot_bases, uint64_t slot_records,
                              uint32_t max_pending) {
  if (!f || slots < 1 || slots > 16 || slot_bases < 1024 || slot_records < 1 || max_pending < 1) {
    fail(SBF_E_INVAL, "server needs a filter, 1..16 slots, >= 1024 bases and >= 1 record per slot");
    return nullptr;
  }
  sbf_server *sv = new (std::nothrow) sbf_server;
  if (!sv) {
    fail(SBF_E_NOMEM, "host allocation of the server");
    return nullptr;
  }
  sv->f = f;
  sv->cap_bases = slot_bases;
  sv->cap_records = slot_records;
  sv->max_pending = max_pending;
  hipError_t e = hipGetDevice(&sv->device);
  sv->slots.resize(slots);
  for (uint32_t i = 0; i < slots && e == hipSuccess; ++i) {
    Slot &s = sv->slots[i];
    e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    // room for up to 15 padding bases per request (a request has >= 1 record)
    const uint64_t room = slot_bases + 16 * (slot_records + 1);
    if (e == hipSuccess) e = hipMalloc((void **)&s.d_seq, room);
    if (e == hipSuccess) e = hipMalloc((void **)&s.d_out, room);
    if (e == hipSuccess) e = hipMalloc((void **)&s.d_off, (slot_records + 1) * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc((void **)&s.d_starts, (room + 31) / 32 * sizeof(uint32_t));
    if (e == hipSuccess) e = hipHostMalloc((void **)&s.h_off, (slot_records + 1) * sizeof(uint64_t), 0);
    if (e == hipSuccess) e = hipHostMalloc((void **)&s.h_desc, slot_records * sizeof(CopyDesc), 0);
    void *dv = nullptr;
    if (e == hipSuccess) e = hipHostGetDevicePointer(&dv, s.h_off, 0);
    if (e == hipSuccess) s.dv_off = (const uint64_t *)dv;
    if (e == hipSuccess) e = hipHostGetDevicePointer(&dv, s.h_desc, 0);
    if (e == hipSuccess) s.dv_desc = (const CopyDesc *)dv;
    // the filter's per-stream scratch for this slot, allocated now rather
    // than inside the first request
    if (e == hipSuccess && sbf::prepare_stream(f, s.stream) != SBF_OK) e = hipErrorOutOfMemory;
  }
  if (e != hipSuccess) {
    fail(e == hipErrorOutOfMemory ? SBF_E_NOMEM : SBF_E_DEVICE, std::string("server setup: ") + hipGetErrorString(e));
    for (Slot &s : sv->slots) release_slot(sv->f, s);
    delete sv;
    return nullptr;
  }
  try {
    sv->thread = std::thread(scheduler, sv);
  } catch (...) {
    fail(SBF_E_NOMEM, "scheduler thread");
    for (Slot &s : sv->slots) release_slot(sv->f, s);
    delete sv;
    return nullptr;
  }
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [sv] { return sv->ready; });
    e = sv->warm_error;
  }
  if (e != hipSuccess) {
    sv->thread.join();
    fail(SBF_E_DEVICE, std::string("server warm-up: ") + hipGetErrorString(e));
    for (Slot &s : sv->slots) release_slot(sv->f, s);
    delete sv;
    return nullptr;
  }
  succeed();
  return sv;
}

int sbf_server_set_batch_window(sbf_server *sv, uint64_t microseconds) {
  if (!sv || microseconds > 1000000) return fail(SBF_E_INVAL, "server needed; window at most 1 s");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->window_ns = (int64_t)microseconds * 1000;
  }
  return succeed();
}

int sbf_server_submit(sbf_server *sv, const char *seq, const uint64_t *off, uint64_t nrec, uint8_t *out,
                      uint64_t *ticket) {
  if (!sv || !off || !ticket || nrec == 0) return fail(SBF_E_INVAL, "server, offsets, ticket and records needed");
  if (off[0] != 0) return fail(SBF_E_INVAL, "off[0] must be 0");
  for (uint64_t r = 0; r < nrec; ++r)
    if (off[r + 1] < off[r]) return fail(SBF_E_INVAL, "offsets decrease");
  const uint64_t bases = off[nrec];
  if (bases && (!seq || !out)) return fail(SBF_E_INVAL, "sequence or output is NULL");
  if (bases > sv->cap_bases || nrec > sv->cap_records)
    return fail(SBF_E_INVAL, "request of " + std::to_string(bases) + " bases / " + std::to_string(nrec) +
                                 " records exceeds a slot (" + std::to_string(sv->cap_bases) + " / " +
                                 std::to_string(sv->cap_records) + ")");
  Request *r = new (std::nothrow) Request;
  if (!r) return fail(SBF_E_NOMEM, "host allocation of a request");
  r->seq = seq;
  r->off = off;
  r->nrec = nrec;
  r->out = out;
  r->bases = bases;
  r->direct_in = bases && device_view(seq);
  r->direct_out = bases && device_view(out);
  r->t_submit = now_ns();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
      delete r;
      return fail(SBF_E_INVAL, "server is stopping");
    }
    if (sv->pending.size() >= sv->max_pending) {
      delete r;
      return fail(SBF_E_BUSY, "pending queue is full");
    }
    r->id = sv->next_id++;
    sv->live[r->id] = r;
    if (bases == 0) {
      r->t_start = r->t_done = r->t_submit;
      r->state = kDone;
    } else {
      sv->pending.push_back(r);
    }
    *ticket = r->id;
  }
  sv->cv_work.notify_one();
  return succeed();
}

int sbf_server_poll(sbf_server *sv, uint64_t ticket) {
  if (!sv) return fail(SBF_E_INVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->live.find(ticket);
  if (it == sv->live.end()) return fail(SBF_E_INVAL, "unknown ticket");
  return it->second->state == kDone ? 1 : 0;
}

int sbf_server_wait(sbf_server *sv, uint64_t ticket, double *latency_ms, double *queue_ms) {
  if (!sv) return fail(SBF_E_INVAL, "server is NULL");
  Request *r;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) return fail(SBF_E_INVAL, "unknown ticket");
    r = it->second;
    sv->cv_done.wait(lk, [r] { return r->state == kDone; });
    sv->live.erase(it);
  }
  if (latency_ms) *latency_ms = (r->t_done - r->t_submit) * 1e-6;
  if (queue_ms) *queue_ms = (r->t_start - r->t_submit) * 1e-6;
  const int status = r->status;
  const std::string err = r->error;
  delete r;
  if (status != SBF_OK) return fail(status, err);
  return succeed();
}

int sbf_server_stats(sbf_server *sv, uint64_t *batches, uint64_t *requests, uint64_t *bases,
                     uint64_t *max_batch_requests) {
  if (!sv) return fail(SBF_E_INVAL, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (batches) *batches = sv->batches;
  if (requests) *requests = sv->requests_done;
  if (bases) *bases = sv->bases_done;
  if (max_batch_requests) *max_batch_requests = sv->max_batch_requests;
  return succeed();
}

void sbf_server_destroy(sbf_server *sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  if (sv->thread.joinable()) sv->thread.join();
  for (Slot &s : sv->slots) release_slot(sv->f, s);
  for (auto &kv : sv->live) delete kv.second;
  delete sv;
}

}  // extern "C"
