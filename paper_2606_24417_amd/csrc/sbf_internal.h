// Host-side interface between the C ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

struct sbf_filter;

namespace sbf {

struct Geometry {
  uint32_t k, s, m, H;
  uint32_t shard_words;  // 64-bit words per shard (4 = the paper's 256-bit shard)
  uint64_t nshards;      // power of two, at most 2^32
};

// One launch over a device sequence.  Insert: every valid k-mer starting in
// [0, len-k+1).  Query: out[i] for i in [0, n_out) (k-mers that leave the
// sequence or cross a record start are invalid and answer 0).
struct SeqArgs {
  const uint8_t *seq;
  uint64_t len;
  const uint32_t *starts;  // record-start bits (1 bit per base) or null
  uint8_t *out;            // query only
  uint64_t n_out;          // query only
  // query only: out holds one bit per k-mer start (bit i%8 of byte i/8), ceil(n_out/8) bytes;
  // supported by the lane-sequential rolling query only (query_packed_supported)
  int packed = 0;
};

// Insert strategies of the rolling kernels: two passes (plain read-modify-write,
// then an atomic repair of lost bits) or one atomic OR per shard word.
constexpr int kInsertTwoPassMode = 0;
constexpr int kInsertAtomicMode = 1;

// Rolling query kernels: lane-sequential (each lane tests its own run of
// k-mers), or two phases with one k-mer per lane in the second, where the
// first lane of each run of equal shards loads and broadcasts (leader) or
// every lane loads (direct).
constexpr int kQueryLaneMode = 0;
constexpr int kQueryLeaderMode = 1;
constexpr int kQueryDirectMode = 2;

// Rolling kernels exist for a few compiled parameter sets.
bool rolling_supported(const Geometry &g);
// Query organisations that can write answers as bits (SeqArgs::packed).
inline bool query_packed_supported(int mode) { return mode == kQueryLaneMode; }

// Launch shape of the rolling kernels: one workgroup per tile, or a
// persistent grid of persistent_wgs workgroups that take tiles from device
// counters (queue: three u32 work-queue counters, one per pass).
struct LaunchShape {
  uint32_t *queue;
  uint32_t persistent_wgs;
  // k-mers per lane of the insert and query tiles (0: the kernel family's
  // default; the compiled lengths are listed by lane_len_supported)
  uint32_t insert_lane_len = 0;
  uint32_t query_lane_len = 0;
};

hipError_t launch_insert_rolling(const Geometry &g, uint64_t *words, const SeqArgs &a, int mode,
                                 const LaunchShape &ls, hipStream_t st);
hipError_t launch_query_rolling(const Geometry &g, const uint64_t *words, const SeqArgs &a, int mode,
                                const LaunchShape &ls, hipStream_t st);
// Wide-shard kernels (kernels_wide.hip): shards of 4, 8 or 16 words for a
// few compiled parameter sets; query answers as bytes only.
bool wide_supported(const Geometry &g);
hipError_t launch_insert_wide(const Geometry &g, uint64_t *words, const SeqArgs &a, int mode, const LaunchShape &ls,
                              hipStream_t st);
hipError_t launch_query_wide(const Geometry &g, const uint64_t *words, const SeqArgs &a, const LaunchShape &ls,
                             hipStream_t st);
// Run-time parameter super-k-mer kernels (kernels_param.hip): any (k, s, m, H)
// with m <= k <= 32, s <= k, H <= 8 and shards of 4, 8 or 16 words; query
// answers as bytes only.
bool param_supported(const Geometry &g);
hipError_t launch_insert_param(const Geometry &g, uint64_t *words, const SeqArgs &a, int mode, const LaunchShape &ls,
                               hipStream_t st);
hipError_t launch_query_param(const Geometry &g, const uint64_t *words, const SeqArgs &a, const LaunchShape &ls,
                              hipStream_t st);
hipError_t launch_insert_generic(const Geometry &g, uint64_t *words, const SeqArgs &a, hipStream_t st);
hipError_t launch_query_generic(const Geometry &g, const uint64_t *words, const SeqArgs &a, hipStream_t st);

// Record the calling thread's last error (code and message) for
// sbf_last_error; returns code.
int record_error(int code, const char *msg);

// Allocate now the per-stream scratch a filter's launches on `stream` would
// otherwise allocate on first use (work-queue counters), so that a latency-
// sensitive caller does not pay a device allocation inside a request; and
// free it when the stream goes away.
int prepare_stream(sbf_filter *f, hipStream_t stream);
void release_stream(sbf_filter *f, hipStream_t stream);

// Utility kernels.
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t st);
hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t value, hipStream_t st);
// Add the number of nonzero bytes of p[0, n) to the device counter *count.
hipError_t launch_count_nonzero_u8(const uint8_t *p, uint64_t n, uint64_t *count, hipStream_t st);
// Add to *sum, over shards, the probability that a k-mer of ideal hashes
// sent to the shard finds all its bits set, and to *bits the set bits.
hipError_t launch_estimate_fpr(const Geometry &g, const uint64_t *words, double *sum, uint64_t *bits,
                               hipStream_t st);
// Set bit off[r] of `starts` for r = 1 .. nrec-1 (starts must be zeroed;
// ceil(len/32) words).
hipError_t launch_mark_record_starts(const uint64_t *off, uint64_t nrec, uint64_t len, uint32_t *starts,
                                     hipStream_t st);

}  // namespace sbf
