/*
 * sbf_probe.h - micro-benchmarks that set the memory rooflines of the SBF
 * kernels on the current GPU (library libsbf_probe.so).
 *
 * The insert and query kernels touch one 32-byte shard per super-k-mer
 * segment at a random place in the filter (Section "Data Layout": 256-bit
 * shards; Section "Speed-of-Light Analysis": DRAM pressure once the filter
 * outgrows the caches).  These probes measure how many such random shard
 * accesses per second the device sustains over a buffer of a given size, plus
 * a streaming copy of known size used to calibrate hardware byte counters.
 */
#ifndef SBF_PROBE_H
#define SBF_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBF_PROBE_READ32 0     /* read one random 32-byte shard (two 16-byte loads) */
#define SBF_PROBE_RMW32 1      /* read a random shard, OR a bit, write it back (plain) */
#define SBF_PROBE_ATOMIC4 2    /* four 64-bit atomic ORs on one random shard */
#define SBF_PROBE_ATOMIC1 3    /* one 64-bit atomic OR on one random shard */
#define SBF_PROBE_COPY 4       /* streaming copy of bytes/2 bytes within the buffer */

/* Run probe `mode` over a device buffer of `bytes` bytes (a power of two,
 * 64 KiB .. 64 GiB; allocated, zeroed and freed by the call) on the current
 * device.  For the random modes, `ops` shard operations are issued (at
 * least 2^20); for SBF_PROBE_COPY, ops is ignored.  On success writes the
 * rate to *per_second (shard operations/s, or bytes moved/s counting read
 * plus write for the copy) and the mean kernel time to *ms, and returns 0;
 * returns -1 for bad arguments, -2 when the allocation fails, -3 on a HIP
 * error.  Each measurement is the mean of three launches after one warm-up
 * launch. */
int sbf_probe_random_access(uint64_t bytes, int mode, uint64_t ops, double *per_second, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* SBF_PROBE_H */
