/*
 * sbf_probe.h - micro-benchmarks that set the memory and integer-ALU
 * rooflines of the SBF kernels on the current GPU (library libsbf_probe.so).
 *
 * The insert and query kernels touch one 32-byte shard per super-k-mer
 * segment at a random place in the filter (Section "Data Layout": 256-bit
 * shards; Section "Speed-of-Light Analysis": DRAM pressure once the filter
 * outgrows the caches).  These probes measure how many such random shard
 * accesses per second the device sustains over a buffer of a given size, with
 * many independent accesses in flight per lane and a sweep of occupancy, so
 * that the best setting is a ceiling for the kernels; plus a streaming copy of
 * known size used to calibrate hardware byte counters.
 */
#ifndef SBF_PROBE_H
#define SBF_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBF_PROBE_READ 0     /* read one random shard (16-byte loads) */
#define SBF_PROBE_RMW 1      /* read a random shard, OR a bit, write it back (plain) */
#define SBF_PROBE_ATOMIC4 2  /* four 64-bit atomic ORs on one random shard */
#define SBF_PROBE_ATOMIC1 3  /* one 64-bit atomic OR on one random shard */
#define SBF_PROBE_COPY 4     /* streaming copy of bytes/2 bytes within the buffer */
#define SBF_PROBE_READ_LINE 5 /* as READ, the shard split over shard_bytes/16 lanes (one 16-byte piece each) */
#define SBF_PROBE_RMW_LINE 6  /* as RMW, the shard split over shard_bytes/16 lanes */
#define SBF_PROBE_RMW_COHERENT 7      /* as RMW, the stores writing through to the coherence point (sc0 sc1) */
#define SBF_PROBE_RMW_LINE_COHERENT 8 /* as RMW_LINE with those stores */

/* Run probe `mode` over a device buffer of `bytes` bytes (a power of two,
 * 64 KiB .. 64 GiB; allocated, zeroed and freed by the call) on the current
 * device.
 *   shard_bytes: 32, 64 or 128 (the filter's shard of 4, 8 or 16 words);
 *   inflight: shards each lane addresses before it uses any of them, so that
 *     inflight * shard_bytes / 16 loads are in flight per lane: 1, 4, 8 or 16
 *     for 32-byte shards, 1, 4 or 8 for 64, 1, 2 or 4 for 128;
 *   wgs_per_cu: 256-lane workgroups launched per compute unit (1 .. 16), each
 *     running its share of the operations (waves per SIMD = wgs_per_cu when
 *     registers allow);
 *   ops: shard operations to issue, at least 2^20 (rounded up to whole
 *     batches of the grid).
 * For SBF_PROBE_COPY only bytes is used.  On success writes the rate to
 * *per_second (shard operations/s, or bytes moved/s counting read plus write
 * for the copy) and the mean kernel time to *ms, and returns 0; returns -1 for
 * bad arguments, -2 when the allocation fails, -3 on a HIP error.  Each
 * measurement is the mean of three launches after one warm-up launch. */
int sbf_probe_random_access(uint64_t bytes, int mode, uint32_t shard_bytes, uint32_t inflight, uint32_t wgs_per_cu,
                            uint64_t ops, double *per_second, double *ms);

/* Integer vector-ALU issue rates behind the in-cache roofline (Section
 * "Speed-of-Light Analysis": in cache the kernels are compute-bound).  Each
 * probe runs one instruction kind in eight independent chains per lane over
 * a grid of 8192 waves; the instructions are those the hashing, sliding
 * minimum and mask tests of the kernels compile to. */
#define SBF_PROBE_VALU_ADD32 0   /* v_add_u32: 32-bit add */
#define SBF_PROBE_VALU_MUL32 1   /* v_mul_lo_u32: low half of a 32x32-bit product */
#define SBF_PROBE_VALU_MAD64 2   /* v_mad_u64_u32: 32x32-bit product plus a 64-bit addend */
#define SBF_PROBE_VALU_SHL64 3   /* v_lshlrev_b64: 64-bit shift */
#define SBF_PROBE_VALU_BITOP3 4  /* v_bitop3_b32: three-input bitwise function */
#define SBF_PROBE_VALU_CMP64 5   /* v_cmp_lt_u64: 64-bit compare into a lane mask */

/* Run VALU probe `op` on the current device.  On success writes the rate in
 * wave-level instructions per second to *wave_instr_per_second and the mean
 * kernel time to *ms and returns 0; -1 for a bad op, -2 when a small device
 * allocation fails, -3 on a HIP error.  Mean of three launches after one
 * warm-up launch. */
int sbf_probe_valu(int op, double *wave_instr_per_second, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* SBF_PROBE_H */
