/*
 * sbf.h - C ABI of an MI355X (gfx950) Super Bloom filter for DNA k-mers.
 *
 * The filter is the sequence-native Super Bloom filter of "cuSBF: A
 * Minimizer-Aware Bloom Filter for Genomic Sequence Data on Modern GPUs":
 * every k-mer of a DNA sequence is sent to the shard picked by the low bits
 * of its minimizer hash (Section "Minimizers and Super-k-mers", Algorithm 1),
 * and inside that shard it is represented by its k-s+1 overlapping s-mers,
 * H bits each (Section "Findere Scheme").  A query answers 1 only when every
 * bit of every s-mer is set (Algorithm 2, Contains).
 *
 * Data layout (Section "Data Layout"): the filter owns one device array of
 * N = 2^P shards, N = next power of two of ceil(bits / 256), at least 1.
 * Shard i is the four 64-bit words at index 4i .. 4i+3; hash index t of an
 * s-mer sets one bit of word t mod 4.  Bit b of word w is (w >> b) & 1.  The
 * array starts zeroed.
 *
 * Alphabet: A/a=0, C/c=1, G/g=2, T/t=3; every other byte (N, separators,
 * padding) is invalid and no k-mer containing it is inserted; such k-mers
 * answer 0.  k-mers are read on the forward strand only.
 *
 * Conventions for every call:
 *   - A function returning int returns SBF_OK (0) or a negative SBF_E_*
 *     code, and records a message readable with sbf_last_error() on the
 *     calling thread.  No C++ exception crosses this boundary.
 *   - "Host" entry points take host pointers, first wait for all work on
 *     the device, run on the filter's own HIP stream and synchronise before
 *     returning (Section "Library Design").
 *   - "_dev" entry points take device pointers and a hipStream_t passed as
 *     void* (NULL = HIP's null stream); they are stream-ordered and do not
 *     synchronise.  The caller keeps the buffers alive until the work on
 *     that stream has finished.
 *   - The caller owns every sequence, offset and output buffer it passes; the
 *     library owns the filter's device array and its internal staging
 *     buffers.  A filter is used by one host thread at a time.
 */
#ifndef SBF_H
#define SBF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SBF_OK 0
#define SBF_E_INVAL (-1)  /* bad argument: parameters, NULL pointer, size */
#define SBF_E_NOMEM (-2)  /* a device or host allocation failed */
#define SBF_E_DEVICE (-3) /* a HIP call or kernel launch failed */
#define SBF_E_BUSY (-4)   /* a request was not admitted: the server's queue is full */

/* Kernel families (sbf_set_variant). */
#define SBF_VARIANT_AUTO 0    /* the fastest super-k-mer kernels for (k,s,m,H) and the shard size, else generic */
#define SBF_VARIANT_ROLLING 1 /* super-k-mer kernels: lane kernels for 4-word shards, wide-shard kernels for 8/16,
                                 run-time parameter kernels for other (k,s,m,H) */
#define SBF_VARIANT_GENERIC 2 /* one k-mer per lane, run-time k, s, m, H */
#define SBF_VARIANT_WIDE 3    /* wide-shard (two-phase, whole-line) super-k-mer kernels, also for 4-word shards */
#define SBF_VARIANT_PARAM 4   /* two-phase super-k-mer kernels with run-time k <= 32, s, m, H <= 8 (any shard size) */

typedef struct sbf_filter sbf_filter; /* opaque; owns its device bit array */

/* Create a filter (Section "Library Design": k, s, m and H configure the
 * filter; the total size in bits fixes the shard count).
 *   k: k-mer length, 1 <= k <= 32 (a k-mer packs into 64 bits).
 *   s: Findere s-mer length, 1 <= s <= k (k-s+1 s-mers per k-mer).
 *   m: minimizer length, 1 <= m <= k (k-m+1 m-mers per k-mer).
 *   H: bits per s-mer, 1 <= H <= 16; hash index t uses word t mod 4.
 *   bits: requested size, 1 <= bits <= 2^40; rounded up to 256 * 2^P.
 * Allocates and zeroes the device array on the current HIP device.
 * Returns NULL on error (SBF_E_INVAL for bad parameters, SBF_E_NOMEM when the
 * device allocation fails, SBF_E_DEVICE otherwise); nothing is left allocated
 * on failure. */
sbf_filter *sbf_create(uint32_t k, uint32_t s, uint32_t m, uint32_t H, uint64_t bits);

/* As sbf_create, with shards of shard_words 64-bit words (4, 8 or 16; the
 * paper's shard is 4 words = 256 bits, and sbf_create uses 4).  Hash index t
 * still writes sector t mod 4; a shard of S words holds S/4 groups of the
 * four sectors, and the group of index t is taken from the log2(S/4) bits of
 * the s-mer hash just above the t-th 6-bit bit address, which needs
 * 64/H >= 6 + log2(S/4) (H <= 9 for S = 8, H <= 8 for S = 16).  The shard
 * count is the power of two at or above ceil(bits / (64 S)).  Filters with
 * S = 8 or 16 run the wide-shard super-k-mer kernels where they are compiled
 * for (k, s, m, H), else the generic kernels; bits and answers differ from
 * S = 4, so S is part of the filter's definition, chosen at creation
 * (sbf_autotune_geometry measures it).  Errors as sbf_create. */
sbf_filter *sbf_create_ex(uint32_t k, uint32_t s, uint32_t m, uint32_t H, uint64_t bits, uint32_t shard_words);

/* Free the filter and its device memory after waiting for its stream.
 * sbf_destroy(NULL) does nothing. */
void sbf_destroy(sbf_filter *f);

/* Insert every valid k-mer of seq[0 .. len) (Algorithm 1).  Host pointer,
 * synchronous.  len < k inserts nothing and returns SBF_OK.  Repeated inserts
 * accumulate by OR. */
int sbf_insert_seq(sbf_filter *f, const char *seq, uint64_t len);

/* Query every k-mer of seq[0 .. len) (Algorithm 2).  out[i] (0 or 1) answers
 * the k-mer starting at seq[i], for i < len-k+1; invalid k-mers give 0.
 * Host pointers, synchronous.  len < k writes nothing.  The filter is not
 * modified. */
int sbf_query_seq(sbf_filter *f, const char *seq, uint64_t len, uint8_t *out);

/* Code and message of the last error on the calling thread (SBF_OK and ""
 * when the last call succeeded).  msg may be NULL.  The string stays valid
 * until the next call into the library on this thread. */
int sbf_last_error(const char **msg);

/* Geometry: number of shards N, filter size in bits (64 * S * N for shards
 * of S words: 256 * N for sbf_create) and number of 64-bit words (S * N).
 * 0 for a NULL filter. */
uint64_t sbf_num_shards(const sbf_filter *f);
uint64_t sbf_num_bits(const sbf_filter *f);
uint64_t sbf_num_words(const sbf_filter *f);

/* Copy the whole bit array to host_dst (nwords must equal sbf_num_words), or
 * overwrite it from host_src.  Both wait for all work on the device first.
 * Together with the parameters this is the full state of the filter, so
 * get + create + set restores it bit for bit. */
int sbf_get_bits(const sbf_filter *f, uint64_t *host_dst, uint64_t nwords);
int sbf_set_bits(sbf_filter *f, const uint64_t *host_src, uint64_t nwords);

/* Zero the bit array, ordered on stream (NULL = HIP's null stream); does
 * not synchronise. */
int sbf_clear(sbf_filter *f, void *stream);

/* Load statistics (Section "False Positive Rate"; Eq. 1 per sector and Eq. 2
 * across the k-s+1 s-mers): *fpr receives the false-positive rate expected
 * for k-mers absent from the filter whose shard is uniform over the shards
 * and whose s-mers hash independently and ideally, i.e. the mean over shards
 * of the product over sectors c of p_c^((k-s+1) n_c), with p_c the fraction of
 * set bits in the shard's words of sector c and n_c the hash indices t < H
 * with t mod 4 = c; *set_bits receives the number of set bits.  Either
 * pointer may be NULL (not both).  Waits for all work on the device first;
 * synchronous.  It reads the bit array only. */
int sbf_estimate_fpr(const sbf_filter *f, double *fpr, uint64_t *set_bits);

/* Device pointer of the bit array (S * N words).  Valid until sbf_destroy. */
const uint64_t *sbf_device_words(const sbf_filter *f);

/* Stream-ordered forms of sbf_insert_seq / sbf_query_seq on device memory
 * (Section "Library Design": device-facing entry points leave ordering to the
 * caller).  d_out has room for len-k+1 bytes. */
int sbf_insert_seq_dev(sbf_filter *f, const char *d_seq, uint64_t len, void *stream);
int sbf_query_seq_dev(sbf_filter *f, const char *d_seq, uint64_t len, uint8_t *d_out,
                      void *stream);

/* Record batches (Section "Sequence-Native Design": records are concatenated
 * and no k-mer spans two records).  Record r is seq[off[r] .. off[r+1]);
 * off has nrec+1 non-decreasing entries with off[0] = 0.  Queries write one
 * byte per base position, out[0 .. off[nrec]): out[off[r]+i] answers k-mer i
 * of record r; the last k-1 positions of each record, and every position of
 * a record shorter than k, are 0.
 * Host form: host pointers, validated, synchronous. */
int sbf_insert_batch(sbf_filter *f, const char *seq, const uint64_t *off, uint64_t nrec);
int sbf_query_batch(sbf_filter *f, const char *seq, const uint64_t *off, uint64_t nrec,
                    uint8_t *out);

/* Device form: d_seq holds len = off[nrec] bases, d_off is a device array of
 * nrec+1 offsets (not read by the host, so it is not validated: off[0] must
 * be 0 and off[nrec] must equal len).  Stream-ordered.  The library keeps one
 * scratch buffer of len/8 bytes per stream used (record starts as bits).
 * Queries on different streams may overlap one another; inserts into one
 * filter must not overlap another insert under SBF_INSERT_TWO_PASS (a store
 * of one could undo a bit the other has already repaired): order them
 * on one stream or with events, or use SBF_INSERT_ATOMIC. */
int sbf_insert_batch_dev(sbf_filter *f, const char *d_seq, uint64_t len, const uint64_t *d_off,
                         uint64_t nrec, void *stream);
int sbf_query_batch_dev(sbf_filter *f, const char *d_seq, uint64_t len, const uint64_t *d_off,
                        uint64_t nrec, uint8_t *d_out, void *stream);

/* Allocation-free form of sbf_query_batch_dev, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * hosts that forbid hipMalloc): same arguments, layout and answers, and it
 * calls no hipMalloc, hipFree or other allocating routine.  Its scratch (the
 * record-start bits and the work-queue counters) is one fixed array of 8 MiB
 * per GPU, held until the process ends, so a batch may have at most 2^26
 * bases (len > 2^26 returns SBF_E_INVAL).  The array is shared by every call
 * on that GPU, whatever the filter or stream: calls that overlap on one GPU
 * (on different streams, or from several host threads) race and must be
 * ordered by the caller.  The scratch is cleared by fill kernels on `stream`
 * (no memset), and the filter's launch settings apply.  Stream-ordered. */
int sbf_query_batch_dev_noalloc(sbf_filter *f, const char *d_seq, uint64_t len, const uint64_t *d_off,
                                uint64_t nrec, uint8_t *d_out, void *stream);

/* The two steps of the device batch form, for callers that reuse one batch
 * or time the kernels apart.  sbf_mark_record_starts_dev zeroes d_starts
 * (ceil(len/32) words) and sets bit off[r] % 32 of word off[r] / 32 for
 * r = 1 .. nrec-1.  The _marked calls then insert or query d_seq[0 .. len)
 * as the record batch those bits describe (d_starts may be NULL for a single
 * record; queries write len bytes).  Stream-ordered. */
int sbf_mark_record_starts_dev(const uint64_t *d_off, uint64_t nrec, uint64_t len, uint32_t *d_starts,
                               void *stream);
int sbf_insert_marked_dev(sbf_filter *f, const char *d_seq, uint64_t len, const uint32_t *d_starts,
                          void *stream);
int sbf_query_marked_dev(sbf_filter *f, const char *d_seq, uint64_t len, const uint32_t *d_starts,
                         uint8_t *d_out, void *stream);

/* Choose the kernel family (SBF_VARIANT_*).  SBF_VARIANT_ROLLING,
 * SBF_VARIANT_WIDE and SBF_VARIANT_PARAM fail with SBF_E_INVAL when no such
 * kernel exists for the filter's (k,s,m,H) and shard size (the wide-shard
 * kernels are compiled for a few parameter sets; the run-time parameter
 * kernels take k <= 32 and H <= 8).  Every family gives bit-identical
 * filters and answers.  Changing the family resets the tile lengths
 * (sbf_set_tile) to the new family's defaults. */
int sbf_set_variant(sbf_filter *f, int variant);
/* The family in effect: SBF_VARIANT_ROLLING (4-word lane kernels),
 * SBF_VARIANT_WIDE, SBF_VARIANT_PARAM or SBF_VARIANT_GENERIC. */
int sbf_get_variant(const sbf_filter *f);

/* Tile size of the super-k-mer kernels, as k-mers per lane (a tile is 256
 * lanes of them; with about 8.5 k-mers per super-k-mer, Section "Minimizers
 * and Super-k-mers", that is the tile's super-k-mer count times 8.5 / 256).
 * 0 selects the family's default.  Compiled lengths:
 *   4-word lane kernels, (31,28,16,4) only: insert 64 or 32 k-mers per lane
 *     for the store pass (default: 64 for an insert call of at least 2^24
 *     k-mers, 32 below; other sets: 32 only); query 48 (default) or 32,
 *     which the insert's repair walk uses as well;
 *   wide-shard kernels: 16 (default) or 32 for insert and query;
 *   run-time parameter kernels: 8 (default) or 16 for insert and query.
 * Other values (and any value for the generic kernels) return SBF_E_INVAL.
 * The result does not depend on the tile size.  sbf_get_tile reads the
 * effective lengths back (0 for the generic kernels; pointers may be NULL;
 * the lane kernels' size-dependent insert default reads as 64). */
int sbf_set_tile(sbf_filter *f, uint32_t insert_kmers_per_lane, uint32_t query_kmers_per_lane);
int sbf_get_tile(const sbf_filter *f, uint32_t *insert_kmers_per_lane, uint32_t *query_kmers_per_lane);

/* How the rolling insert kernel writes finished super-k-mer segments:
 *   SBF_INSERT_TWO_PASS (default): a pass of read-OR-write updates of each
 *     segment's shard (stores that write through to the device's coherence
 *     point, so that racing updates only drop each other's bits), then a
 *     second pass over the same segments that atomically ORs back any bit a
 *     concurrent update overwrote;
 *   SBF_INSERT_ATOMIC: one 64-bit atomic OR per shard word, as in the paper's
 *     Algorithm 1.
 * Both produce the same filter; the generic kernel always uses atomics. */
#define SBF_INSERT_TWO_PASS 0
#define SBF_INSERT_ATOMIC 1
int sbf_set_insert_mode(sbf_filter *f, int mode);

/* How the rolling query kernel is organised:
 *   SBF_QUERY_LANE (default): each lane walks 48 consecutive k-mers, builds
 *     the mask of each k-mer's (k-s+1)*H bits from its s-mers and tests it
 *     one k-mer later against the k-mer's shard, which the lane loads only
 *     where the shard changes (once per super-k-mer);
 *   SBF_QUERY_LEADER: a first pass stores shards and bit addresses in LDS, a
 *     second tests one k-mer per lane; the first lane of each run of equal
 *     shards loads the 32-byte shard and the run's other lanes receive it by
 *     a cross-lane permute (Algorithm 2's leader load and shuffle);
 *   SBF_QUERY_DIRECT: as SBF_QUERY_LEADER, but every valid lane loads.
 * All three give the same answers. */
#define SBF_QUERY_LANE 0
#define SBF_QUERY_LEADER 1
#define SBF_QUERY_DIRECT 2
int sbf_set_query_mode(sbf_filter *f, int mode);

/* Launch shape of the rolling kernels: 0 workgroups per CU launches one
 * workgroup per tile; n > 0 launches a persistent grid of n workgroups per
 * compute unit that take tiles from a device work-queue counter until the
 * batch is done.  Insert and query are set separately (n <= 32; default 4
 * for both, the fastest measured shape).  The
 * counters live per stream, so persistent calls on one stream are ordered;
 * sbf_get_launch reads the settings back (any pointer may be NULL). */
int sbf_set_launch(sbf_filter *f, uint32_t insert_wgs_per_cu, uint32_t query_wgs_per_cu);
int sbf_get_launch(const sbf_filter *f, uint32_t *insert_wgs_per_cu, uint32_t *query_wgs_per_cu, int *insert_mode,
                   int *query_mode);

/* Batched form: capture, once, a HIP graph that optionally clears the filter,
 * marks the record starts of an insert batch and of a query batch, inserts
 * the first and queries the second (device batches as in
 * sbf_insert_batch_dev / sbf_query_batch_dev; either may be NULL), with the
 * kernel organisation and launch shape in effect at creation.  The graph
 * owns its scratch (record-start bits, work-queue counters) and refers to
 * the caller's buffers and to f, which must outlive it.  sbf_graph_launch
 * replays it on stream (NULL = HIP's null stream); replays on one stream are
 * ordered, replays on different streams must not overlap.  Returns NULL on
 * error (see sbf_last_error). */
typedef struct sbf_graph sbf_graph;
sbf_graph *sbf_graph_create(sbf_filter *f, int clear_first, const char *d_ins, uint64_t ins_len,
                            const uint64_t *d_ins_off, uint64_t ins_nrec, const char *d_q, uint64_t q_len,
                            const uint64_t *d_q_off, uint64_t q_nrec, uint8_t *d_out);
int sbf_graph_launch(sbf_graph *g, void *stream);
void sbf_graph_destroy(sbf_graph *g);

/* Autotuner: on the given device insert and query batches, time every insert
 * strategy, query organisation and compiled tile length (sbf_set_tile) with
 * one workgroup per tile and with persistent grids of 1, 2, 4 and 8
 * workgroups per CU (median of three runs after a warm-up) on f itself, whose
 * words are first saved to a temporary device buffer of the filter's size
 * and restored afterwards (f's contents are unchanged; the buffer must fit in
 * device memory), then apply the fastest settings to f.  A text report of
 * every timing is written to report (NUL-terminated, truncated to
 * report_len; may be NULL).  Synchronous. */
int sbf_autotune(sbf_filter *f, const char *d_ins, uint64_t ins_len, const uint64_t *d_ins_off, uint64_t ins_nrec,
                 const char *d_q, uint64_t q_len, const uint64_t *d_q_off, uint64_t q_nrec, char *report,
                 uint64_t report_len);

/* Shard-geometry autotuner (Section "Data Layout": the shard is sized to the
 * memory system).  For shards of 4, 8 and 16 words (those valid for H), it
 * creates a filter of the given parameters and size on the current device,
 * runs sbf_autotune on it with the insert and query device batches (record
 * batches as in sbf_insert_batch_dev), then inserts the insert batch and
 * measures the false-positive rate on the negative batch (k-mers answered
 * present over its valid k-mers; every valid k-mer of a full filter answers
 * present, which counts them).  It returns the geometry with the lowest
 * insert + query time among those whose FPR is at most max_fpr, or, if none
 * is, the one with the lowest FPR, in *shard_words (required) with its tuned
 * tile lengths and its FPR (optional outputs, may be NULL).  The shard size
 * changes the filter's bits, so the caller creates its filter with it
 * (sbf_create_ex).  A report of every trial is written to report as in
 * sbf_autotune.  Synchronous; each trial filter is freed before the next. */
int sbf_autotune_geometry(uint32_t k, uint32_t s, uint32_t m, uint32_t H, uint64_t bits, const char *d_ins,
                          uint64_t ins_len, const uint64_t *d_ins_off, uint64_t ins_nrec, const char *d_q,
                          uint64_t q_len, const uint64_t *d_q_off, uint64_t q_nrec, const char *d_neg,
                          uint64_t neg_len, const uint64_t *d_neg_off, uint64_t neg_nrec, double max_fpr,
                          uint32_t *shard_words, uint32_t *insert_kmers_per_lane, uint32_t *query_kmers_per_lane,
                          double *fpr, char *report, uint64_t report_len);

/* Served form: a request loop over a resident filter with continuous
 * batching.  The server runs a scheduler thread with `slots` execution slots
 * (1..16), each a HIP stream with device staging for slot_bases bases and
 * slot_records records (the memory budget is slots x (2 x slot_bases +
 * slot_bases/8 + 8 x slot_records) bytes).  Whenever a slot is free, it
 * admits the pending requests in arrival order while they fit the slot,
 * joins them into one record batch, and runs copy-in, record-start marking,
 * the query kernel and copy-out on the slot's stream; later requests join
 * the next free slot, so batches overlap on the device.  While a server
 * exists, use the filter only through it (queries) or after destroying it.
 *
 * sbf_server_set_batch_window: hold a free slot up to `microseconds` (at
 * most 1 s; default 0) after the oldest pending request arrived, unless the
 * pending requests already fill the slot, so that more requests join one
 * batch: larger batches for up to that much added latency.
 * sbf_server_submit: one query request, a record batch in host memory (seq,
 * off with nrec+1 entries, off[0] = 0; out receives off[nrec] bytes as in
 * sbf_query_batch).  The buffers must stay valid and unchanged until the
 * request completes; pinned host memory lets the copies run asynchronously.
 * Returns a ticket.  SBF_E_INVAL if the request cannot fit one slot,
 * SBF_E_BUSY if max_pending requests are already waiting.
 * sbf_server_poll: 1 when the request is done, 0 while it is not.
 * sbf_server_wait: block until done, release the ticket, and report the
 * latency from submission to answers in host memory and the part spent
 * waiting for admission (either pointer may be NULL); returns the request's
 * status.
 * sbf_server_stats: batches run, requests and bases answered, and the most
 * requests joined in one batch.
 * sbf_server_destroy: finish every admitted and pending request, then free
 * the server. */
typedef struct sbf_server sbf_server;
sbf_server *sbf_server_create(sbf_filter *f, uint32_t slots, uint64_t slot_bases, uint64_t slot_records,
                              uint32_t max_pending);
int sbf_server_set_batch_window(sbf_server *sv, uint64_t microseconds);
int sbf_server_submit(sbf_server *sv, const char *seq, const uint64_t *off, uint64_t nrec, uint8_t *out,
                      uint64_t *ticket);
int sbf_server_poll(sbf_server *sv, uint64_t ticket);
int sbf_server_wait(sbf_server *sv, uint64_t ticket, double *latency_ms, double *queue_ms);
int sbf_server_stats(sbf_server *sv, uint64_t *batches, uint64_t *requests, uint64_t *bases,
                     uint64_t *max_batch_requests);
void sbf_server_destroy(sbf_server *sv);

/* Bytes of sequence per chunk of the host entry points (default 64 MiB; at
 * least 4096).  Inputs longer than this are processed in chunks that overlap
 * by k-1 bases, pipelined over two HIP streams: while one chunk's kernel
 * runs, the next chunk is copied into pinned host memory and sent to the
 * device, and the previous chunk's answers come back.  With the lane query
 * (SBF_QUERY_LANE, the default) answers cross the host link as one bit per
 * k-mer and are spread to bytes on the host (the k-mer starts per chunk are
 * then rounded down to a multiple of 64).  A caller buffer that is already
 * pinned (hipHostMalloc, torch pin_memory) is copied from directly, and for
 * byte answers copied to directly.  The library holds up to two chunks of
 * device and pinned host memory (plus the answers for queries) until the
 * filter is destroyed. */
int sbf_set_staging_bytes(sbf_filter *f, uint64_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* SBF_H */
