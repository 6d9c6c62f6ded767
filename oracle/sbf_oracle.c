/*
 * CPU oracle for the Super Bloom filter (SBF) sequence-native insert and
 * query path of "cuSBF: A Minimizer-Aware Bloom Filter for Genomic Sequence
 * Data on Modern GPUs".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, per-k-mer
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header or constant table with the GPU library; it reads its inputs
 * as plain byte arrays.
 *
 * Every k-mer is handled on its own, exactly in the order of the paper's
 * Algorithm 1 (insert) and Algorithm 2 (query): pack the k-mer, take the
 * minimum minimizer hash over its k-m+1 m-mers, pick the shard from the low
 * bits of that minimum, then walk the k-s+1 s-mers and their H bit addresses.
 * No grouping into super-k-mers, no rolling hashes and no segmented
 * reductions: those are the GPU's business, and OR is commutative and
 * idempotent, so they cannot change the result.
 *
 * Readings where the paper is silent (each one listed with its reason in the
 * design notes of the repository):
 *   - base codes A/a=0, C/c=1, G/g=2, T/t=3, every other byte invalid
 *     (paper: 2 bits per base, a separator such as N is invalid);
 *   - forward strand only (the algorithms hash the packed k-mer directly);
 *   - the first base of a window is the most significant symbol;
 *   - minimizer hash: one multiply by floor(2^64/phi) (Fibonacci hashing);
 *   - s-mer hash: the first xorshift-multiply round of the SplitMix64
 *     finaliser followed by its closing xorshift-31;
 *   - bit address: the low 6 bits of slice t when 64/H >= 6, else the top 6
 *     bits of the hash times a golden-ratio salt;
 *   - shard count: next power of two of ceil(bits / shard bits), at least 1.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>

#define ORC_MINIMIZER_MUL 0x9E3779B97F4A7C15ULL /* floor(2^64 / golden ratio) */
#define ORC_SMER_MUL 0xBF58476D1CE4E5B9ULL      /* SplitMix64 first multiplier */

/* ---------------------------------------------------------------------------
 * Alphabet (Section "Library Design": DNA uses 2 bits per base; Section
 * "Sequence-Native Design": a separator such as N is an invalid symbol).
 * Returns 0..3, or -1 for an invalid byte.
 * ------------------------------------------------------------------------- */
int orc_base_code(unsigned char c)
{
    switch (c) {
    case 'A': case 'a': return 0;
    case 'C': case 'c': return 1;
    case 'G': case 'g': return 2;
    case 'T': case 't': return 3;
    default: return -1;
    }
}

/* Minimizer hash (Section "Optimizations", role-specialised hashing: a single
 * multiplicative mix). */
uint64_t orc_hash_minimizer(uint64_t y)
{
    return y * ORC_MINIMIZER_MUL;
}

/* s-mer hash (Section "Optimizations": a stronger mix with an additional
 * xorshift). */
uint64_t orc_hash_smer(uint64_t v)
{
    uint64_t u = (v ^ (v >> 30)) * ORC_SMER_MUL;
    return u ^ (u >> 31);
}

/* Bit address of hash index t inside its 64-bit sector (Section
 * "Optimizations", bit-slicing and the salted fallback for narrow slices). */
uint32_t orc_bit_address(uint64_t g, uint32_t t, uint32_t H)
{
    uint32_t W = 64u / H;
    if (W >= 6u)
        return (uint32_t)((g >> (t * W)) & 63u);
    uint64_t salt = ORC_MINIMIZER_MUL * (2ULL * t + 1ULL);
    return (uint32_t)((g * salt) >> 58);
}

/* Word of the shard that hash index t updates (Section "Data Layout": hash
 * index t goes to sector t mod 4).  shard_words S = 4 is the paper's 256-bit
 * shard; S = 8 or 16 spreads the same four sectors over S/4 groups, choosing
 * the group from the bits just above the bit address. */
uint32_t orc_word_index(uint64_t g, uint32_t t, uint32_t H, uint32_t S)
{
    uint32_t groups = S / 4u;
    uint32_t group = 0;
    if (groups > 1u) {
        uint32_t W = 64u / H;
        group = (uint32_t)((g >> (t * W + 6u)) % groups);
    }
    return (t % 4u) + 4u * group;
}

/* Shard count (Section "Data Layout": 2^P shards, the count rounded up to a
 * power of two so that the shard index is a bitwise AND). */
uint64_t orc_num_shards(uint64_t bits, uint32_t S)
{
    uint64_t per = 64ULL * S;
    uint64_t need = bits / per + ((bits % per) != 0);
    uint64_t n = 1;
    if (need < 1)
        need = 1;
    while (n < need)
        n <<= 1;
    return n;
}

/* Pack L bases starting at x into an integer, first base most significant.
 * Returns 0 on an invalid base (ValidKmer / PackKmer of Algorithm 1). */
int orc_pack(const unsigned char *x, uint32_t L, uint64_t *out)
{
    uint64_t v = 0;
    for (uint32_t j = 0; j < L; j++) {
        int c = orc_base_code(x[j]);
        if (c < 0)
            return 0;
        v = (v << 2) | (uint64_t)c;
    }
    *out = v;
    return 1;
}

/* The L-mer at offset j of a packed k-mer (Subwindow of Algorithms 1 and 2):
 * equal to packing bases j .. j+L-1 of the k-mer. */
uint64_t orc_subwindow(uint64_t K, uint32_t k, uint32_t L, uint32_t j)
{
    uint64_t shifted = K >> (2u * (k - L - j));
    if (L >= 32u)
        return shifted;
    return shifted & ((1ULL << (2u * L)) - 1ULL);
}

/* Minimum minimizer hash over the k-m+1 m-mers of a packed k-mer (the
 * minimizer loop of Algorithms 1 and 2; only the minimum value is used). */
uint64_t orc_min_hash(uint64_t K, uint32_t k, uint32_t m)
{
    uint64_t best = UINT64_MAX;
    for (uint32_t i = 0; i + m <= k; i++) {
        uint64_t h = orc_hash_minimizer(orc_subwindow(K, k, m, i));
        if (h < best)
            best = h;
    }
    return best;
}

typedef struct {
    uint32_t k, s, m, H, S; /* S = 64-bit words per shard */
    uint64_t nshards;
} orc_params;

static uint64_t shard_of(const orc_params *p, uint64_t K)
{
    return orc_min_hash(K, p->k, p->m) & (p->nshards - 1ULL);
}

/* Set one bit of a filter word.  With `shared` the OR is atomic (relaxed), so
 * that several threads may insert into one filter at once; OR is commutative
 * and idempotent, so the result does not depend on their interleaving. */
static void or_bit(uint64_t *word, uint64_t bit, int shared)
{
    if (shared)
        __atomic_fetch_or(word, bit, __ATOMIC_RELAXED);
    else
        *word |= bit;
}

/* InsertKmer of Algorithm 1 for one valid packed k-mer. */
static void insert_kmer(const orc_params *p, uint64_t *F, uint64_t K, int shared)
{
    uint64_t shard = shard_of(p, K);
    uint64_t *words = F + shard * p->S;
    for (uint32_t i = 0; i + p->s <= p->k; i++) {
        uint64_t g = orc_hash_smer(orc_subwindow(K, p->k, p->s, i));
        for (uint32_t t = 0; t < p->H; t++)
            or_bit(&words[orc_word_index(g, t, p->H, p->S)], 1ULL << orc_bit_address(g, t, p->H), shared);
    }
}

/* Contains of Algorithm 2 for one valid packed k-mer: true only when every
 * bit of every s-mer is set in the k-mer's shard. */
int orc_contains_kmer(const orc_params *p, const uint64_t *F, uint64_t K)
{
    uint64_t shard = shard_of(p, K);
    const uint64_t *words = F + shard * p->S;
    for (uint32_t i = 0; i + p->s <= p->k; i++) {
        uint64_t g = orc_hash_smer(orc_subwindow(K, p->k, p->s, i));
        for (uint32_t t = 0; t < p->H; t++) {
            uint64_t w = words[orc_word_index(g, t, p->H, p->S)];
            if (!((w >> orc_bit_address(g, t, p->H)) & 1ULL))
                return 0;
        }
    }
    return 1;
}

/* Insert every valid k-mer of every record.  Record r is
 * seq[off[r] .. off[r+1]); k-mers never span two records (Section
 * "Sequence-Native Design": records are separated by an invalid symbol). */
static void insert_records(uint32_t k, uint32_t s, uint32_t m, uint32_t H, uint32_t S,
                           uint64_t nshards, uint64_t *F, const unsigned char *seq,
                           const uint64_t *off, uint64_t nrec, int shared)
{
    orc_params p = {k, s, m, H, S, nshards};
    for (uint64_t r = 0; r < nrec; r++) {
        uint64_t a = off[r], b = off[r + 1];
        for (uint64_t i = a; i + k <= b; i++) {
            uint64_t K;
            if (orc_pack(seq + i, k, &K))
                insert_kmer(&p, F, K, shared);
        }
    }
}

void orc_insert_records(uint32_t k, uint32_t s, uint32_t m, uint32_t H, uint32_t S,
                        uint64_t nshards, uint64_t *F, const unsigned char *seq,
                        const uint64_t *off, uint64_t nrec)
{
    insert_records(k, s, m, H, S, nshards, F, seq, off, nrec, 0);
}

/* As orc_insert_records, with atomic ORs: threads may insert different
 * records (or k-1-overlapping pieces of one) into one filter concurrently. */
void orc_insert_records_shared(uint32_t k, uint32_t s, uint32_t m, uint32_t H, uint32_t S,
                               uint64_t nshards, uint64_t *F, const unsigned char *seq,
                               const uint64_t *off, uint64_t nrec)
{
    insert_records(k, s, m, H, S, nshards, F, seq, off, nrec, 1);
}

/* Query every k-mer position.  out is indexed by base position: out[i] is the
 * answer for the k-mer starting at seq[i]; it is 0 for invalid k-mers, for
 * k-mers that would leave their record, and for positions outside
 * [off[0], off[nrec]) (Algorithm 2: an invalid k-mer writes false). */
void orc_query_records(uint32_t k, uint32_t s, uint32_t m, uint32_t H, uint32_t S,
                       uint64_t nshards, const uint64_t *F, const unsigned char *seq,
                       const uint64_t *off, uint64_t nrec, uint8_t *out)
{
    orc_params p = {k, s, m, H, S, nshards};
    for (uint64_t r = 0; r < nrec; r++) {
        uint64_t a = off[r], b = off[r + 1];
        for (uint64_t i = a; i < b; i++) {
            uint64_t K;
            out[i] = 0;
            if (i + k <= b && orc_pack(seq + i, k, &K))
                out[i] = (uint8_t)orc_contains_kmer(&p, F, K);
        }
    }
}

/* Shard index of the k-mer at every position (UINT64_MAX when invalid). */
void orc_kmer_shards(uint32_t k, uint32_t m, uint64_t nshards, const unsigned char *seq,
                     uint64_t len, uint64_t *shard)
{
    for (uint64_t i = 0; i + k <= len; i++) {
        uint64_t K;
        shard[i] = orc_pack(seq + i, k, &K)
                       ? (orc_min_hash(K, k, m) & (nshards - 1ULL))
                       : UINT64_MAX;
    }
}

/* Minimum minimizer hash of the k-mer at every position (0 when invalid,
 * with valid[i] telling the two apart). */
void orc_kmer_min_hashes(uint32_t k, uint32_t m, const unsigned char *seq, uint64_t len,
                         uint64_t *mu, uint8_t *valid)
{
    for (uint64_t i = 0; i + k <= len; i++) {
        uint64_t K;
        valid[i] = (uint8_t)orc_pack(seq + i, k, &K);
        mu[i] = valid[i] ? orc_min_hash(K, k, m) : 0;
    }
}

/* Runs of the segmented reduction (Algorithm 1 and its figure on segmented
 * warp reduction): contiguous active entries with equal shard form one run;
 * an inactive entry has a per-lane sentinel shard and so ends a run and forms
 * none.  Returns the number of runs; each run costs one atomic per word. */
uint64_t orc_count_runs(const uint64_t *shard, const uint8_t *active, uint64_t n)
{
    uint64_t runs = 0;
    for (uint64_t i = 0; i < n; i++) {
        if (!active[i])
            continue;
        if (i == 0 || !active[i - 1] || shard[i - 1] != shard[i])
            runs++;
    }
    return runs;
}

/* Super-k-mer segments of a record batch: maximal runs of consecutive valid
 * k-mers of one record with the same shard.  Each costs one shard
 * read-modify-write on insert and one shard read on query.  If lengths is not
 * NULL, the length of segment j is written to lengths[j] (capacity cap). */
uint64_t orc_count_segments(uint32_t k, uint32_t m, uint64_t nshards, const unsigned char *seq,
                            const uint64_t *off, uint64_t nrec, uint32_t *lengths, uint64_t cap)
{
    uint64_t nseg = 0;
    for (uint64_t r = 0; r < nrec; r++) {
        uint64_t a = off[r], b = off[r + 1];
        int open = 0;
        uint64_t prev = 0;
        uint32_t run = 0;
        for (uint64_t i = a; i + k <= b; i++) {
            uint64_t K;
            if (!orc_pack(seq + i, k, &K)) {
                if (open && lengths && nseg - 1 < cap)
                    lengths[nseg - 1] = run;
                open = 0;
                continue;
            }
            uint64_t sh = orc_min_hash(K, k, m) & (nshards - 1ULL);
            if (open && sh == prev) {
                run++;
            } else {
                if (open && lengths && nseg - 1 < cap)
                    lengths[nseg - 1] = run;
                nseg++;
                run = 1;
                open = 1;
            }
            prev = sh;
        }
        if (open && lengths && nseg - 1 < cap)
            lengths[nseg - 1] = run;
    }
    return nseg;
}
