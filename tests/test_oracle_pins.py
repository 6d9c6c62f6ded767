"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names what fixes the expected value: a published test vector, a
closed form, a worked example printed in the paper, a special case that
reduces to a plain structure, brute force on tiny inputs (string slicing and
Python sets instead of the oracle's bit arithmetic), or a statistical
prediction from the Bloom false-positive equations.  None of these tests needs
a GPU.
"""

from math import isqrt

import numpy as np
import pytest

import oracle
import synth
from conftest import golden

MASK64 = (1 << 64) - 1
_TR = str.maketrans("ACGTacgt", "01230123")


def pack_str(s: str) -> int:
    """Base-4 numeral of a DNA string, first base most significant."""
    return int(s.translate(_TR), 4) if s else 0


def rand_dna(rng, n, alphabet="ACGT"):
    return "".join(rng.choice(list(alphabet), n))


def slice_bits(g: int, lo: int, width: int) -> int:
    """Bits lo .. lo+width-1 of a 64-bit value, read from its binary string."""
    b = format(g, "064b")
    return int(b[64 - lo - width: 64 - lo], 2)


# --- hash functions -----------------------------------------------------------

def test_minimizer_constant_is_floor_2_64_over_phi():
    """h_M(1) is the multiplier; Fibonacci hashing fixes it as floor(2^64/phi),
    derived here from an integer square root of 5."""
    P = 1 << 256
    s5 = isqrt(5 * P * P)
    expected = ((s5 - P) << 64) // (2 * P)  # floor(2^64 * (sqrt5 - 1) / 2)
    assert oracle.hash_minimizer(1) == expected == 0x9E3779B97F4A7C15


def test_minimizer_hash_is_multiplicative():
    """A single multiplicative mix is additive mod 2^64; with h(1) pinned above,
    additivity fixes h(y) = y * h(1) for every y."""
    rng = np.random.default_rng(1)
    assert oracle.hash_minimizer(0) == 0
    for _ in range(2000):
        a = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        b = int(rng.integers(0, 1 << 32))
        assert oracle.hash_minimizer((a + b) & MASK64) == (oracle.hash_minimizer(a) + oracle.hash_minimizer(b)) & MASK64


def _inv_xorshift_right(z: int, r: int) -> int:
    x = z
    for _ in range(64 // r + 1):
        x = z ^ (x >> r)
    return x & MASK64


def test_smer_hash_matches_splitmix64_published_vectors():
    """The s-mer hash is the first xorshift-multiply round of the SplitMix64
    finaliser plus its closing xorshift-31.  Undo the finaliser's outer stages
    on the published outputs to get the expected inner value for each state."""
    lines = [l.split() for l in open(golden("splitmix64_seed1234567.txt")) if l.strip() and not l.startswith("#")]
    seed = int(lines[0][1])
    outs = [int(l[0]) for l in lines[1:]]
    gamma, c2 = 0x9E3779B97F4A7C15, 0x94D049BB133111EB
    c2_inv = pow(c2, -1, 1 << 64)
    state = seed
    for z in outs:
        state = (state + gamma) & MASK64
        y = _inv_xorshift_right(z, 31)            # before the final xorshift 31
        y = (y * c2_inv) & MASK64                 # before the second multiply
        inner = _inv_xorshift_right(y, 27)        # = first round(state)
        expected = inner ^ (inner >> 31)
        assert oracle.hash_smer(state) == expected
    assert oracle.hash_smer(0) == 0


@pytest.mark.parametrize("H", list(range(1, 11)))
def test_bit_address_is_low_six_bits_of_slice(H):
    """Bit-slicing: with W = 64//H >= 6, hash index t uses slice t; the address
    is read here from the binary string of the hash."""
    rng = np.random.default_rng(H)
    W = 64 // H
    for _ in range(300):
        g = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        for t in range(H):
            assert oracle.bit_address(g, t, H) == slice_bits(g, t * W, 6)
            assert oracle.word_index(g, t, H, 4) == t % 4


# Known answers of the salted bit address for narrow slices (64 // H < 6,
# i.e. H >= 11): beta_t(g) = top 6 bits of g * salt_t mod 2^64 with
# salt_t = floor(2^64/phi) * (2t + 1) mod 2^64 (Section "Optimizations":
# a golden-ratio-derived salt when the slices are too narrow for a 6-bit
# address).  The rows were written out with Python integers, t = 0 .. 15.
SALTED_BETA = {
    0x0123456789ABCDEF: [3, 9, 15, 22, 28, 34, 40, 47, 53, 59, 2, 8, 14, 20, 27, 33],
    0xFFFFFFFFFFFFFFFF: [24, 9, 58, 43, 28, 12, 61, 46, 31, 16, 1, 50, 35, 20, 4, 53],
    0x8000000000000001: [7, 22, 37, 52, 3, 19, 34, 49, 0, 15, 30, 45, 60, 11, 27, 42],
    0xDEADBEEFCAFEF00D: [23, 6, 53, 36, 20, 3, 50, 33, 16, 63, 46, 29, 13, 60, 43, 26],
}


@pytest.mark.parametrize("H", [11, 12, 13, 16])
def test_salted_bit_address_known_answers(H):
    """H >= 11 leaves slices narrower than 6 bits, so each hash index takes the
    top 6 bits of the hash times its own odd golden-ratio salt.  Checked
    against the written-out table, and by hand on two inputs: g = 1 gives the
    top bits of the salt itself, and g = 2^63 + 1 adds 2^63 to it (an odd salt
    times 2^63 is 2^63 mod 2^64), flipping only the top bit of the address.
    The salt for t is (2t + 1) times the minimizer multiplier, so beta_t(g) is
    also the top 6 bits of the (pinned) minimizer hash of (2t + 1) g."""
    for g, row in SALTED_BETA.items():
        for t in range(H):
            assert oracle.bit_address(g, t, H) == row[t], (hex(g), t)
            assert oracle.word_index(g, t, H, 4) == t % 4
    for t in range(H):
        top = oracle.bit_address(1, t, H)
        assert oracle.bit_address((1 << 63) + 1, t, H) == top ^ 32
        assert top == oracle.hash_minimizer(2 * t + 1) >> 58
    assert oracle.bit_address(1, 0, H) == 0x9E3779B97F4A7C15 >> 58 == 39
    rng = np.random.default_rng(H)
    for _ in range(200):
        g = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        for t in range(H):
            assert oracle.bit_address(g, t, H) == oracle.hash_minimizer(((2 * t + 1) * g) & MASK64) >> 58


def test_word_index_groups_for_wider_shards():
    rng = np.random.default_rng(7)
    for S, gbits in ((8, 1), (16, 2)):
        for H in (1, 2, 3, 4):
            W = 64 // H
            for _ in range(100):
                g = int(rng.integers(0, 1 << 62))
                for t in range(H):
                    assert oracle.word_index(g, t, H, S) == t % 4 + 4 * slice_bits(g, t * W + 6, gbits)


def test_base_codes_exhaustive():
    table = {ord("A"): 0, ord("C"): 1, ord("G"): 2, ord("T"): 3,
             ord("a"): 0, ord("c"): 1, ord("g"): 2, ord("t"): 3}
    for c in range(256):
        assert oracle.base_code(c) == table.get(c, -1)


@pytest.mark.parametrize("bits,S,n", [(1, 4, 1), (256, 4, 1), (257, 4, 2), (512, 4, 2), (513, 4, 4),
                                      (1 << 24, 4, 1 << 16), (1_600_000_000, 4, 1 << 23),
                                      (48_000_000_000, 4, 1 << 28), (1 << 24, 8, 1 << 15),
                                      (1 << 24, 16, 1 << 14)])
def test_num_shards_closed_form(bits, S, n):
    assert oracle.num_shards(bits, S) == n


# --- packing and windows ---------------------------------------------------------

def test_subwindow_equals_packing_the_substring():
    rng = np.random.default_rng(3)
    for k in (5, 9, 17, 31, 32):
        for _ in range(20):
            s = rand_dna(rng, k)
            K = pack_str(s)
            for L in range(1, k + 1):
                for j in range(0, k - L + 1):
                    assert oracle.subwindow(K, k, L, j) == pack_str(s[j:j + L])


def brute_min_hash(kmer: str, m: int) -> int:
    return min(oracle.hash_minimizer(pack_str(kmer[j:j + m])) for j in range(len(kmer) - m + 1))


def test_minimizer_brute_force_over_substrings():
    rng = np.random.default_rng(4)
    seq = rand_dna(rng, 400) + "N" + rand_dna(rng, 100)
    for k, m in ((31, 16), (21, 11), (32, 32), (9, 5), (31, 1)):
        mu, valid = oracle.kmer_min_hashes(k, m, seq)
        for i in range(len(seq) - k + 1):
            kmer = seq[i:i + k]
            assert valid[i] == ("N" not in kmer)
            if valid[i]:
                assert mu[i] == brute_min_hash(kmer, m)


def expected_single_kmer_bits(kmer, k, s, m, H, nshards, S=4):
    """(word index, bit) pairs set by inserting one k-mer, from string slices."""
    shard = brute_min_hash(kmer, m) & (nshards - 1)
    W = 64 // H
    gbits = (S // 4).bit_length() - 1
    out = set()
    for i in range(k - s + 1):
        g = oracle.hash_smer(pack_str(kmer[i:i + s]))
        for t in range(H):
            beta = slice_bits(g, t * W, 6) if W >= 6 else oracle.bit_address(g, t, H)
            group = slice_bits(g, t * W + 6, gbits) if gbits else 0
            out.add((shard * S + t % 4 + 4 * group, beta))
    return out


def set_bits(F):
    nz = np.flatnonzero(F)
    return {(int(w), b) for w in nz for b in range(64) if (int(F[w]) >> b) & 1}


@pytest.mark.parametrize("k,s,m,H,bits,S", [
    (31, 28, 16, 4, 1 << 24, 4), (31, 31, 16, 4, 1 << 20, 4), (31, 24, 12, 8, 1 << 22, 4),
    (32, 32, 32, 1, 1 << 16, 4), (32, 20, 10, 3, 1 << 18, 4), (9, 6, 5, 2, 4096, 4),
    (31, 28, 16, 4, 1 << 24, 8), (31, 28, 16, 2, 1 << 24, 16), (21, 19, 11, 16, 1 << 20, 4),
    (31, 28, 16, 6, 1 << 24, 4), (1, 1, 1, 1, 256, 4)])
def test_single_kmer_insert_brute_force(k, s, m, H, bits, S):
    rng = np.random.default_rng(k * 1000 + s * 10 + H)
    p = oracle.Params(k, s, m, H, bits, S)
    for _ in range(25):
        kmer = rand_dna(rng, k, "ACGTacgt")
        F = oracle.insert(p, p.empty(), kmer)
        assert set_bits(F) == expected_single_kmer_bits(kmer.upper(), k, s, m, H, p.nshards, S)
        assert oracle.query(p, F, kmer)[0] == 1


# --- closed forms and special cases ---------------------------------------------

@pytest.mark.parametrize("H", [1, 2, 3, 4, 8, 10, 16])
@pytest.mark.parametrize("S", [4, 8, 16])
def test_all_A_closed_form(H, S):
    """Every m-mer and s-mer of A^n packs to 0, both hashes of 0 are 0, so the
    filter holds exactly bit 0 of words 0..min(H,4)-1 of shard 0."""
    if S > 4 and 64 // H < 6 + (S // 4).bit_length() - 1:
        pytest.skip("wider shards need slices of at least 6 + log2(S/4) bits")
    p = oracle.Params(31, 28, 16, H, 1 << 20, S)
    F = oracle.insert(p, p.empty(), "A" * 200)
    expect = np.zeros_like(F)
    expect[: min(H, 4)] = 1
    assert np.array_equal(F, expect)
    assert oracle.query(p, F, "A" * 31).tolist() == [1]
    assert oracle.query(p, F, "A" * 15 + "N" + "A" * 15).tolist() == [0]
    assert oracle.query(p, F, "a" * 40).tolist() == [1] * 10


def test_single_shard_filter_is_set_of_smers():
    """bits <= 256 gives one shard: the filter is the OR of the bits of every
    distinct s-mer that lies in some valid k-mer (Python set of strings)."""
    rng = np.random.default_rng(11)
    k, s, m, H = 31, 28, 16, 4
    p = oracle.Params(k, s, m, H, 200)
    assert p.nshards == 1
    seq = rand_dna(rng, 60) + "N" + rand_dna(rng, 45)
    F = oracle.insert(p, p.empty(), seq)
    smers = set()
    for i in range(len(seq) - k + 1):
        kmer = seq[i:i + k]
        if "N" not in kmer:
            smers.update(kmer[j:j + s] for j in range(k - s + 1))
    expect = np.zeros(4, dtype=np.uint64)
    for x in smers:
        g = oracle.hash_smer(pack_str(x))
        for t in range(H):
            expect[t % 4] |= np.uint64(1 << slice_bits(g, 16 * t, 6))
    assert np.array_equal(F, expect)


def test_s_equals_k_is_blocked_bloom_of_kmers():
    """s = k (z = 0): a blocked Bloom filter whose block is the minimizer shard
    and whose H bits come from the hash of the whole k-mer."""
    rng = np.random.default_rng(12)
    k, m, H = 25, 12, 4
    p = oracle.Params(k, k, m, H, 1 << 16)
    seq = rand_dna(rng, 500)
    F = oracle.insert(p, p.empty(), seq)
    expect = p.empty()
    for i in range(len(seq) - k + 1):
        kmer = seq[i:i + k]
        shard = brute_min_hash(kmer, m) & (p.nshards - 1)
        g = oracle.hash_smer(pack_str(kmer))
        for t in range(H):
            expect[shard * 4 + t % 4] |= np.uint64(1 << slice_bits(g, 16 * t, 6))
    assert np.array_equal(F, expect)


def test_m_equals_k_every_kmer_is_its_own_minimizer():
    rng = np.random.default_rng(13)
    p = oracle.Params(21, 18, 21, 4, 1 << 22)
    seq = rand_dna(rng, 300)
    sh = oracle.kmer_shards(p, seq)
    for i in range(len(seq) - 21 + 1):
        assert sh[i] == oracle.hash_minimizer(pack_str(seq[i:i + 21])) & (p.nshards - 1)


# --- set semantics and invariants -----------------------------------------------

def test_huge_filter_answers_exact_set_membership():
    """With 2^30 bits and 5000 inserted k-mers a false positive needs 16 bit
    hits in a shard that holds ~0 other s-mers, so answers equal exact
    membership in the inserted set (Python set of strings)."""
    rng = np.random.default_rng(21)
    k = 31
    p = oracle.Params(k, 28, 16, 4, 1 << 30)
    ins = [rand_dna(rng, k) for _ in range(4000)]
    seq = rand_dna(rng, 1000 + k - 1)
    F = p.empty()
    oracle.insert(p, F, "".join(ins), np.arange(0, 4000 * k + 1, k))
    oracle.insert(p, F, seq)
    inserted = set(ins) | {seq[i:i + k] for i in range(len(seq) - k + 1)}
    probe = ins[:500] + [rand_dna(rng, k) for _ in range(3000)] + [seq[i:i + k] for i in range(0, 1000, 7)]
    probe += [x[:10] + "N" + x[11:] for x in ins[:50]]
    ans = oracle.query(p, F, "".join(probe), np.arange(0, len(probe) * k + 1, k))[::k]
    assert ans.tolist() == [int(x in inserted) for x in probe]


def test_union_order_and_record_independence():
    rng = np.random.default_rng(22)
    p = oracle.Params(31, 28, 16, 4, 1 << 14)
    A = rand_dna(rng, 3000)
    B = rand_dna(rng, 2000) + "NN" + rand_dna(rng, 500)
    FA = oracle.insert(p, p.empty(), A)
    FB = oracle.insert(p, p.empty(), B)
    FAB = oracle.insert(p, oracle.insert(p, p.empty(), A), B)
    FBA = oracle.insert(p, oracle.insert(p, p.empty(), B), A)
    assert np.array_equal(FAB, FA | FB) and np.array_equal(FBA, FA | FB)
    # a batch of two records never inserts a k-mer that spans them
    Fbatch = oracle.insert(p, p.empty(), A + B, [0, len(A), len(A) + len(B)])
    assert np.array_equal(Fbatch, FA | FB)
    assert not np.array_equal(Fbatch, oracle.insert(p, p.empty(), A + B))
    # chunks overlapping by k-1 bases insert the same k-mers
    cuts = [0, 700, 1001, 2990, 3000]
    Fch = p.empty()
    for a, b in zip(cuts[:-1], cuts[1:]):
        oracle.insert(p, Fch, A[a:min(len(A), b + 30)])
    assert np.array_equal(Fch, FA)
    # every k-mer as its own record
    kmers = [A[i:i + 31] for i in range(len(A) - 30)]
    Fk = oracle.insert(p, p.empty(), "".join(kmers), np.arange(0, 31 * len(kmers) + 1, 31))
    assert np.array_equal(Fk, FA)


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_parallel_insert_and_query_equal_the_serial_ones(threads):
    """The threaded forms used on full-size workloads (k-1-overlapping pieces;
    atomic ORs into one filter) give the serial oracle's filter and answers:
    OR is commutative and idempotent, and every k-mer start belongs to one
    piece whose bases contain the whole k-mer."""
    rng = np.random.default_rng(26 + threads)
    p = oracle.Params(31, 28, 16, 4, 1 << 14)
    lengths = [int(x) for x in rng.integers(0, 400, 40)] + [5000, 0, 31, 30]
    seq = np.frombuffer(rand_dna(rng, sum(lengths), "ACGT" * 30 + "N").encode(), dtype=np.uint8)
    off = np.concatenate(([0], np.cumsum(lengths))).astype(np.uint64)
    want = oracle.insert(p, p.empty(), seq, off)
    got = oracle.insert_parallel(p, p.empty(), seq, off, threads=threads)
    assert np.array_equal(got, want)
    assert np.array_equal(oracle.query_parallel(p, want, seq, off, threads=threads), oracle.query(p, want, seq, off))
    # one long record cut into many pieces
    one = np.array([0, seq.size], dtype=np.uint64)
    assert np.array_equal(oracle.insert_parallel(p, p.empty(), seq, one, threads=threads),
                          oracle.insert(p, p.empty(), seq, one))
    assert np.array_equal(oracle.query_parallel(p, want, seq, one, threads=threads),
                          oracle.query(p, want, seq, one, per_base=True))
    # pieces partition the k-mer starts and cover their k-mers
    for n in (1, 2, 7, 64):
        cov = np.zeros(seq.size, dtype=np.int64)
        for a, b, e, loc in oracle.pieces(off, seq.size, n, 31):
            cov[a:b] += 1
            assert e == min(seq.size, b + 30) and loc[0] == 0 and loc[-1] == e - a
        assert (cov[:seq.size - 30] == 1).all() and not cov[seq.size - 30:].any()


def test_query_zero_false_negatives_read_only_and_idempotent():
    rng = np.random.default_rng(23)
    p = oracle.Params(31, 28, 16, 4, 1 << 12)
    seq = rand_dna(rng, 5000, "ACGTN" * 30 + "n")
    F = oracle.insert(p, p.empty(), seq)
    F0 = F.copy()
    a1 = oracle.query(p, F, seq)
    a2 = oracle.query(p, F, seq)
    assert np.array_equal(F, F0) and np.array_equal(a1, a2)
    valid = np.array([all(c in "ACGTacgt" for c in seq[i:i + 31]) for i in range(len(seq) - 30)])
    assert np.all(a1[valid] == 1) and np.all(a1[~valid] == 0)


def test_short_and_empty_inputs():
    p = oracle.Params(31, 28, 16, 4, 1 << 12)
    F = oracle.insert(p, p.empty(), "ACGT" * 7)  # 28 bases < k
    assert not F.any()
    assert oracle.query(p, F, "ACGT" * 7).size == 0
    assert oracle.query(p, F, "").size == 0
    out = oracle.query(p, F, "A" * 40 + "C" * 10, [0, 0, 20, 50, 50])
    assert out.size == 50 and not out.any()


def test_record_ends_answer_zero_on_a_nonempty_filter():
    """Answers are per base position; the last k-1 positions of each record
    (and every position of a record shorter than k) answer 0 even when the
    k-mer that starts there and runs into the next record is in the filter
    (Section "Sequence-Native Design": no k-mer spans two records; Algorithm 2
    writes false for an invalid k-mer).  The concatenation of the records is
    inserted as one record, so every spanning k-mer is present; with 2^30 bits
    the answers are exact membership, computed here from string slices."""
    rng = np.random.default_rng(24)
    k = 31
    p = oracle.Params(k, 28, 16, 4, 1 << 30)
    lengths = [45, 0, 31, 5, 32, 100, 30, 64, 1, 40]
    recs = [rand_dna(rng, n, "ACGT" * 20 + "N") for n in lengths]
    seq = "".join(recs)
    off = np.concatenate(([0], np.cumsum(lengths))).astype(np.uint64)
    F = oracle.insert(p, p.empty(), seq)          # one record: spanning k-mers inserted
    present = {seq[i:i + k] for i in range(len(seq) - k + 1) if "N" not in seq[i:i + k]}
    out = oracle.query(p, F, seq, off)
    assert out.size == len(seq)
    want = []
    for r in recs:
        for i in range(len(r)):
            kmer = r[i:i + k]
            want.append(int(len(kmer) == k and kmer in present))
    assert out.tolist() == want
    # the spanning k-mers themselves answer 1 when queried as one record
    whole = oracle.query(p, F, seq)
    assert whole.tolist() == [int(seq[i:i + k] in present) for i in range(len(seq) - k + 1)]
    assert int(whole.sum(dtype=np.int64)) > sum(want)


def brute_segments(recs, k, m, nshards):
    """Maximal runs of consecutive valid k-mers of one record with one shard,
    from string slices (a k-mer with a byte outside ACGTacgt is invalid and
    ends the run; a record start ends it too)."""
    lengths = []
    for rec in recs:
        prev = None
        for i in range(len(rec) - k + 1):
            kmer = rec[i:i + k]
            if any(c not in "ACGTacgt" for c in kmer):
                prev = None
                continue
            sh = brute_min_hash(kmer.upper(), m) & (nshards - 1)
            if prev is not None and sh == prev:
                lengths[-1] += 1
            else:
                lengths.append(1)
            prev = sh
    return lengths


@pytest.mark.parametrize("bits", [256, 1024, 1 << 14, 1 << 40])
def test_segment_count_brute_force_with_invalid_bases_and_records(bits):
    """Super-k-mer segments (one shard access each; the denominators of the
    out-of-cache rooflines) against a brute-force count over string slices, on
    record batches with N bases and short records.  With one or four shards
    nearly every pair of neighbouring k-mers shares a shard, so a run that
    failed to end at an invalid k-mer or at a record start would change the
    count."""
    rng = np.random.default_rng(bits % 1000 + 25)
    k, m = 31, 16
    p = oracle.Params(k, 28, m, 4, bits)
    for trial in range(6):
        lengths = [int(x) for x in rng.integers(0, 140, 12)] + [31, 32, 30]
        recs = [rand_dna(rng, n, "ACGT" * 12 + "Nn") for n in lengths]
        rng.shuffle(recs)
        seq = "".join(recs)
        off = np.concatenate(([0], np.cumsum([len(r) for r in recs]))).astype(np.uint64)
        want = brute_segments(recs, k, m, p.nshards)
        n, got = oracle.count_segments(p, seq, off, with_lengths=True)
        assert n == len(want)
        assert got.tolist() == want
        assert oracle.count_segments(p, seq, off) == len(want)


# --- worked examples of the paper --------------------------------------------

def test_fig3_segmented_reduction_atomic_count():
    rows = {l.split()[0]: l.split()[1:] for l in open(golden("fig3_segmented_reduction.txt"))
            if l.strip() and not l.startswith("#")}
    names = rows["lanes"]
    active = [int(x) for x in rows["active"]]
    ids = {n: i for i, n in enumerate(sorted(set(names) - {"-"}))}
    shards = [ids.get(n, 1000 + i) for i, n in enumerate(names)]
    words = int(rows["words_per_shard"][0])
    assert sum(active) * words == int(rows["atomics_without_reduction"][0])
    assert oracle.count_runs(shards, active) * words == int(rows["atomics_with_reduction"][0])


def test_default_configuration_tests_16_bits_per_kmer():
    """(k - s + 1) * H = 16 independent bit tests at k=31, s=28, H=4: a single
    k-mer insert into an empty filter sets at most 16 bits."""
    rng = np.random.default_rng(31)
    p = oracle.Params(31, 28, 16, 4, 1 << 24)
    counts = [len(set_bits(oracle.insert(p, p.empty(), rand_dna(rng, 31)))) for _ in range(200)]
    assert max(counts) == 16 and min(counts) >= 12


def test_mean_super_kmer_length_matches_density():
    """Random minimizers on random sequence: density 2/(w+1), mean super-k-mer
    length (w+1)/2 = 8.5 at k=31, m=16.  A filter large enough that distinct
    minimizers almost never share a shard."""
    seq = synth.uniform_acgt(1_000_000, 7)
    p = oracle.Params(31, 28, 16, 4, 1 << 40)
    nseg, lengths = oracle.count_segments(p, seq, with_lengths=True)
    mean = (seq.size - 30) / nseg
    assert abs(mean - 8.5) / 8.5 < 0.02
    assert lengths.max() <= 16 + 2  # one minimizer covers at most w k-mers (rare equal-shard merges)


# --- false-positive rate ------------------------------------------------------------

def _independent_kmers(n, k, seed):
    q = synth.uniform_acgt(n * k, seed)
    return q, np.arange(0, n * k + 1, k, dtype=np.uint64)


def _occupancy_moment(balls_max, e, bins=64):
    """E[(X/bins)^e] for X = occupied bins after n balls, n = 0..balls_max."""
    out = np.zeros(balls_max + 1)
    P = np.zeros(bins + 1)
    P[0] = 1.0
    j = np.arange(bins + 1)
    for n in range(balls_max + 1):
        out[n] = float(np.sum(P * (j / bins) ** e))
        Q = P * j / bins
        Q[1:] += P[:-1] * (bins - j[:-1]) / bins
        P = Q
    return out


@pytest.mark.parametrize("bits,H,s", [(1 << 22, 4, 28), (1 << 23, 8, 28), (1 << 23, 1, 31), (1 << 23, 3, 28)])
def test_fpr_matches_conditional_prediction(bits, H, s):
    """Given the filter and an ideal s-mer hash, a random alien k-mer is a false
    positive with probability prod_w (popcount(word w of its shard)/64)^((z+1)c_w)
    (Bloom Eq. 1 per sector, Findere Eq. 2 across the z+1 s-mers).  The measured
    count must sit in the 99.9% interval of that expectation."""
    k, m = 31, 16
    p = oracle.Params(k, s, m, H, bits)
    F = oracle.insert(p, p.empty(), synth.uniform_acgt(1_000_000, 41))
    n = 400_000
    q, qoff = _independent_kmers(n, k, 42)
    ans = oracle.query(p, F, q, qoff)[qoff[:-1].astype(np.int64)]
    shard = oracle.kmer_shards(p, q)[qoff[:-1].astype(np.int64)]
    pop = np.array([bin(int(w)).count("1") for w in F], dtype=np.float64).reshape(-1, 4)
    c = np.bincount(np.arange(H) % 4, minlength=4)
    z1 = k - s + 1
    prob = np.prod((pop[shard] / 64.0) ** (z1 * c[None, :]), axis=1)
    mean = prob.sum()
    sd = np.sqrt(np.sum(prob * (1 - prob)))
    assert abs(ans.sum() - mean) <= 3.29 * sd + 1.0, (ans.sum(), mean, sd)


@pytest.mark.parametrize("bits", [1 << 22, 1 << 23])
def test_fpr_matches_unconditional_closed_form(bits):
    """Closed form from the filter's design, not its contents: super-k-mers per
    shard ~ Poisson(segments / N), each adds L+z s-mers; per sector the bits
    are the occupancy of those balls in 64 bins; epsilon = E[prod_w
    E[(X_w/64)^(z+1)]].  Within 10% of the measured rate."""
    k, s, m, H = 31, 28, 16, 4
    p = oracle.Params(k, s, m, H, bits)
    ins = synth.uniform_acgt(1_000_000, 51)
    F = oracle.insert(p, p.empty(), ins)
    nseg, lengths = oracle.count_segments(p, ins, with_lengths=True)
    lam = nseg / p.nshards
    rng = np.random.default_rng(52)
    draws = 200_000
    cnt = rng.poisson(lam, draws)
    tot = np.zeros(draws, dtype=np.int64)
    z = k - s
    seg_balls = lengths.astype(np.int64) + z
    for i in range(1, cnt.max() + 1):
        has = cnt >= i
        tot[has] += seg_balls[rng.integers(0, seg_balls.size, has.sum())]
    mom = _occupancy_moment(int(tot.max()), z + 1)
    eps = np.mean(mom[tot] ** 4)
    n = 1_000_000 if bits > (1 << 22) else 300_000
    q, qoff = _independent_kmers(n, k, 53)
    meas = oracle.query(p, F, q, qoff)[qoff[:-1].astype(np.int64)].mean()
    assert abs(meas - eps) / eps < 0.10, (meas, eps)


def test_near_alien_kmers_revert_to_single_smer_rate():
    """A k-mer one substitution away from an inserted one shares z of its z+1
    s-mers, so its false-positive rate is far above that of a random alien."""
    k = 31
    p = oracle.Params(k, 28, 16, 4, 1 << 22)
    ins = synth.uniform_acgt(1_000_000, 61)
    F = oracle.insert(p, p.empty(), ins)
    rng = np.random.default_rng(62)
    n = 100_000
    starts = rng.integers(0, ins.size - k, n)
    near = ins[starts[:, None] + np.arange(k)].copy()
    col = np.full(n, k - 1)  # substitute the last base: 3 of the 4 s-mers stay
    near[np.arange(n), col] = synth.ACGT[(np.searchsorted(synth.ACGT, near[np.arange(n), col]) + 1) % 4]
    qoff = np.arange(0, n * k + 1, k, dtype=np.uint64)
    near_rate = oracle.query(p, F, near.reshape(-1), qoff)[qoff[:-1].astype(np.int64)].mean()
    q, qoff2 = _independent_kmers(n, k, 63)
    alien_rate = oracle.query(p, F, q, qoff2)[qoff2[:-1].astype(np.int64)].mean()
    assert near_rate > 3 * alien_rate
