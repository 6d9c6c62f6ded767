"""Host-side counting in bench.py: valid k-mer positions per record against a
brute-force count on a small sequence with invalid bytes."""

import numpy as np

import bench


def test_valid_kmers_brute_force():
    rng = np.random.default_rng(11)
    alphabet = np.frombuffer(b"ACGTNacgtx", dtype=np.uint8)
    p = np.array([22, 22, 22, 22, 2, 2.5, 2.5, 2.5, 2.5, 1.0])
    seq = rng.choice(alphabet, size=4000, p=p / p.sum()).astype(np.uint8)
    off = np.array([0, 100, 130, 1000, 1000, 1006, 3000, 4000], dtype=np.uint64)
    ok = set(b"ACGTacgt")
    for k in (1, 7, 31):
        want = 0
        for r in range(off.size - 1):
            a, b = int(off[r]), int(off[r + 1])
            want += sum(all(c in ok for c in seq[i:i + k]) for i in range(a, b - k + 1))
        assert bench.valid_kmers(seq, off, k) == want


def test_valid_kmers_all_valid_equals_positions():
    seq = np.frombuffer(b"ACGT" * 250, dtype=np.uint8)
    off = np.array([0, 10, 500, 1000], dtype=np.uint64)
    assert bench.valid_kmers(seq, off, 31) == bench.kmer_positions(off, 31) == (500 - 10 - 30) + (500 - 30)


def test_parallel_baseline_pieces_equal_one_insert():
    """The CPU baseline's parallel insert (pieces with k-1 overlap and their
    record starts, filters OR-ed) builds the filter of one serial insert."""
    import oracle

    rng = np.random.default_rng(3)
    ins = rng.choice(np.frombuffer(b"ACGTN", dtype=np.uint8), size=120_000,
                     p=[.24, .24, .24, .24, .04]).astype(np.uint8)
    ioff = np.array([0, 1000, 1010, 50_000, 50_030, 90_000, 120_000], dtype=np.uint64)
    p = oracle.Params(31, 28, 16, 4, 1 << 20)
    for total in (120_000, 61_237):
        clip = ioff[ioff <= total] if ioff[-1] <= total else np.concatenate((ioff[ioff < total], [total]))
        want = oracle.insert(p, p.empty(), ins[:total], clip.astype(np.uint64))
        for n in (1, 3, 16):
            got = p.empty()
            for a, e, loc in bench._insert_pieces(ioff, total, n, 31):
                got |= oracle.insert(p, p.empty(), ins[a:e], loc)
            assert np.array_equal(got, want), (total, n)
