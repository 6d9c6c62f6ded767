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
