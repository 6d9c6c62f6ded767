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


def test_cpu_baseline_sample_batches():
    """The CPU baseline's genome prefix keeps whole records and clips the last
    one; its query sample takes every read class of the workload, negatives
    from the workload's own negative reads and positives from the prefix (all
    of their error-free k-mers are then in the prefix's filter)."""
    import oracle
    import synth

    seq = np.frombuffer(b"ACGT" * 3000, dtype=np.uint8)
    off = np.array([0, 100, 5000, 12000], dtype=np.uint64)
    for n, want in ((50, [0, 50]), (100, [0, 100]), (101, [0, 100, 101]), (7000, [0, 100, 5000, 7000]),
                    (20000, [0, 100, 5000, 12000])):
        s, o = bench._prefix_batch(seq, off, n)
        assert s.size == min(n, 12000) and o.tolist() == want
    w = synth.tiny_workload()
    pre = bench._prefix_batch(*w["insert"], 300_000)
    q, qoff = bench.cpu_query_sample(w, pre, 100_000, 5)
    assert abs(bench.kmer_positions(qoff, 31) - 100_000) < 1000
    lens = np.diff(qoff.astype(np.int64))
    assert lens.size == 2
    p = oracle.Params(31, 28, 16, 4, 1 << 24)
    F = oracle.insert(p, p.empty(), *pre)
    ans = oracle.query(p, F, q, qoff)
    pos = ans[:int(qoff[1])]
    assert pos[:int(qoff[1]) - 30].mean() > 0.5   # positives drawn from the prefix (1% substitutions)
    neg_start = int(w["query"][1][1])
    assert np.array_equal(q[int(qoff[1]):], w["query"][0][neg_start:neg_start + int(lens[1])])
