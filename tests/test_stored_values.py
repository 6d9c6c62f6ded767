"""Stored values used by bench.py and the full-size GPU tests come from the
oracle: recount the small workload's super-k-mer segments, rebuild its oracle
filter and answers, and compare with the committed file."""

import json
import os

import numpy as np

import oracle
import synth
from conftest import ROOT

STORED = os.path.join(ROOT, "tests", "golden", "segment_counts.json")


def test_tiny_segment_counts_match_the_oracle():
    d = json.load(open(STORED))["tiny"]
    w = synth.tiny_workload()
    p = oracle.Params(w["k"], w["s"], w["m"], w["H"], w["bits"])
    assert d["nshards"] == p.nshards
    for part in ("insert", "query"):
        seq, off = w[part]
        assert d[part]["bases"] == seq.size
        assert d[part]["segments"] == oracle.count_segments(p, seq, off)
        lens = np.diff(off.astype(np.int64))
        assert d[part]["kmers"] == int(np.maximum(lens - w["k"] + 1, 0).sum())


def test_stored_segment_density_is_that_of_random_minimizers():
    """Random minimizers over windows of w = k-m+1 m-mers start a new
    super-k-mer at a fraction 2/(w+1) of positions (Section "Minimizers and
    Super-k-mers": mean length about (w+1)/2); genomes with 5% repeats and
    150 bp reads stay within a few percent of it."""
    d = json.load(open(STORED))
    w = 31 - 16 + 1
    for name, e in d.items():
        for part in ("insert", "query"):
            spk = e[part]["segments"] / e[part]["kmers"]
            if part == "query" and name != "tiny":
                # read ends cut segments: one extra start per read on average
                assert 2 / (w + 1) < spk < 2 / (w + 1) * 1.15, (name, part, spk)
            else:
                assert abs(spk - 2 / (w + 1)) < 0.02 * 2 / (w + 1), (name, part, spk)


def test_tiny_oracle_digests_match_the_oracle():
    """The stored filter and answer digests of the small workload equal those
    of the oracle rebuilt here, serially and with the threaded forms."""
    import hashlib

    d = json.load(open(STORED))["tiny"]
    w = synth.tiny_workload()
    p = oracle.Params(w["k"], w["s"], w["m"], w["H"], w["bits"])
    F = oracle.insert(p, p.empty(), *w["insert"])
    assert np.array_equal(oracle.insert_parallel(p, p.empty(), *w["insert"], threads=4), F)
    ans = oracle.query(p, F, *w["query"])
    assert np.array_equal(oracle.query_parallel(p, F, *w["query"], threads=4), ans)
    assert hashlib.sha256(F.tobytes()).hexdigest() == d["oracle_filter"]["sha256"]
    assert int(np.bitwise_count(F).sum()) == d["oracle_filter"]["set_bits"]
    assert hashlib.sha256(ans.tobytes()).hexdigest() == d["oracle_answers"]["sha256"]
    assert int(ans.sum()) == d["oracle_answers"]["present"] and ans.size == d["oracle_answers"]["bytes"]
    assert len(d["oracle_filter"]["block_sha256"]) == -(-F.size // d["oracle_filter"]["block_words"])
    # the query's first record is a substring of the inserted sequence: all of
    # its k-mers are present (no false negatives)
    qoff = w["query"][1]
    assert ans[:int(qoff[1]) - 30].all()
