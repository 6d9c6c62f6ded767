"""Stored values used by bench.py come from the oracle: recount the small
workload's super-k-mer segments and compare with the committed file."""

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
