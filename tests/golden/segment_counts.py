"""Writes segment_counts.json next to this file: for each benchmark workload,
the number of super-k-mer segments (maximal runs of consecutive valid k-mers
of one record with one minimizer shard, Section "Minimizers and Super-k-mers")
of its insert batch and its query batch, counted by the oracle over every
record.  Each segment costs one shard access on the insert (read-modify-write)
and query (read) paths, so these counts are the algorithmic memory traffic of
the out-of-cache roofline.

    python tests/golden/segment_counts.py [workload ...]   (default: out_of_cache in_cache)

Calls only oracle/ and synth/.
"""

from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "segment_counts.json")


def kmer_positions(off: np.ndarray, k: int) -> int:
    lens = np.diff(off.astype(np.int64))
    return int(np.maximum(lens - k + 1, 0).sum())


def count(p, batch, parts: int = 64) -> int:
    """Segments of a record batch; records are independent, so the batch is
    split into record ranges counted on threads (the oracle call releases the
    interpreter lock)."""
    seq, off = batch
    nrec = off.size - 1
    if nrec <= 0:
        return 0
    cuts = np.unique(np.linspace(0, nrec, min(parts, nrec) + 1).astype(np.int64))
    jobs = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        lo, hi = int(off[a]), int(off[b])
        jobs.append((seq[lo:hi], off[a:b + 1] - off[a]))
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        return int(sum(ex.map(lambda j: oracle.count_segments(p, j[0], j[1]), jobs)))


def main(names):
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t0 = time.perf_counter()
        w = {"in_cache": synth.in_cache_workload, "out_of_cache": synth.out_of_cache_workload,
             "tiny": synth.tiny_workload}[name]()
        p = oracle.Params(w["k"], w["s"], w["m"], w["H"], w["bits"])
        entry = {"workload": w["name"], "k": w["k"], "m": w["m"], "filter_bits_requested": int(w["bits"]),
                 "nshards": int(p.nshards)}
        for part in ("insert", "query"):
            seq, off = w[part]
            entry[part] = {"bases": int(seq.size), "kmers": kmer_positions(off, w["k"]),
                           "segments": count(p, (seq, off))}
            entry[part]["segments_per_kmer"] = entry[part]["segments"] / max(1, entry[part]["kmers"])
        res[name] = entry
        print(name, json.dumps(entry), "%.0fs" % (time.perf_counter() - t0), flush=True)
        del w
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or ["out_of_cache", "in_cache"])
