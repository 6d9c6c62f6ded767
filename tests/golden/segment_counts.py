"""Writes segment_counts.json next to this file.  For each benchmark workload:

* the number of super-k-mer segments (maximal runs of consecutive valid k-mers
  of one record with one minimizer shard, Section "Minimizers and
  Super-k-mers") of its insert batch and its query batch, counted by the
  oracle over every record.  Each segment costs one shard access on the
  insert (read-modify-write) and query (read) paths, so these counts are the
  algorithmic memory traffic of the out-of-cache roofline;
* the oracle's filter after inserting the whole insert batch (Algorithm 1)
  and its answers to the whole query batch (Algorithm 2), as SHA-256 digests
  of the little-endian words and of the answer bytes, whole and per block
  (2^23 words = 64 MiB of filter, 2^26 answer bytes), with the number of set
  bits and of k-mers answered present.  The full-size GPU tests compare the
  GPU's filter and answers with these digests, and bench.py compares its
  answer count with the stored one.

    python tests/golden/segment_counts.py [--shard-words S] [workload ...]
        (default: tiny in_cache out_of_cache batched; S = 4, the paper's
        shard; with S = 8 or 16 the entries are stored as <workload>_S<S>)

Calls only oracle/ and synth/; the oracle runs on every CPU (threads over
k-1-overlapping pieces, atomic ORs into one filter).
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
FILTER_BLOCK_WORDS = 1 << 23
ANSWER_BLOCK_BYTES = 1 << 26
WORKLOADS = {"in_cache": synth.in_cache_workload, "out_of_cache": synth.out_of_cache_workload,
             "tiny": synth.tiny_workload, "batched": synth.batched_workload}


def digests(a: np.ndarray, block: int):
    """SHA-256 of the array's bytes (little-endian), whole and per block of
    `block` elements."""
    import hashlib

    a = np.ascontiguousarray(a)
    if a.dtype.byteorder == ">":
        a = a.byteswap().view(a.dtype.newbyteorder("<"))
    whole = hashlib.sha256()
    blocks = []
    for i in range(0, a.size, block):
        b = memoryview(a[i:i + block]).cast("B")
        whole.update(b)
        blocks.append(hashlib.sha256(b).hexdigest())
    return whole.hexdigest(), blocks


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
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return int(sum(ex.map(lambda j: oracle.count_segments(p, j[0], j[1]), jobs)))


def main(names, shard_words=4):
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t0 = time.perf_counter()
        w = WORKLOADS[name]()
        p = oracle.Params(w["k"], w["s"], w["m"], w["H"], w["bits"], shard_words=shard_words)
        entry = {"workload": w["name"], "k": w["k"], "s": w["s"], "m": w["m"], "H": w["H"],
                 "filter_bits_requested": int(w["bits"]), "nshards": int(p.nshards)}
        if shard_words != 4:
            entry["shard_words"] = shard_words
        for part in ("insert", "query"):
            seq, off = w[part]
            entry[part] = {"bases": int(seq.size), "kmers": kmer_positions(off, w["k"]),
                           "segments": count(p, (seq, off))}
            entry[part]["segments_per_kmer"] = entry[part]["segments"] / max(1, entry[part]["kmers"])
        print(name, "segments %.0fs" % (time.perf_counter() - t0), flush=True)
        F = oracle.insert_parallel(p, p.empty(), *w["insert"])
        whole, blocks = digests(F, FILTER_BLOCK_WORDS)
        entry["oracle_filter"] = {"words": int(F.size), "set_bits": int(np.bitwise_count(F).sum(dtype=np.int64)),
                                  "sha256": whole, "block_words": FILTER_BLOCK_WORDS, "block_sha256": blocks}
        print(name, "filter %.0fs" % (time.perf_counter() - t0), flush=True)
        ans = oracle.query_parallel(p, F, *w["query"])
        del F
        whole, blocks = digests(ans, ANSWER_BLOCK_BYTES)
        entry["oracle_answers"] = {"bytes": int(ans.size), "present": int(ans.sum(dtype=np.int64)),
                                   "sha256": whole, "block_bytes": ANSWER_BLOCK_BYTES, "block_sha256": blocks}
        del ans
        res[name if shard_words == 4 else "%s_S%d" % (name, shard_words)] = entry
        print(name, json.dumps({k: v for k, v in entry.items() if not k.startswith("oracle")}),
              "present", entry["oracle_answers"]["present"], "%.0fs" % (time.perf_counter() - t0), flush=True)
        del w
        with open(OUT, "w") as f:
            json.dump(res, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    argv = sys.argv[1:]
    sw = 4
    if argv[:1] == ["--shard-words"]:
        sw = int(argv[1])
        argv = argv[2:]
    main(argv or ["tiny", "in_cache", "out_of_cache", "batched"], sw)
