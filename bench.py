"""Benchmark of the SBF insert + query path on one MI355X.

One step = clear the filter, insert a synthetic genome (record batch of
contigs), query a batch of reads; all on device-resident input, on torch's
current stream.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W]
                  [--workload out_of_cache|in_cache|tiny|batched|served|host|sweep]
                  [--no-cpu-baseline] [--no-in-cache]

The default workload is the out-of-cache one (3 Gbp genome into an 8 GiB
filter, 10M short + 100k long reads); its line carries the in-cache workload
(100 Mbp into 256 MiB) as a second key.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

PEAK_HBM_GBS = 8000.0        # MI355X HBM3E, GB/s
PEAK_INT_TOPS = 39.3216      # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz, 32-bit integer lane-ops (T/s)
# 32-bit integer VALU operations per k-mer of the rolling formulation
# (encode 1, window pack 2, minimizer hash 3, sliding minimum 9, shard mask 1,
# s-mer hash 10, H=4 bit addresses 4; insert adds one-hot + segment OR 16,
# query adds the (k-s+1)*H = 16 bit tests at 2 ops each plus the output 1)
OPS_PER_KMER = {"insert": 46, "query": 63}
KERNEL_SOURCES = ["paper_2606_24417_amd/csrc/kernels_rolling.hip", "paper_2606_24417_amd/csrc/kernels_wide.hip",
                  "paper_2606_24417_amd/csrc/sbf_tiles.h", "paper_2606_24417_amd/csrc/sbf_device.h",
                  "paper_2606_24417_amd/csrc/sbf_segments.h"]


def kernel_source_hash() -> str:
    """Hash of the kernel sources with comments and whitespace removed, so that
    stored counters stay valid across comment-only edits, and of the compiler
    flags they are built with (a flag can change the code as much as an
    edit)."""
    import re

    from paper_2606_24417_amd import build as B

    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
        h.update(" ".join(B.HIPCC_FLAGS + B.SOURCE_FLAGS.get(os.path.basename(p), [])).encode())
    return h.hexdigest()[:16]


def counter_traffic(workload: str, kernel: str, launches_kmers: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "counters_%s.json" % workload)
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = d.get("kernels", {}).get(kernel)
    if not k:
        return None
    return float(k["hbm_bytes_per_launch"])


def kmer_positions(off: np.ndarray, k: int) -> int:
    lens = np.diff(off.astype(np.int64))
    return int(np.maximum(lens - k + 1, 0).sum())


_ACGT = np.zeros(256, dtype=np.bool_)
_ACGT[np.frombuffer(b"ACGTacgt", dtype=np.uint8)] = True


def valid_kmers(seq: np.ndarray, off: np.ndarray, k: int, chunk: int = 1 << 28) -> int:
    """k-mer positions whose k bases are all A/C/G/T (either case), counted
    per record; equal to kmer_positions when the sequence has no other byte."""
    bad = sum(int(np.count_nonzero(~_ACGT[seq[i:i + chunk]])) for i in range(0, seq.size, chunk))
    if bad == 0:
        return kmer_positions(off, k)
    total = 0
    for r in range(off.size - 1):
        a, b = int(off[r]), int(off[r + 1])
        if b - a < k:
            continue
        inv = np.concatenate(([0], np.cumsum(~_ACGT[seq[a:b]], dtype=np.int64)))
        total += int(np.count_nonzero(inv[k:] == inv[:-k]))
    return total


def host_cpu() -> dict:
    """CPU model and the number of CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 0
    return {"cpu_model": model, "host_cpus": n}


def workload(name: str):
    if name == "in_cache":
        return synth.in_cache_workload()
    if name == "out_of_cache":
        return synth.out_of_cache_workload()
    if name == "tiny":
        return synth.tiny_workload()
    raise SystemExit("unknown workload %s" % name)


def _prefix_batch(seq, off, n):
    """The first n bases of a record batch, with its offsets clipped."""
    n = int(min(n, seq.size))
    o = off.astype(np.uint64)
    return seq[:n], np.concatenate((o[o < n], [np.uint64(n)]))


def cpu_query_sample(w, ins_prefix, kmers, seed):
    """A bounded sample of the workload's query batch with about `kmers` k-mer
    positions: from every read class (short and long reads), the same share
    of reads as in the workload; negatives are the workload's own negative
    reads, positives are fresh reads of the same lengths drawn (with the same
    1% substitutions) from the inserted genome prefix, so that they are
    present in the sample's filter as the workload's positives are in the full
    filter."""
    qs, qoff = w["query"]
    k = w["k"]
    lens = np.diff(qoff.astype(np.int64))
    total = kmer_positions(qoff, k)
    frac = min(1.0, kmers / max(1, total))
    pseq, poff = ins_prefix
    longest = int(np.diff(poff.astype(np.int64)).max())

    def take(first, end):
        # reads of the class, or a cut of its first read when the class has
        # too few reads for the sample's share
        want = (end - first) * frac
        if want >= 1:
            n = int(round(want))
            return lens[first:first + n]
        return np.array([max(k, int(lens[first] * want))], dtype=np.int64)

    parts = []
    for ci, (p0, p1, n0, n1) in enumerate(w["read_classes"]):
        plen = np.minimum(take(p0, p1), longest)
        parts.append(synth.sample_reads(pseq, poff, plen.size, plen, seed + ci))
        nlen = take(n0, n1)
        a = int(qoff[n0])
        noff = np.concatenate(([0], np.cumsum(nlen))).astype(np.uint64)
        parts.append((qs[a:a + int(noff[-1])], noff))
    return synth.concat(*parts)


def cpu_baseline(w, budget_s: float = 12.0):
    """The oracle (plain C, unchanged arithmetic) on a bounded sample of the
    workload, timed on one thread and on every CPU this process may use, with
    one filter of the workload's full size (out of cache for the large
    workloads) that all threads share: the insert runs the oracle's
    shared-filter entry point (the same per-k-mer definition with atomic ORs)
    over k-1-overlapping pieces, the query splits the sample's reads over the
    threads.  About budget_s seconds of wall time in the timed regions."""
    import oracle

    k = w["k"]
    p = oracle.Params(w["k"], w["s"], w["m"], w["H"], w["bits"])
    ins, ioff = w["insert"]
    nt = host_cpu()["host_cpus"] or 1
    F = np.zeros(p.nwords, dtype=np.uint64)
    F[:] = 0  # touch the pages outside the timed regions
    # calibrate on a small prefix, then size the samples to the time budget
    n_cal = min(200_000, ins.size)
    t0 = time.perf_counter()
    oracle.insert(p, F, ins[:n_cal])
    per_kmer = max(1e-6, time.perf_counter() - t0) / max(1, n_cal - k + 1)
    share = 0.25 * budget_s / per_kmer  # k-mers one thread handles in a quarter of the budget

    # one thread
    s1 = _prefix_batch(ins, ioff, max(n_cal, share))
    F[:] = 0
    t0 = time.perf_counter()
    oracle.insert(p, F, *s1)
    t_ins = time.perf_counter() - t0
    k_ins = kmer_positions(s1[1], k)
    q1 = cpu_query_sample(w, s1, share, 7001)
    t0 = time.perf_counter()
    oracle.query(p, F, *q1)
    t_q = time.perf_counter() - t0
    k_q = kmer_positions(q1[1], k)
    single = (k_ins + k_q) / (t_ins + t_q)

    # every CPU, one shared filter
    sm = _prefix_batch(ins, ioff, max(s1[0].size, nt * share))
    qm = cpu_query_sample(w, sm, nt * share, 7101)
    F[:] = 0
    t0 = time.perf_counter()
    oracle.insert_parallel(p, F, *sm, threads=nt)
    t_ins_mt = time.perf_counter() - t0
    k_ins_mt = kmer_positions(sm[1], k)
    t0 = time.perf_counter()
    oracle.query_parallel(p, F, *qm, threads=nt)
    t_q_mt = time.perf_counter() - t0
    k_q_mt = kmer_positions(qm[1], k)
    del F
    multi = (k_ins_mt + k_q_mt) / (t_ins_mt + t_q_mt)
    return {"value": multi, "unit": "k-mers/s", "cores": nt, "kind": "oracle", **host_cpu(),
            "single_thread_value": single,
            "sample": "filter of the workload's size (%d bits, %.2f GiB) shared by all threads; %d threads: first %d "
                      "bases of the genome inserted (%d k-mers, atomic ORs) + %d query reads (%d k-mers: the "
                      "workload's negative reads of every class and as many positives drawn from the inserted "
                      "bases), insert %.3g k-mers/s, query %.3g k-mers/s; one thread: %d k-mers inserted + %d "
                      "queried, insert %.3g k-mers/s, query %.3g k-mers/s" % (
                          p.nwords * 64, p.nwords * 8 / 2**30, nt, sm[0].size, k_ins_mt, qm[1].size - 1, k_q_mt,
                          k_ins_mt / t_ins_mt, k_q_mt / max(t_q_mt, 1e-9), k_ins, k_q, k_ins / t_ins,
                          k_q / max(t_q, 1e-9))}


def stored_oracle(workload_name: str):
    """The oracle's stored results for a workload (tests/golden/segment_counts.json,
    written by tests/golden/segment_counts.py), or None."""
    path = os.path.join(ROOT, "tests", "golden", "segment_counts.json")
    if not os.path.exists(path):
        return None
    return json.load(open(path)).get(workload_name)


def stored_segments(workload_name: str, part: str, kmers: int):
    """Super-k-mer segments (one shard access each) of a workload's insert or
    query batch, as counted over every record by tests/golden/segment_counts.py
    and stored in tests/golden/segment_counts.json; None when absent or taken on
    a batch of another size."""
    path = os.path.join(ROOT, "tests", "golden", "segment_counts.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path)).get(workload_name, {}).get(part)
    if not d or int(d["kmers"]) != int(kmers):
        return None
    return int(d["segments"])


PROBE_NAMES = ["read", "rmw", "atomic4", "atomic1", "copy", "read_line", "rmw_line", "rmw_coherent",
               "rmw_line_coherent"]
# in-flight depths compiled into the probe per shard size (include/sbf_probe.h)
PROBE_DEPTHS = {32: (1, 4, 8, 16), 64: (1, 4, 8), 128: (1, 2, 4)}
PROBE_WGS = (1, 2, 4, 8)


def _probe_fn():
    import ctypes

    from paper_2606_24417_amd import build

    L = ctypes.CDLL(build.PROBE_LIB)
    fn = L.sbf_probe_random_access
    fn.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    return fn


def probe_once(mib, mode, shard_bytes=32, inflight=1, wgs_per_cu=4, ops=1 << 28):
    """One random-access probe launch configuration: (rate per second, ms)."""
    import ctypes

    rate, ms = ctypes.c_double(), ctypes.c_double()
    rc = _probe_fn()(int(mib) << 20, mode, shard_bytes, inflight, wgs_per_cu, ops, ctypes.byref(rate),
                     ctypes.byref(ms))
    if rc != 0:
        raise SystemExit("probe failed rc=%d (mode %d, %d MiB, %d B, depth %d, %d WG/CU)" % (
            rc, mode, mib, shard_bytes, inflight, wgs_per_cu))
    return rate.value, ms.value


def probe_ceiling(mib, mode, shard_bytes=32, ops=1 << 28):
    """Best rate of random shard operations over the in-flight depths and
    occupancies the probe offers: the ceiling a kernel doing the same
    accesses could reach.  Returns (best, table of every setting)."""
    table = []
    for d in PROBE_DEPTHS[shard_bytes]:
        for wg in PROBE_WGS:
            rate, ms = probe_once(mib, mode, shard_bytes, d, wg, ops)
            table.append({"inflight": d, "wgs_per_cu": wg, "G_per_s": round(rate / 1e9, 2), "ms": round(ms, 3)})
    best = max(table, key=lambda r: r["G_per_s"])
    return best, table


def run_probes(sizes_mib, modes=(0, 1, 2, 3), shard_bytes=(32,), quiet=False):
    """Random shard-access ceilings (include/sbf_probe.h) per buffer size."""
    out = []
    for mib in sizes_mib:
        for sb in shard_bytes:
            row = {"buffer_mib": mib, "shard_bytes": sb}
            for mode in modes:
                best, table = probe_ceiling(mib, mode, sb)
                row[PROBE_NAMES[mode]] = {"best_G_per_s": best["G_per_s"], "inflight": best["inflight"],
                                          "wgs_per_cu": best["wgs_per_cu"], "ms": best["ms"],
                                          "sweep": [(r["inflight"], r["wgs_per_cu"], r["G_per_s"]) for r in table]}
            out.append(row)
            print(json.dumps(row), file=sys.stderr if quiet else sys.stdout, flush=True)
    return out


def run_copy_probe(mib):
    rate, ms = probe_once(mib, 4)
    row = {"buffer_mib": mib, "copy_GBps": round(rate / 1e9, 1), "ms": round(ms, 4)}
    print(json.dumps(row), flush=True)
    return row


VALU_OPS = ["add32", "mul32", "mad64", "shl64", "bitop3", "cmp64"]
SBF_PROBE_VALU_ADD32 = 0


def valu_rate(op):
    """Wave-level instructions per second of VALU probe `op` (include/sbf_probe.h)."""
    import ctypes

    from paper_2606_24417_amd import build

    L = ctypes.CDLL(build.PROBE_LIB)
    fn = L.sbf_probe_valu
    fn.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    rate, ms = ctypes.c_double(), ctypes.c_double()
    rc = fn(op, ctypes.byref(rate), ctypes.byref(ms))
    if rc != 0:
        raise SystemExit("VALU probe failed rc=%d (op %d)" % (rc, op))
    return rate.value


def run_valu_probes():
    """Integer VALU issue rates from libsbf_probe.so (include/sbf_probe.h),
    as wave-level instructions per second and as a fraction of one wave64
    instruction per SIMD every four cycles at 2.4 GHz (256 CUs)."""
    import ctypes

    from paper_2606_24417_amd import build

    L = ctypes.CDLL(build.PROBE_LIB)
    fn = L.sbf_probe_valu
    fn.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    full = 256 * 4 * 2.4e9 / 4
    row = {"one_per_4_cycles_G_wave_instr_per_s": round(full / 1e9, 1)}
    for op, name in enumerate(VALU_OPS):
        rate, ms = ctypes.c_double(), ctypes.c_double()
        rc = fn(op, ctypes.byref(rate), ctypes.byref(ms))
        if rc != 0:
            raise SystemExit("VALU probe failed rc=%d (op %s)" % (rc, name))
        row[name] = {"G_wave_instr_per_s": round(rate.value / 1e9, 1), "of_one_per_4_cycles": round(rate.value / full, 3),
                     "ms": round(ms.value, 3)}
    print(json.dumps(row), flush=True)
    return row


def bench_batched(args):
    """Batched form: the whole insert batch and query batch in one persistent
    launch each, captured in a HIP graph, against the plain per-batch launch
    of the same reads in batches of 2000 reads.  Bits and answers must match."""
    import torch

    from paper_2606_24417_amd import Filter, Graph

    t0 = time.perf_counter()
    w = synth.batched_workload(args.scale)
    ins, ioff = w["insert"]
    qs, qoff = w["query"]
    k = w["k"]
    print("[bench] batched workload in %.1fs: %d+%d reads, %d+%d bases" % (
        time.perf_counter() - t0, ioff.size - 1, qoff.size - 1, ins.size, qs.size), file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    d_ins = torch.from_numpy(ins).to(dev)
    d_ioff = torch.from_numpy(ioff.view(np.int64)).to(dev)
    d_q = torch.from_numpy(qs).to(dev)
    d_qoff = torch.from_numpy(qoff.view(np.int64)).to(dev)
    f = Filter(w["k"], w["s"], w["m"], w["H"], w["bits"])
    report = f.autotune(d_ins, d_ioff, d_q, d_qoff)
    print(report, file=sys.stderr, flush=True)
    tuned = f.get_launch()
    out_g = torch.zeros(qs.size, dtype=torch.uint8, device=dev)
    g = Graph(f, d_ins, d_ioff, d_q, d_qoff, out_g, clear_first=True)
    # plain per-batch launches: batches of 2000 reads, one workgroup per tile
    per = 2000
    nb_i = (ioff.size - 1 + per - 1) // per
    nb_q = (qoff.size - 1 + per - 1) // per

    def batches(off, dseq, nb):
        res = []
        for b in range(nb):
            r0, r1 = b * per, min(off.size - 1, (b + 1) * per)
            a0, a1 = int(off[r0]), int(off[r1])
            res.append((dseq[a0:a1], torch.from_numpy((off[r0:r1 + 1] - off[r0]).view(np.int64)).to(dev), a0, a1))
        return res

    bi = batches(ioff, d_ins, nb_i)
    bq = batches(qoff, d_q, nb_q)
    out_p = torch.zeros(qs.size, dtype=torch.uint8, device=dev)
    h = Filter(w["k"], w["s"], w["m"], w["H"], w["bits"])

    def plain_step():
        h.clear()
        for seq, off, a0, a1 in bi:
            h.insert(seq, off)
        for seq, off, a0, a1 in bq:
            h.query(seq, off, out=out_p[a0:a1])

    def graph_step():
        g.launch()

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        times = []
        for _ in range(steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t) * 1e3)
        return float(np.median(times)), times

    plain_ms, _ = timed(plain_step, max(1, args.steps // 4))
    graph_ms, gt = timed(graph_step, args.steps)
    same_bits = bool(np.array_equal(f.get_bits(), h.get_bits()))
    same_ans = bool(torch.equal(out_g, out_p))
    n_kmers = kmer_positions(ioff, k) + kmer_positions(qoff, k)
    res = {"metric": "batched form: insert+query k-mers/s, one persistent launch under hipGraph vs per-batch launches",
           "value": n_kmers / (graph_ms * 1e-3), "unit": "k-mers/s", "graph_ms": round(graph_ms, 3),
           "plain_per_batch_ms": round(plain_ms, 3), "speedup": round(plain_ms / graph_ms, 2),
           "plain_batches": nb_i + nb_q, "reads_per_batch": per, "tuned": tuned,
           "identical_bits": same_bits, "identical_answers": same_ans,
           "p50_ms": round(float(np.percentile(gt, 50)), 3), "p99_ms": round(float(np.percentile(gt, 99)), 3),
           "config": {"workload": w["name"], "filter_bits": f.num_bits, "kmers": n_kmers}}
    g.close()
    f.close()
    h.close()
    print(json.dumps(res), flush=True)


def bench_served(args):
    """Served form: the out-of-cache (or, with --scale, smaller) genome stays
    resident; query requests of 1..10000 reads (log-uniform count, log-normal
    lengths) arrive by a Poisson process; report p50/p99 latency and k-mers/s
    per offered rate, with every answer checked against a direct query."""
    import torch

    from paper_2606_24417_amd import Filter, Server

    t0 = time.perf_counter()
    if args.scale >= 1.0:
        lens = synth.out_of_cache_contigs(301)
        g = synth.genome(lens, 301)
    else:
        g = synth.genome([int(20_000_000 * args.scale * 30)] * 5, 301)
    kmers = int(np.maximum(np.diff(g[1].astype(np.int64)) - 30, 0).sum())
    f = Filter(31, 28, 16, 4, 16 * kmers)
    dev = torch.device("cuda:0")
    f.insert(torch.from_numpy(g[0]).to(dev), torch.from_numpy(g[1].view(np.int64)).to(dev))
    torch.cuda.synchronize()
    print("[bench] served filter: %d bases inserted, %d bits, %.1fs" % (g[0].size, f.num_bits,
                                                                        time.perf_counter() - t0),
          file=sys.stderr, flush=True)
    rng = np.random.default_rng(501)
    nreq = args.requests
    counts = np.exp(rng.uniform(0, np.log(10_000), nreq)).astype(np.int64)
    reqs = []
    for i, c in enumerate(counts):
        L = synth.lognormal_lengths(int(c), 502_000 + i)
        if i % 2 == 0:
            seq, off = synth.sample_reads(g[0], g[1], int(c), L, 503_000 + i)
        else:
            seq, off = synth.random_reads(int(c), L, 504_000 + i)
        reqs.append((torch.from_numpy(seq).pin_memory(), off, torch.zeros(seq.size, dtype=torch.uint8).pin_memory()))
    total_bases = sum(int(r[1][-1]) for r in reqs)
    req_kmers = [kmer_positions(r[1], 31) for r in reqs]
    print("[bench] %d requests, %d bases, %.1fs" % (nreq, total_bases, time.perf_counter() - t0), file=sys.stderr,
          flush=True)
    # answers of a direct device query, for checking
    ref = []
    for seq, off, _ in reqs[: min(nreq, 64)]:
        ref.append(f.query(seq.to(dev), torch.from_numpy(off.view(np.int64)).to(dev)).cpu())
    slot_bases = max(1 << 26, max(int(r[1][-1]) for r in reqs))
    slot_recs = max(1 << 16, max(r[1].size - 1 for r in reqs))
    rows = []
    # one resident server for every rate, as in a serving process; its first
    # requests (fresh buffers and streams) are an untimed warm-up
    sv = Server(f, slots=args.slots, slot_bases=slot_bases, slot_records=slot_recs, max_pending=1 << 20)
    if args.window_us:
        sv.set_batch_window(args.window_us)
    for seq, off, out in reqs[:32]:
        sv.wait(sv.submit(seq, off, out))
    tk = [sv.submit(seq, off, out) for seq, off, out in reqs[:32]]
    for t in tk:
        sv.wait(t)
    prev = sv.stats()
    # The client's own CPU work between rates (refilling and comparing answer
    # tensors) runs on one thread: OpenMP workers keep spinning after a
    # parallel region, and with the client's spin loop and the server's
    # scheduler they can exceed a container's CPU quota, which throttles every
    # thread of the process, the scheduler included, for milliseconds.
    torch_threads = torch.get_num_threads()
    torch.set_num_threads(1)
    for rate in [float(x) for x in args.rates.split(",")]:
        for i in range(len(ref)):
            reqs[i][2].fill_(7)  # answers of this rate only
        time.sleep(0.2)
        gaps = rng.exponential(1.0 / rate, nreq)
        tickets = []
        start = time.perf_counter()
        due = start
        for i, (seq, off, out) in enumerate(reqs):
            due += gaps[i]
            while time.perf_counter() < due:
                pass
            tickets.append(sv.submit(seq, off, out))
        waits = [sv.wait(t) for t in tickets]
        lat = [x[0] for x in waits]
        span = time.perf_counter() - start
        st = sv.stats()
        batches = st["batches"] - prev["batches"]
        prev = st
        ok = all(torch.equal(reqs[i][2], ref[i]) for i in range(len(ref)))
        row = {"offered_req_per_s": rate, "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3), "kmers_per_s": sum(req_kmers) / span,
               "achieved_req_per_s": round(nreq / span, 1), "batches": batches,
               "mean_batch_requests": round(nreq / max(1, batches), 2),
               "max_batch_requests_so_far": st["max_batch_requests"], "answers_match_direct_query": ok,
               "p99_queue_ms": round(float(np.percentile([x[1] for x in waits], 99)), 3),
               "slowest": [{"ms": round(lat[i], 3), "queue_ms": round(waits[i][1], 3), "index": int(i),
                            "bases": int(reqs[i][1][-1])} for i in np.argsort(lat)[::-1][:3]]}
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    sv.close()
    torch.set_num_threads(torch_threads)
    res = {"metric": "served form: query latency p50/p99 (ms) and k-mers/s under Poisson arrivals",
           "unit": "ms", "higher_is_better": False, "value": rows[0]["p50_ms"], "rates": rows,
           "config": {"workload": "served: %d bp genome resident, %d requests of 1..10000 reads" % (g[0].size, nreq),
                      "filter_bits": f.num_bits, "slots": args.slots, "slot_bases": slot_bases,
                      "batch_window_us": args.window_us}}
    f.close()
    print(json.dumps(res), flush=True)


def bench_host(args):
    """Host-resident input: the in-cache workload's insert and query batches
    given to the host entry points (chunked, pipelined over two streams),
    with the caller's buffers pinned or pageable, against the same step on
    device-resident input.  Wall clock per step; answers and bits must match."""
    import torch

    from paper_2606_24417_amd import Filter

    w = workload("in_cache" if args.scale >= 1.0 else "tiny")
    k = w["k"]
    ins, ioff = w["insert"]
    qs, qoff = w["query"]
    n_kmers = kmer_positions(ioff, k) + kmer_positions(qoff, k)
    dev = torch.device("cuda:0")
    f = Filter(w["k"], w["s"], w["m"], w["H"], w["bits"])
    if args.staging_mib:
        f.set_staging_bytes(args.staging_mib << 20)
    d_ins = torch.from_numpy(ins).to(dev)
    d_ioff = torch.from_numpy(ioff.view(np.int64)).to(dev)
    d_q = torch.from_numpy(qs).to(dev)
    d_qoff = torch.from_numpy(qoff.view(np.int64)).to(dev)
    d_out = torch.empty(qs.size, dtype=torch.uint8, device=dev)
    p_ins = torch.from_numpy(ins).pin_memory()
    p_q = torch.from_numpy(qs).pin_memory()
    p_out = torch.zeros(qs.size, dtype=torch.uint8).pin_memory()
    h_out = np.zeros(qs.size, dtype=np.uint8)

    def device_step():
        f.clear(torch.cuda.current_stream())
        f.insert(d_ins, d_ioff)
        f.query(d_q, d_qoff, out=d_out)
        torch.cuda.synchronize()

    def pinned_step():
        f.clear()
        f.insert(p_ins, ioff)
        f.query(p_q, qoff, out=p_out)

    def pageable_step():
        f.clear()
        f.insert(ins, ioff)
        f.query(qs, qoff, out=h_out)

    def timed(fn):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(args.steps):
            t0 = time.perf_counter()
            fn()
            t.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(t))

    dev_ms = timed(device_step)
    ref_bits = f.get_bits()
    ref_ans = d_out.cpu().numpy()
    pin_ms = timed(pinned_step)
    same_pin = bool(np.array_equal(f.get_bits(), ref_bits)) and bool(np.array_equal(p_out.numpy(), ref_ans))
    page_ms = timed(pageable_step)
    same_page = bool(np.array_equal(f.get_bits(), ref_bits)) and bool(np.array_equal(h_out, ref_ans))
    # sequence in (one byte per base), answers back as bits (lane query)
    pcie_bytes = ins.size + qs.size + (qs.size + 7) // 8
    res = {"metric": "host-resident input: insert+query k-mers/s through the host entry points",
           "value": n_kmers / (pin_ms * 1e-3), "unit": "k-mers/s", "higher_is_better": True,
           "pinned_ms": round(pin_ms, 3), "pageable_ms": round(page_ms, 3), "device_resident_ms": round(dev_ms, 3),
           "pageable_kmers_per_s": n_kmers / (page_ms * 1e-3),
           "device_resident_kmers_per_s": n_kmers / (dev_ms * 1e-3),
           "transfer_loss_pinned": round(1 - dev_ms / pin_ms, 4),
           "transfer_loss_pageable": round(1 - dev_ms / page_ms, 4),
           "host_link_GBps_pinned": round(pcie_bytes / (pin_ms * 1e-3) / 1e9, 2),
           "identical_to_device_path": same_pin and same_page,
           "staging_bytes": (args.staging_mib << 20) if args.staging_mib else 64 << 20,
           "config": {"workload": w["name"], "filter_bits": f.num_bits, "kmers": n_kmers, "bases_in": int(ins.size + qs.size)}}
    f.close()
    print(json.dumps(res), flush=True)


FAMILY_NAMES = {1: "lane", 2: "generic", 3: "wide-shard", 4: "run-time parameter"}


def bench_sweep(args):
    """(s, m, H) sweep at k = 31 over s in 24..31, m in 12..20, H in 1..8 on the
    in-cache workload (scaled by --scale): per point, the FPR on the negative
    reads, a zero-false-negative check on genome k-mers, and insert and query
    kernel time of the run-time parameter kernels (one kernel family over the
    whole grid, so that times compare parameters) and of the family the
    library picks by itself (compiled lane or wide-shard kernels where they
    exist).  Then the shard geometries (4, 8, 16 words) at (28, 16, 4) with
    every family that runs them.  The FPR against filter size is the
    fpr_curve workload."""
    import torch

    from paper_2606_24417_amd import VARIANT_AUTO, VARIANT_PARAM, Filter

    t0 = time.perf_counter()
    w = synth.in_cache_workload(args.scale)
    k = w["k"]
    ins, ioff = w["insert"]
    qs, qoff = w["query"]
    npos = w["n_pos_records"]
    neg0 = int(qoff[npos])
    neg_kmers = kmer_positions(qoff[npos:] - qoff[npos], k)
    n_ins_kmers = kmer_positions(ioff, k)
    n_q_kmers = kmer_positions(qoff, k)
    dev = torch.device("cuda:0")
    d_ins = torch.from_numpy(ins).to(dev)
    d_ioff = torch.from_numpy(ioff.view(np.int64)).to(dev)
    d_q = torch.from_numpy(qs).to(dev)
    d_qoff = torch.from_numpy(qoff.view(np.int64)).to(dev)
    d_out = torch.empty(qs.size, dtype=torch.uint8, device=dev)
    d_ref = torch.empty(qs.size, dtype=torch.uint8, device=dev)
    fn_len = int(min(ioff[1], 1_000_000))
    d_fn = d_ins[:fn_len]
    d_fn_out = torch.empty(fn_len - k + 1, dtype=torch.uint8, device=dev)
    print("[bench] sweep workload in %.1fs: %d + %d k-mers" % (time.perf_counter() - t0, n_ins_kmers, n_q_kmers),
          file=sys.stderr, flush=True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def timed(f, out, insert_only=False):
        ti, tq = [], []
        for rep in range(3):
            f.clear(torch.cuda.current_stream())
            ev[0].record()
            f.insert(d_ins, d_ioff)
            ev[1].record()
            if not insert_only:
                f.query(d_q, d_qoff, out=out)
            ev[2].record()
            torch.cuda.synchronize()
            ti.append(ev[0].elapsed_time(ev[1]))
            tq.append(ev[1].elapsed_time(ev[2]))
        return round(float(np.median(ti)), 4), round(float(np.median(tq)), 4)

    rows = []
    grid = [(s_, m_, h_) for s_ in range(24, 32) for m_ in range(12, 21) for h_ in range(1, 9)]
    if args.sweep_points:
        grid = grid[: args.sweep_points]
    for i, (s_, m_, h_) in enumerate(grid):
        f = Filter(k, s_, m_, h_, w["bits"])
        f.variant = VARIANT_PARAM
        pi, pq = timed(f, d_out)
        f.query(d_fn, out=d_fn_out)
        torch.cuda.synchronize()
        fp = int(d_out[neg0:].sum().item())
        no_fn = bool(int(d_fn_out.sum().item()) == fn_len - k + 1)
        # the insert's other strategy: one atomic OR per segment word
        f.set_insert_mode(1)
        pa, _ = timed(f, d_out, insert_only=True)
        f.set_insert_mode(0)
        row = {"s": s_, "m": m_, "H": h_, "fpr": fp / max(1, neg_kmers), "param_insert_ms": pi,
               "param_insert_atomic_ms": pa, "param_query_ms": pq, "zero_fn": no_fn}
        f.variant = VARIANT_AUTO
        if f.variant != VARIANT_PARAM:
            # a compiled family for this point: its own times, and the same
            # answers as the run-time parameter kernels
            ai, aq = timed(f, d_ref)
            row.update({"variant": FAMILY_NAMES[f.variant], "insert_ms": ai, "query_ms": aq,
                        "answers_equal": bool(torch.equal(d_out, d_ref))})
        else:
            row.update({"variant": FAMILY_NAMES[VARIANT_PARAM], "insert_ms": pi, "query_ms": pq})
        rows.append(row)
        f.close()
        if (i + 1) % 48 == 0:
            print("[bench] sweep %d/%d points" % (i + 1, len(grid)), file=sys.stderr, flush=True)
    # shard geometry (4, 8, 16 words per shard) at (28, 16, 4), each with
    # every family that runs it
    geometry = []
    for S, variants in ((4, (1, 4, 2)), (8, (3, 4, 2)), (16, (3, 4, 2))):
        for variant in variants:
            f = Filter(k, 28, 16, 4, w["bits"], shard_words=S)
            f.variant = variant
            ti, tq = timed(f, d_out)
            geometry.append({"shard_words": S, "kernels": FAMILY_NAMES[variant], "filter_bits": f.num_bits,
                             "fpr": int(d_out[neg0:].sum().item()) / max(1, neg_kmers), "insert_ms": ti,
                             "query_ms": tq})
            f.close()
    all_ok = all(r["zero_fn"] for r in rows)
    same = all(r.get("answers_equal", True) for r in rows)
    best = min(rows, key=lambda r: r["fpr"])
    fastest = min(rows, key=lambda r: r["param_insert_ms"] + r["param_query_ms"])
    res = {"metric": "sweep: FPR and insert/query kernel ms per (s,m,H) at k=31, 16 bits per k-mer",
           "unit": "fpr", "points": len(rows), "zero_false_negatives_everywhere": all_ok,
           "compiled_and_param_answers_equal": same, "best_fpr": best, "fastest_param": fastest,
           "at_28_16_4": next((r for r in rows if (r["s"], r["m"], r["H"]) == (28, 16, 4)), None),
           "rows": rows, "geometry": geometry,
           "config": {"workload": w["name"] + " (scale %g)" % args.scale, "filter_bits": w["bits"],
                      "insert_kmers": n_ins_kmers, "query_kmers": n_q_kmers, "negative_kmers": neg_kmers}}
    print(json.dumps(res), flush=True)


def bench_fpr_curve(args):
    """False-positive rate against filter size (Section "False Positive Rate":
    independent random k-mers queried after a genome insert): the in-cache
    genome (scaled by --scale) is inserted at (31, 28, 16, 4) into filters of
    2^22 .. 2^38 and 2^39 bits, with 4- and 16-word shards, and --fpr-kmers
    independent uniform random 31-mers (generated on the device in batches of
    2^26, each k-mer followed by an 'N' so that it is its own record, and kept
    resident) are queried.  Each point reports the measured count of k-mers
    answered present beside the filter's own prediction (sbf_estimate_fpr: the
    mean over shards of the product of its sectors' set-bit fractions, the
    exact expectation for uniformly sharded queries with ideal s-mer hashes)
    and the 99.9% Poisson interval of that expectation."""
    import torch
    from scipy.stats import poisson

    from paper_2606_24417_amd import Filter

    t0 = time.perf_counter()
    w = synth.in_cache_workload(args.scale)
    k = w["k"]
    ins, ioff = w["insert"]
    n_ins = kmer_positions(ioff, k)
    dev = torch.device("cuda:0")
    d_ins = torch.from_numpy(ins).to(dev)
    d_ioff = torch.from_numpy(ioff.view(np.int64)).to(dev)
    total = int(args.fpr_kmers)
    per = 1 << 26
    batches = []
    for i in range((total + per - 1) // per):
        n = min(per, total - i * per)
        batches.append(synth.separated_uniform_kmers(n, k, 7000 + i, device=dev))
    out = torch.empty(per * (k + 1), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    print("[bench] fpr curve: %d genome k-mers, %d random %d-mers in %d batches ready in %.1fs" % (
        n_ins, total, k, len(batches), time.perf_counter() - t0), file=sys.stderr, flush=True)
    sizes = [1 << lg for lg in range(22, 39, 2)] + [1 << 39]
    rows = []
    for S in (4, 16):
        for bits in sizes:
            f = Filter(k, 28, 16, 4, bits, shard_words=S)
            f.insert(d_ins, d_ioff)
            est, set_bits = f.estimate_fpr()
            present = 0
            for b in batches:
                o = f.query(b, out=out[: b.numel() - k + 1])
                present += int(o.sum(dtype=torch.int64).item())
            f.close()
            mu = total * est
            lo, hi = (int(poisson.ppf(0.0005, mu)), int(poisson.ppf(0.9995, mu))) if mu > 0 else (0, 0)
            rows.append({"shard_words": S, "bits": bits, "bits_per_kmer": round(bits / n_ins, 3),
                         "set_fraction": round(set_bits / bits, 6), "present": present, "fpr": present / total,
                         "predicted_fpr": est, "expected": round(mu, 3), "interval_99_9": [lo, hi],
                         "within": bool(lo <= present <= hi)})
            print("[bench] S=%2d bits 2^%d: %d present (%.3g), predicted %.4g [%d, %d]" % (
                S, bits.bit_length() - 1, present, present / total, mu, lo, hi), file=sys.stderr, flush=True)
    res = {"metric": "FPR of independent uniform random 31-mers vs filter size at (31,28,16,4)", "unit": "fpr",
           "random_kmers": total, "rows": rows, "all_within_interval": all(r["within"] for r in rows),
           "config": {"workload": w["name"] + " (scale %g)" % args.scale, "genome_kmers": n_ins}}
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="out_of_cache",
                    choices=["in_cache", "out_of_cache", "tiny", "batched", "served", "host", "sweep", "fpr_curve"])
    ap.add_argument("--fpr-kmers", type=float, default=1e9, help="fpr_curve: random k-mers per filter size")
    ap.add_argument("--sweep-points", type=int, default=0, help="sweep: only the first n (s,m,H) points")
    ap.add_argument("--staging-mib", type=int, default=0, help="host: chunk size of the host entry points")
    ap.add_argument("--scale", type=float, default=1.0, help="batched/served workload size factor")
    ap.add_argument("--rates", default="1000,2000,5000,10000,20000,50000", help="served: offered requests/s")
    ap.add_argument("--requests", type=int, default=1000, help="served: requests per offered rate")
    ap.add_argument("--slots", type=int, default=4, help="served: server execution slots")
    ap.add_argument("--window-us", type=int, default=0, help="served: batching window in microseconds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-in-cache", action="store_true",
                    help="out_of_cache: skip the in-cache workload reported as a second key")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the live roofline probes (random access out of cache, 32-bit add rate in cache)")
    ap.add_argument("--variant", type=int, default=0, help="0 auto, 1 rolling, 2 generic, 3 wide-shard, 4 run-time parameter")
    ap.add_argument("--shard-words", type=int, default=4, choices=[4, 8, 16],
                    help="64-bit words per shard (4 = the paper's 256-bit shard)")
    ap.add_argument("--tile", type=str, default="", help="k-mers per lane for insert,query (0 = default)")
    ap.add_argument("--bits", type=int, default=0, help="filter size override (default: the workload's)")
    ap.add_argument("--query-mode", type=int, default=0, help="0 lane-sequential, 1 leader load + broadcast, 2 every lane loads")
    ap.add_argument("--insert-mode", type=int, default=0, help="0 two-pass, 1 atomic")
    ap.add_argument("--launch", type=str, default="",
                    help="persistent workgroups per CU for insert,query (0 = one workgroup per tile; "
                         "default: the library's)")
    ap.add_argument("--autotune", action="store_true", help="run the library autotuner on the workload first")
    ap.add_argument("--probe", action="store_true",
                    help="print random-access, copy and integer VALU roofline probes, then exit")
    ap.add_argument("--probe-valu", action="store_true", help="print the integer VALU issue-rate probes, then exit")
    ap.add_argument("--probe-read-mib", type=int, default=0,
                    help="run only the random 32-byte read probe on a buffer of this many MiB (counter calibration)")
    ap.add_argument("--probe-copy-mib", type=int, default=0,
                    help="run only the streaming-copy probe on a buffer of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (--gpus %d requested)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    if args.probe:
        run_probes([2, 32, 256, 1024, 8192])
        run_probes([8192], modes=(0, 1), shard_bytes=(64, 128))
        run_probes([8192], modes=(5, 6), shard_bytes=(32, 64, 128))
        run_probes([256, 8192], modes=(7, 8), shard_bytes=(32, 128))
        for mib in (2, 32, 256, 8192):
            run_copy_probe(mib)
        run_valu_probes()
        return
    if args.probe_valu:
        run_valu_probes()
        return
    if args.probe_copy_mib:
        run_copy_probe(args.probe_copy_mib)
        return
    if args.probe_read_mib:
        # one fixed setting, for counter calibration
        rate, ms = probe_once(args.probe_read_mib, 0, 32, 8, 4)
        print(json.dumps({"buffer_mib": args.probe_read_mib, "read_G_per_s": round(rate / 1e9, 2), "ms": ms,
                          "ops": 1 << 28}), flush=True)
        return

    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "served":
        bench_served(args)
        return
    if args.workload == "host":
        bench_host(args)
        return
    if args.workload == "sweep":
        bench_sweep(args)
        return
    if args.workload == "fpr_curve":
        bench_fpr_curve(args)
        return

    res = measure(args, args.workload, with_cpu=not args.no_cpu_baseline)
    if args.workload == "out_of_cache" and not args.no_in_cache:
        # the in-cache workload as a second key of the same line
        sub = measure(args, "in_cache", with_cpu=False)
        res["in_cache"] = {key: sub[key] for key in (
            "value", "ms_per_step", "config", "p50_batch_ms", "p99_batch_ms", "insert_kmers_per_s",
            "query_kmers_per_s", "insert_ms_median", "query_ms_median", "query_present", "oracle_check",
            "roofline", "roofline_other")}
    print(json.dumps(res), flush=True)
    # a mismatch with the stored oracle results fails the run; a workload
    # without stored results (another filter size, say) only reports so
    if any(r.get("oracle_check", {}).get("ok") is False for r in (res, res.get("in_cache", {}))):
        sys.exit(1)


def _sha256(a: np.ndarray) -> str:
    h = hashlib.sha256()
    step = 1 << 28
    for i in range(0, a.size, step):
        h.update(memoryview(np.ascontiguousarray(a[i:i + step])).cast("B"))
    return h.hexdigest()


def measure(args, name, with_cpu):
    """One workload: W untimed and K timed steps (clear the filter, mark the
    record starts of both batches, insert the genome, query the reads), with
    HIP events around the insert and the query on torch's current stream, on
    which the library launches its kernels.  After the timed steps the filter
    and answers are checked against the oracle's stored digests."""
    import torch

    from paper_2606_24417_amd import Filter

    t_gen = time.perf_counter()
    w = workload(name)
    if args.bits:
        w["bits"] = args.bits
    S = args.shard_words
    # stored oracle results (segment counts, digests) of this workload at this geometry
    key = name if S == 4 else "%s_S%d" % (name, S)
    t_gen = time.perf_counter() - t_gen
    k = w["k"]
    ins, ioff = w["insert"]
    qs, qoff = w["query"]
    n_ins_kmers = kmer_positions(ioff, k)
    n_q_kmers = kmer_positions(qoff, k)
    print("[bench] workload %s generated in %.1fs: insert %d bases (%d k-mers), query %d bases (%d k-mers)" % (
        name, t_gen, ins.size, n_ins_kmers, qs.size, n_q_kmers), file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    d_ins = torch.from_numpy(ins).to(dev)
    d_ioff = torch.from_numpy(ioff.view(np.int64)).to(dev)
    d_q = torch.from_numpy(qs).to(dev)
    d_qoff = torch.from_numpy(qoff.view(np.int64)).to(dev)
    d_out = torch.empty(qs.size, dtype=torch.uint8, device=dev)
    f = Filter(w["k"], w["s"], w["m"], w["H"], w["bits"], shard_words=S)
    if args.variant:
        f.variant = args.variant
    if args.tile:
        f.set_tile(*(int(x) for x in args.tile.split(",")))
    f.set_query_mode(args.query_mode)
    f.set_insert_mode(args.insert_mode)
    if args.launch:
        li, lq = (int(x) for x in args.launch.split(","))
        f.set_launch(li, lq)
    if args.autotune:
        report = f.autotune(d_ins, d_ioff, d_q, d_qoff)
        print(report, file=sys.stderr, flush=True)
    ins_starts = Filter.mark_record_starts(d_ioff, ins.size)
    q_starts = Filter.mark_record_starts(d_qoff, qs.size)
    torch.cuda.synchronize()

    def step(ev=None):
        if ev:
            ev[0].record()
        f.clear(torch.cuda.current_stream())
        Filter.mark_record_starts(d_ioff, ins.size, ins_starts)
        Filter.mark_record_starts(d_qoff, qs.size, q_starts)
        if ev:
            ev[1].record()
        f.insert_marked(d_ins, ins_starts)
        if ev:
            ev[2].record()
        f.query_marked(d_q, q_starts, d_out)
        if ev:
            ev[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([e[0].elapsed_time(e[3]) for e in evs])
    ins_ms = np.array([e[1].elapsed_time(e[2]) for e in evs])
    q_ms = np.array([e[2].elapsed_time(e[3]) for e in evs])
    ms_per_step = wall * 1e3 / args.steps

    # Check of this run, outside the timed region: the filter left by the last
    # step and the answers of its query against the oracle's results for the
    # whole workload, stored by tests/golden/segment_counts.py.
    ans = d_out.cpu().numpy()
    n_q_valid = int(ans.sum(dtype=np.int64))
    stored = stored_oracle(key)
    check = {"ok": None, "note": "no stored oracle result for this workload"}
    if stored and "oracle_answers" in stored and stored["query"]["bases"] == qs.size and not args.bits:
        ans_ok = _sha256(ans) == stored["oracle_answers"]["sha256"]
        bits_ok = _sha256(f.get_bits()) == stored["oracle_filter"]["sha256"]
        check = {"ok": bool(ans_ok and bits_ok and n_q_valid == stored["oracle_answers"]["present"]),
                 "present": n_q_valid, "oracle_present": stored["oracle_answers"]["present"],
                 "answers_sha256_equal": ans_ok, "filter_sha256_equal": bits_ok}
    del ans
    print("[bench] %s oracle check: %s" % (name, json.dumps(check)), file=sys.stderr, flush=True)

    total_kmers = n_ins_kmers + n_q_kmers
    value = total_kmers / (ms_per_step * 1e-3)
    q_rate = n_q_kmers / (np.median(q_ms) * 1e-3)
    i_rate = n_ins_kmers / (np.median(ins_ms) * 1e-3)
    # Roofline of the dominant work: the insert is two launches (store pass,
    # then repair walk) unless it runs in atomic mode; the query is one.
    settings = f.get_launch()
    family = FAMILY_NAMES[f.variant]
    tile_i, tile_q = f.get_tile()
    settings.update({"family": family, "shard_words": S, "insert_kmers_per_lane": tile_i,
                     "query_kmers_per_lane": tile_q})
    ins_launches = 1 if settings["insert_mode"] == 1 else 2
    if family == "wide-shard":
        q_kernel = "query_wide_kernel<31,28,16,4,%d,%d>" % (S, tile_q)
        ins_kernels = ("insert_wide_kernel<31,28,16,4,%d,%d> store pass + repair walk (two launches)" % (S, tile_i),
                       "insert_wide_kernel<31,28,16,4,%d,%d> (atomic)" % (S, tile_i))
    elif family == "run-time parameter":
        q_kernel = "query_param_kernel<%d,%d>" % (S, tile_q)
        ins_kernels = ("insert_param_kernel<%d,%d> store pass + query_param_kernel<%d,%d> repair walk"
                       % (S, tile_i, S, tile_i), "insert_param_kernel<%d,%d> (atomic)" % (S, tile_i))
    else:
        q_kernel = {0: "query_lane_kernel", 1: "query_rolling_kernel (leader)", 2: "query_rolling_kernel (direct)"}[
            settings["query_mode"]] + "<31,28,16,4>"
        ins_kernels = ("insert_rolling_kernel<31,28,16,4> store pass + query_lane_kernel<31,28,16,4> repair walk",
                       "insert_rolling_kernel<31,28,16,4> (atomic)")
    in_cache = name != "out_of_cache"

    valu = None
    if in_cache and not args.no_probe:
        valu = round(valu_rate(SBF_PROBE_VALU_ADD32) * 64 / 1e12, 2)
    probe = None
    if not in_cache and not args.no_probe:
        # ceilings of random shard reads and read-modify-writes of this shard
        # size over an 8 GiB buffer (best over in-flight depth and occupancy,
        # with the shard moved by one lane or split over shard/16 lanes as the
        # wide-shard kernels do), measured now
        # (the insert's read-modify-writes race between XCDs, so its stores
        # write through to the coherence point; the probe does the same)
        probe = {}
        sb = 8 * S
        for access, mode, line_mode in (("read", 0, 5), ("rmw", 7, 8)):
            best, _ = probe_ceiling(8192, mode, sb)
            best_l, _ = probe_ceiling(8192, line_mode, sb)
            best_l["lanes_per_shard"] = sb // 16
            probe[access] = best if best["G_per_s"] >= best_l["G_per_s"] else best_l
        print("[bench] random-access ceilings (8 GiB, %d B): %s" % (sb, json.dumps(probe)), file=sys.stderr, flush=True)

    def roofline(part, ms, kmers, launches):
        if in_cache:
            ops = OPS_PER_KMER[part] * kmers
            achieved = ops / (ms * 1e-3) / 1e12
            r = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_INT_TOPS, "unit": "TOP/s (int32)",
                 "frac": round(achieved / PEAK_INT_TOPS, 4), "ops_per_kmer": OPS_PER_KMER[part]}
        else:
            nseg = stored_segments(key, part, kmers)
            seqs = w[part]
            if nseg is None:
                r = {"bound": "hbm", "achieved": None, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": None,
                     "note": "no stored segment count for this workload"}
            else:
                per_seg = 8 * S if part == "query" else 16 * S
                nbytes = nseg * per_seg + seqs[0].size * (2 if part == "query" else 1)
                achieved = nbytes / (ms * 1e-3) / 1e9
                r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "segments": nseg,
                     "algorithmic_bytes": nbytes}
        r["traffic"] = counter_traffic(key, part, kmers)
        if in_cache and valu is not None:
            # the same algorithmic ops against the 32-bit add rate measured now
            # on this GPU (simple 32-bit ops issue faster than one wave64
            # instruction per four cycles on gfx950, so this rate exceeds the
            # unit-count peak)
            r["valu_probe"] = {"add32_T_lane_ops_per_s": valu, "frac": round(r["achieved"] / valu, 4)}
        if probe is not None and r.get("segments"):
            # segments (one random access of a whole shard each) per second against
            # the probe's best random read rate (query) or read-modify-write
            # rate (insert)
            seg_rate = r["segments"] / (ms * 1e-3)
            best = probe["read" if part == "query" else "rmw"]
            peak = best["G_per_s"] * 1e9
            r["random_access"] = {"segments_per_s": seg_rate, "probe_ceiling_per_s": peak,
                                  "probe": ("read" if part == "query" else "read-modify-write, coherent stores")
                                  + " %d B" % (8 * S),
                                  "probe_setting": {"inflight": best["inflight"], "wgs_per_cu": best["wgs_per_cu"]},
                                  "frac": round(seg_rate / peak, 4)}
        r["launches"] = launches
        r["kernel_ms"] = round(ms, 4)
        return r

    q_mean = float(np.mean(q_ms))
    i_mean = float(np.mean(ins_ms))
    roof_q = roofline("query", q_mean, n_q_kmers, 1)
    roof_q["kernel"] = q_kernel
    roof_i = roofline("insert", i_mean, n_ins_kmers, ins_launches)
    roof_i["kernel"] = ins_kernels[0] if ins_launches == 2 else ins_kernels[1]
    if q_mean >= i_mean / ins_launches:
        roof, roof_other = roof_q, roof_i
    else:
        roof, roof_other = roof_i, roof_q

    res = {
        "metric": "insert & query k-mers/s at k=31,s=28,m=16,H=4 on 1 MI355X; p50/p99 batch ms",
        "value": value,
        "unit": "k-mers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": w["name"], "k": w["k"], "s": w["s"], "m": w["m"], "H": w["H"],
                   "filter_bits": f.num_bits, "shard_words": S, "insert_kmers": n_ins_kmers, "query_kmers": n_q_kmers,
                   "insert_valid_kmers": valid_kmers(ins, ioff, k), "query_valid_kmers": valid_kmers(qs, qoff, k),
                   "parallelism": "single GPU"},
        "p50_batch_ms": round(float(np.percentile(step_ms, 50)), 4),
        "p99_batch_ms": round(float(np.percentile(step_ms, 99)), 4),
        "insert_kmers_per_s": i_rate,
        "query_kmers_per_s": q_rate,
        "insert_ms_median": round(float(np.median(ins_ms)), 4),
        "query_ms_median": round(float(np.median(q_ms)), 4),
        "query_present": n_q_valid,
        "oracle_check": check,
        "settings": settings,
        "roofline": roof,
        "roofline_other": roof_other,
        "cpu_baseline": None,
    }
    f.close()
    del d_ins, d_q, d_out, d_ioff, d_qoff, ins_starts, q_starts
    torch.cuda.empty_cache()
    if with_cpu:
        t0 = time.perf_counter()
        res["cpu_baseline"] = cpu_baseline(w)
        print("[bench] cpu baseline in %.1fs" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    return res


if __name__ == "__main__":
    main()
