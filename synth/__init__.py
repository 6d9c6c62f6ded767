"""Seeded synthetic DNA workloads (inputs only; no filter arithmetic).

Both the GPU path and the CPU oracle read the arrays this module returns; it
imports neither of them.  Stand-ins for the paper's genomes, which are not
available here:

* background: iid bases, GC content 41% (P(A)=P(T)=0.295, P(C)=P(G)=0.205);
* repeats: families of length U{300..6000} with U{2..50} copies, each copy the
  family consensus with 1% iid substitutions, placed forward-strand at random
  non-overlapping positions until 5% of the bases are repeat copies;
* reads: positives start uniformly inside one contig (forward strand, 1% iid
  substitutions), negatives are fresh background sequence.

Sequences are ``uint8`` ASCII arrays; record batches carry ``uint64`` offsets
with ``nrec + 1`` entries (record r is ``seq[off[r]:off[r+1]]``).  A query
batch's ``read_classes`` lists (first positive record, end, first negative
record, end) for each read class (short and long reads).
"""

from __future__ import annotations

import concurrent.futures as _cf
import os

import numpy as np

ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)
_CHUNK = 1 << 26


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _lut(gc: float) -> np.ndarray:
    """65536-entry table mapping a uniform 16-bit draw to a base with the given
    GC content (A and T share 1-gc, C and G share gc)."""
    at = (1.0 - gc) / 2.0
    cuts = np.array([at, 0.5, 0.5 + gc / 2.0]) * 65536.0
    u = np.arange(65536)
    idx = np.searchsorted(np.round(cuts).astype(np.int64), u, side="right")
    return ACGT[idx]


def background(n: int, seed, gc: float = 0.41) -> np.ndarray:
    """n iid bases.  Deterministic for a given seed regardless of threads:
    chunk c of 2^26 bases draws from its own spawned seed."""
    n = int(n)
    out = np.empty(n, dtype=np.uint8)
    if n == 0:
        return out
    lut = _lut(gc)
    nchunks = (n + _CHUNK - 1) // _CHUNK
    ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
    seeds = ss.spawn(nchunks)

    def work(c):
        a = c * _CHUNK
        b = min(n, a + _CHUNK)
        draws = np.random.default_rng(seeds[c]).integers(0, 65536, b - a, dtype=np.uint16)
        np.take(lut, draws, out=out[a:b])

    if nchunks == 1:
        work(0)
    else:
        with _cf.ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nchunks)))
    return out


def uniform_acgt(n: int, seed) -> np.ndarray:
    """n iid uniform bases (GC 50%)."""
    return background(n, seed, gc=0.5)


def substitute(seq: np.ndarray, rate: float, rng: np.random.Generator) -> np.ndarray:
    """Copy of seq with iid substitutions at the given rate, each to one of the
    three other bases chosen uniformly."""
    out = seq.copy()
    if rate <= 0 or seq.size == 0:
        return out
    step = 1 << 24
    for a in range(0, seq.size, step):
        part = out[a:a + step]
        pos = np.flatnonzero(rng.random(part.size, dtype=np.float32) < rate)
        if pos.size:
            code = np.searchsorted(ACGT, part[pos])
            code = (code + rng.integers(1, 4, pos.size)) % 4
            part[pos] = ACGT[code]
    return out


def genome(contig_lengths, seed, gc: float = 0.41, repeat_frac: float = 0.05,
           fam_len=(300, 6000), copies=(2, 50), divergence: float = 0.01):
    """Multi-contig genome with diverged repeat families.  Returns (seq, off)."""
    lengths = np.asarray(contig_lengths, dtype=np.int64)
    off = np.zeros(lengths.size + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lengths)
    total = int(off[-1])
    ss = np.random.SeedSequence(seed)
    s_bg, s_rep = ss.spawn(2)
    seq = background(total, s_bg, gc)
    rng = np.random.default_rng(s_rep)
    budget = int(repeat_frac * total)
    copy_fam, copy_len, cons = [], [], []
    placed = 0
    while placed < budget:
        L = int(rng.integers(fam_len[0], fam_len[1] + 1))
        c = int(rng.integers(copies[0], copies[1] + 1))
        c = max(1, min(c, (budget - placed + L - 1) // L))
        cons.append(background(L, rng.integers(0, 2**63), gc))
        copy_fam += [len(cons) - 1] * c
        copy_len += [L] * c
        placed += L * c
    ncopy = len(copy_fam)
    if ncopy == 0:
        return seq, off
    copy_len = np.asarray(copy_len, dtype=np.int64)
    # assign copies to contigs in proportion to contig length, then lay them
    # out with random gaps so that they never overlap or cross a contig end
    contig = rng.choice(lengths.size, size=ncopy, p=lengths / lengths.sum())
    order = rng.permutation(ncopy)
    for ci in range(lengths.size):
        mine = order[contig[order] == ci]
        if mine.size == 0:
            continue
        used = int(copy_len[mine].sum())
        free = int(lengths[ci]) - used
        if free < 0:
            raise ValueError("repeat copies do not fit in contig %d" % ci)
        cuts = np.sort(rng.integers(0, free + 1, mine.size))
        gaps = np.diff(np.concatenate([[0], cuts]))
        pos = int(off[ci])
        for j, g in zip(mine, gaps):
            pos += int(g)
            L = int(copy_len[j])
            seq[pos:pos + L] = substitute(cons[copy_fam[j]], divergence, rng)
            pos += L
    return seq, off


def sample_reads(seq: np.ndarray, off: np.ndarray, n: int, lengths, seed,
                 sub_rate: float = 0.01):
    """n forward-strand reads, each inside one contig, with iid substitutions.
    lengths: an int or an array of n read lengths.  Returns (reads, roff)."""
    rng = np.random.default_rng(seed)
    n = int(n)
    lens = np.full(n, int(lengths), dtype=np.int64) if np.isscalar(lengths) else np.asarray(lengths, dtype=np.int64)
    clen = np.diff(off.astype(np.int64))
    roff = np.zeros(n + 1, dtype=np.uint64)
    roff[1:] = np.cumsum(lens)
    out = np.empty(int(roff[-1]), dtype=np.uint8)
    # contig chosen with probability proportional to its number of start positions
    room = np.maximum(clen[None, :] - lens[:, None] + 1, 0).astype(np.float64)
    cum = np.cumsum(room, axis=1)
    ci = (cum < rng.random(n)[:, None] * cum[:, -1:]).sum(axis=1)
    ci = np.minimum(ci, clen.size - 1)
    start = off[ci].astype(np.int64) + (rng.random(n) * room[np.arange(n), ci]).astype(np.int64)
    ro = roff.astype(np.int64)
    per = max(1, (1 << 24) // max(1, int(lens.mean())))
    for a in range(0, n, per):
        b = min(n, a + per)
        L = lens[a:b]
        idx = np.repeat(start[a:b] - ro[a:b], L) + np.arange(int(ro[b] - ro[a])) + ro[a]
        out[ro[a]:ro[b]] = seq[idx]
    return substitute(out, sub_rate, rng), roff


def random_reads(n: int, lengths, seed, gc: float = 0.41):
    """n reads of fresh background sequence.  Returns (reads, roff)."""
    n = int(n)
    lens = np.full(n, int(lengths), dtype=np.int64) if np.isscalar(lengths) else np.asarray(lengths, dtype=np.int64)
    roff = np.zeros(n + 1, dtype=np.uint64)
    roff[1:] = np.cumsum(lens)
    return background(int(roff[-1]), seed, gc), roff


def lognormal_lengths(n: int, seed, median: float = 500.0, sigma: float = 1.0,
                      lo: int = 100, hi: int = 50000) -> np.ndarray:
    """Read lengths, log-normal, truncated to [lo, hi] by redrawing."""
    rng = np.random.default_rng(seed)
    mu = np.log(median) - 0.08
    out = np.empty(0, dtype=np.int64)
    while out.size < n:
        x = np.round(rng.lognormal(mu, sigma, 2 * n)).astype(np.int64)
        out = np.concatenate([out, x[(x >= lo) & (x <= hi)]])
    return out[:n]


def concat(*batches):
    """Concatenate (seq, off) record batches into one batch."""
    seqs = [b[0] for b in batches]
    offs = []
    base = 0
    for s, o in batches:
        offs.append(o[:-1].astype(np.uint64) + np.uint64(base))
        base += int(o[-1])
    offs.append(np.array([base], dtype=np.uint64))
    return np.concatenate(seqs), np.concatenate(offs)


# --- the workloads ----------------------------------------------------------

def tiny_workload():
    """1 Mbp uniform sequence into 2^24 bits; query a 500 kbp substring of it
    plus 500 kbp of fresh sequence (two records)."""
    ins = uniform_acgt(1_000_000, 101)
    rng = np.random.default_rng(102)
    a = int(rng.integers(0, ins.size - 500_000 + 1))
    pos = ins[a:a + 500_000].copy()
    neg = uniform_acgt(500_000, 103)
    q, qoff = concat((pos, np.array([0, pos.size], dtype=np.uint64)),
                     (neg, np.array([0, neg.size], dtype=np.uint64)))
    return dict(name="tiny: 1 Mbp into 2^24 bits", k=31, s=28, m=16, H=4, bits=1 << 24,
                insert=(ins, np.array([0, ins.size], dtype=np.uint64)), query=(q, qoff),
                n_pos_records=1, read_classes=[(0, 1, 1, 2)])


def in_cache_workload(scale: float = 1.0):
    """100 Mbp genome (5 contigs of 20 Mbp) at 16 bits per k-mer; 1M positive
    150 bp reads with 1% substitutions plus 1M random 150 bp reads."""
    contig = int(20_000_000 * scale)
    nreads = int(1_000_000 * scale)
    g = genome([contig] * 5, 201)
    pos = sample_reads(g[0], g[1], nreads, 150, 202)
    neg = random_reads(nreads, 150, 203)
    q = concat(pos, neg)
    return dict(name="in-cache: 100 Mbp genome, 2M x 150 bp reads", k=31, s=28, m=16, H=4,
                bits=16 * int(g[1][-1]), insert=g, query=q, n_pos_records=nreads,
                read_classes=[(0, nreads, nreads, 2 * nreads)])


def out_of_cache_contigs(seed=301, total=3_000_000_000):
    rng = np.random.default_rng(seed)
    lens = []
    while sum(lens) < total:
        lens.append(int(rng.integers(50_000_000, 250_000_001)))
    lens[-1] -= sum(lens) - total
    return lens


def out_of_cache_workload(scale: float = 1.0):
    """3 Gbp multi-contig genome at 16 bits per k-mer; 5M+5M 150 bp reads and
    50k+50k long reads of U{10000..20000} bp (positives with 1% errors)."""
    total = int(3_000_000_000 * scale)
    lens = out_of_cache_contigs(301, total)
    g = genome(lens, 301)
    nshort = int(5_000_000 * scale)
    nlong = int(50_000 * scale)
    rng = np.random.default_rng(304)
    llen = rng.integers(10_000, 20_001, 2 * nlong)
    pos = sample_reads(g[0], g[1], nshort, 150, 302)
    neg = random_reads(nshort, 150, 303)
    lpos = sample_reads(g[0], g[1], nlong, llen[:nlong], 304)
    lneg = random_reads(nlong, llen[nlong:], 305)
    q = concat(pos, neg, lpos, lneg)
    return dict(name="out-of-cache: 3 Gbp genome, 10M x 150 bp + 100k long reads", k=31, s=28,
                m=16, H=4, bits=16 * total, insert=g, query=q,
                read_classes=[(0, nshort, nshort, 2 * nshort),
                              (2 * nshort, 2 * nshort + nlong, 2 * nshort + nlong, 2 * nshort + 2 * nlong)])


def batched_workload(scale: float = 1.0):
    """2M reads of log-normal length (median 500 bp, 100..50000) sampled with
    1% substitutions from a 100 Mbp genome, inserted; then 2M more reads of the
    same length law, half positive and half random, queried."""
    n = int(2_000_000 * scale)
    g = genome([int(20_000_000 * max(scale, 0.05))] * 5, 201)
    ins = sample_reads(g[0], g[1], n, lognormal_lengths(n, 401), 402)
    half = n // 2
    qpos = sample_reads(g[0], g[1], half, lognormal_lengths(half, 403), 404)
    qneg = random_reads(n - half, lognormal_lengths(n - half, 405), 406)
    q = concat(qpos, qneg)
    kmers = int(np.maximum(np.diff(ins[1].astype(np.int64)) - 30, 0).sum())
    return dict(name="batched: 2M log-normal reads (median 500 bp) inserted, 2M queried", k=31, s=28, m=16, H=4,
                bits=16 * kmers, insert=ins, query=q)


def separated_uniform_kmers(n: int, k: int, seed: int, device="cpu"):
    """n independent uniform k-mers as one record of n*(k+1) bases on a torch
    device: each k-mer is followed by one 'N', so the record's valid k-mers
    are exactly the n drawn ones, at positions i*(k+1).  Drawn with torch's
    seeded generator on that device (the stream differs between devices)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    c = torch.randint(0, 4, (n, k + 1), generator=g, device=device, dtype=torch.uint8)
    # codes 0..3 -> 'A' 'C' 'G' 'T' (65, 67, 71, 84) without a gather
    seq = 65 + 2 * c + 2 * (c >= 2).to(torch.uint8) + 11 * (c == 3).to(torch.uint8)
    seq[:, k] = ord("N")
    return seq.reshape(-1)
