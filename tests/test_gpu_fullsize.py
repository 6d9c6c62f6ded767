"""Full-size GPU checks in the launch configuration bench.py times.

Every filter word and every answer byte is compared with the oracle:

* in-cache workload (100 Mbp genome at 16 bits per k-mer, 2M reads): the
  oracle runs here, on every CPU (threads over k-1-overlapping pieces, atomic
  ORs into one filter), and both results are compared element by element;
* out-of-cache workload (3 Gbp genome into 8 GiB, 10.1M reads) and batched
  workload (2M log-normal reads inserted and 2M queried through one HIP
  graph): the GPU's filter and answers are compared with the SHA-256 digests
  of the oracle's, per 64 MiB block, stored by tests/golden/segment_counts.py
  (which calls only the oracle and the input generator);
* a reduced batched workload (5% of the reads) through the graph against the
  oracle run here.

Properties that hold at any size are checked as well: every inserted k-mer is
present, and false positives on random reads match the prediction from the
filter's own sector popcounts.
"""

import hashlib
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth
from conftest import golden

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def Filter(*a, **kw):
    from paper_2606_24417_amd import Filter as F

    return F(*a, **kw)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def off_dev(off):
    return torch.from_numpy(off.astype(np.uint64).view(np.int64)).cuda()


def stored(name):
    return json.load(open(golden("segment_counts.json")))[name]


def block_digests(a: np.ndarray, block: int):
    """SHA-256 per block of `block` elements (threads; hashlib releases the
    interpreter lock on large buffers)."""
    a = np.ascontiguousarray(a)
    starts = range(0, a.size, block)
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(lambda i: hashlib.sha256(memoryview(a[i:i + block]).cast("B")).hexdigest(), starts))


def check_against_stored(name, bits, ans):
    """Filter words and answer bytes against the oracle's stored digests; on a
    mismatch, name the blocks that differ."""
    d = stored(name)
    fb = d["oracle_filter"]["block_words"]
    got = block_digests(bits, fb)
    bad = [i for i, (x, y) in enumerate(zip(got, d["oracle_filter"]["block_sha256"])) if x != y]
    assert bits.size == d["oracle_filter"]["words"] and not bad, \
        "filter differs from the oracle's in %d of %d blocks of %d words (first: %s)" % (
            len(bad), len(got), fb, bad[:8])
    assert int(np.bitwise_count(bits).sum(dtype=np.int64)) == d["oracle_filter"]["set_bits"]
    ab = d["oracle_answers"]["block_bytes"]
    got = block_digests(ans, ab)
    bad = [i for i, (x, y) in enumerate(zip(got, d["oracle_answers"]["block_sha256"])) if x != y]
    assert ans.size == d["oracle_answers"]["bytes"] and not bad, \
        "answers differ from the oracle's in %d of %d blocks of %d bytes (first: %s)" % (
            len(bad), len(got), ab, bad[:8])
    assert int(ans.sum(dtype=np.int64)) == d["oracle_answers"]["present"]


def sample_records(rng, off, n):
    nrec = off.size - 1
    return np.sort(rng.choice(nrec, size=min(n, nrec), replace=False))


def check_fpr_prediction(p, F, ans, qs, qoff, idx):
    c = np.bincount(np.arange(p.H) % 4, minlength=4)
    z1 = p.k - p.s + 1
    expect = 0.0
    got = 0
    for r in idx:
        read = qs[int(qoff[r]):int(qoff[r + 1])]
        sh = oracle.kmer_shards(p, read)
        ok = sh != np.iinfo(np.uint64).max
        words = F.reshape(-1, 4)[sh[ok].astype(np.int64)]
        pop = np.bitwise_count(words).astype(np.float64)
        expect += np.prod((pop / 64.0) ** (z1 * c[None, :]), axis=1).sum()
        got += int(ans[int(qoff[r]):int(qoff[r]) + sh.size][ok].sum())
    print("FPR check: %d false positives, %.1f expected" % (got, expect), flush=True)
    # k-mers of one read share s-mers, so the count is over-dispersed: allow
    # 25% plus 5 Poisson standard deviations
    assert abs(got - expect) <= 0.25 * expect + 5 * np.sqrt(expect) + 2


def genome_kmers_present(self_ans, off, k):
    valid = np.ones(self_ans.size, dtype=bool)
    for r in range(off.size - 1):
        valid[max(int(off[r]), int(off[r + 1]) - (k - 1)):int(off[r + 1])] = False
    return bool(self_ans[valid].all()) and not self_ans[~valid].any()


def test_in_cache_full_size():
    w = synth.in_cache_workload()
    print("case in-cache full size", flush=True)
    p = oracle.Params(w["k"], w["s"], w["m"], w["H"], w["bits"])
    ins, ioff = w["insert"]
    qs, qoff = w["query"]
    f = Filter(w["k"], w["s"], w["m"], w["H"], w["bits"])
    d_ins = to_dev(ins)
    f.insert(d_ins, off_dev(ioff))
    d_ans = f.query(to_dev(qs), off_dev(qoff))
    d_self = f.query(d_ins, off_dev(ioff))
    torch.cuda.synchronize()
    bits = f.get_bits()
    ans = d_ans.cpu().numpy()
    self_ans = d_self.cpu().numpy()
    f.close()
    assert genome_kmers_present(self_ans, ioff, w["k"])
    print("oracle insert of 100 Mbp and query of 2M reads", flush=True)
    F = oracle.insert_parallel(p, p.empty(), ins, ioff)
    bad = np.flatnonzero(bits != F)
    assert bad.size == 0, "filter differs in %d of %d words" % (bad.size, F.size)
    want = oracle.query_parallel(p, F, qs, qoff)
    bad = np.flatnonzero(ans != want)
    assert bad.size == 0, "answers differ at %d of %d positions (first %s)" % (bad.size, ans.size, bad[:8])
    check_against_stored("in_cache", bits, ans)
    # false positives among sampled negative reads match the prediction from
    # the filter's own sector popcounts (ideal s-mer hash); random reads share
    # the genome's 41% GC, which loads shards unevenly, so the uniform-sequence
    # closed form does not apply here
    rng = np.random.default_rng(1)
    nneg = (qoff.size - 1) // 2
    nidx = nneg + sample_records(rng, qoff[nneg:] - qoff[nneg], 20_000)
    check_fpr_prediction(p, bits, ans, qs, qoff, nidx)


def test_out_of_cache_full_size():
    w = synth.out_of_cache_workload()
    print("case out-of-cache full size", flush=True)
    k = w["k"]
    p = oracle.Params(w["k"], w["s"], w["m"], w["H"], w["bits"])
    assert p.nshards == 1 << 28
    ins, ioff = w["insert"]
    qs, qoff = w["query"]
    d = stored("out_of_cache")
    assert d["insert"]["bases"] == ins.size and d["query"]["bases"] == qs.size
    f = Filter(w["k"], w["s"], w["m"], w["H"], w["bits"])
    d_ins = to_dev(ins)
    d_ioff = off_dev(ioff)
    f.insert(d_ins, d_ioff)
    d_ans = f.query(to_dev(qs), off_dev(qoff))
    torch.cuda.synchronize()
    ans = d_ans.cpu().numpy()
    del d_ans
    # every genome k-mer is present
    d_self = f.query(d_ins, d_ioff)
    torch.cuda.synchronize()
    present = int(d_self.sum().item())
    del d_self
    n_valid = int(sum(max(0, int(ioff[r + 1] - ioff[r]) - k + 1) for r in range(ioff.size - 1)))
    assert present == n_valid
    bits = f.get_bits()
    f.close()
    print("comparing 8 GiB of filter and 3 GB of answers with the oracle's digests", flush=True)
    check_against_stored("out_of_cache", bits, ans)
    short_n = 10_000_000
    fpr = ans[int(qoff[short_n // 2]):int(qoff[short_n])].sum() / (short_n // 2 * (150 - k + 1))
    print("out-of-cache FPR on random reads: %.3g" % fpr, flush=True)
    rng = np.random.default_rng(2)
    nidx = short_n // 2 + sample_records(rng, qoff[short_n // 2:short_n + 1] - qoff[short_n // 2], 20_000)
    check_fpr_prediction(p, bits, ans, qs, qoff, nidx)


def _graph_run(w):
    from paper_2606_24417_amd import Graph

    ins, ioff = w["insert"]
    qs, qoff = w["query"]
    d_ins, d_ioff, d_q, d_qoff = to_dev(ins), off_dev(ioff), to_dev(qs), off_dev(qoff)
    d_out = torch.full((qs.size,), 7, dtype=torch.uint8, device="cuda")
    f = Filter(w["k"], w["s"], w["m"], w["H"], w["bits"])
    g = Graph(f, d_ins, d_ioff, d_q, d_qoff, d_out, clear_first=True)
    g.launch()
    torch.cuda.synchronize()
    first = d_out.cpu().numpy()
    d_out.fill_(9)
    g.launch()  # a replay gives the same filter and answers
    torch.cuda.synchronize()
    bits = f.get_bits()
    ans = d_out.cpu().numpy()
    g.close()
    f.close()
    assert np.array_equal(first, ans)
    return bits, ans


def test_batched_full_size_graph():
    """The batched workload itself (2M reads of log-normal length up to 50 kbp,
    inserted and then 2M queried, in one persistent launch each under a HIP
    graph) against the oracle's stored digests."""
    w = synth.batched_workload()
    print("case batched full size", flush=True)
    d = stored("batched")
    assert d["insert"]["bases"] == w["insert"][0].size and d["query"]["bases"] == w["query"][0].size
    bits, ans = _graph_run(w)
    check_against_stored("batched", bits, ans)


def test_batched_reduced_graph_against_oracle():
    w = synth.batched_workload(0.05)
    print("case batched 5%", flush=True)
    p = oracle.Params(w["k"], w["s"], w["m"], w["H"], w["bits"])
    bits, ans = _graph_run(w)
    F = oracle.insert_parallel(p, p.empty(), *w["insert"])
    assert np.array_equal(bits, F)
    assert np.array_equal(ans, oracle.query_parallel(p, F, *w["query"]))
