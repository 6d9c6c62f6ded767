"""The allocation-free query entry point (sbf_query_batch_dev_noalloc) against
the allocating one (sbf_query_batch_dev), through the C ABI: two calls in a
row on one filter, the second with a smaller batch, must give answers
identical to the allocating form and to the oracle; a batch above the fixed
scratch is rejected before any device work."""

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _batch(seed, n_reads, lo, hi):
    rng = np.random.default_rng(seed)
    lens = rng.integers(lo, hi + 1, size=n_reads)
    off = np.concatenate(([0], np.cumsum(lens))).astype(np.uint64)
    seq = synth.uniform_acgt(int(off[-1]), seed + 1)
    # a few invalid bases, so that validity and record starts both matter
    bad = rng.choice(seq.size, size=max(1, seq.size // 5000), replace=False)
    seq[bad] = ord("N")
    return seq, off


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _off(o):
    return torch.from_numpy(o.astype(np.uint64).view(np.int64)).cuda()


# (1, 1): a persistent grid of one workgroup per CU, smaller than the first
# batch's tile count, so its work-queue counters (in the scratch) are used
@pytest.mark.parametrize("launch", [(1, 1), (0, 0)])
def test_noalloc_query_matches_allocating_query(launch):
    from paper_2606_24417_amd import Filter

    k, s, m, H, bits = 31, 28, 16, 4, 1 << 22
    ins = synth.uniform_acgt(3_000_000, 7)
    f = Filter(k, s, m, H, bits)
    f.set_launch(*launch)
    f.insert(_dev(ins))
    p = oracle.Params(k, s, m, H, bits)
    F = oracle.insert(p, p.empty(), ins)
    # the filter's own sequence as reads plus random reads: present and absent
    # answers both occur; the second batch is smaller than the first
    for seed, n_reads, lo, hi in [(11, 20000, 20, 400), (12, 700, 1, 200)]:
        seq, off = _batch(seed, n_reads, lo, hi)
        half = int(off[n_reads // 2])
        seq[:half] = ins[:half]
        print("case noalloc launch=%s seed=%d bases=%d" % (launch, seed, seq.size), flush=True)
        d_seq, d_off = _dev(seq), _off(off)
        out_na = torch.full((seq.size,), 7, dtype=torch.uint8, device="cuda")
        f.query_batch_dev_noalloc(d_seq, d_off, out_na)
        out_ref = f.query(d_seq, d_off)
        torch.cuda.synchronize()
        got, ref = out_na.cpu().numpy(), out_ref.cpu().numpy()
        want = oracle.query(p, F, seq, off)
        assert np.array_equal(got, ref)
        assert np.array_equal(got, want)
        assert want[:half].sum() > 0
    f.close()


# every kernel family behind the same entry point: compiled lane kernels at
# their default (above), run-time parameter kernels (4- and 8-word shards),
# wide-shard kernels and the generic kernels
@pytest.mark.parametrize("params,S,variant", [((31, 26, 14, 5), 4, 0), ((31, 27, 17, 3), 8, 4),
                                              ((31, 28, 16, 4), 16, 3), ((31, 28, 16, 4), 4, 2)])
def test_noalloc_query_every_family(params, S, variant):
    from paper_2606_24417_amd import Filter

    bits = 1 << 22
    ins = synth.uniform_acgt(2_000_000, 17)
    f = Filter(*params, bits, shard_words=S)
    if variant:
        f.variant = variant
    f.set_launch(1, 1)
    f.insert(_dev(ins))
    p = oracle.Params(*params, bits, shard_words=S)
    F = oracle.insert(p, p.empty(), ins)
    for seed, n_reads, lo, hi in [(21, 8000, 20, 400), (22, 500, 1, 200)]:
        seq, off = _batch(seed, n_reads, lo, hi)
        half = int(off[n_reads // 2])
        seq[:half] = ins[:half]
        print("case noalloc family params=%s S=%d variant=%d seed=%d" % (params, S, f.variant, seed), flush=True)
        d_seq, d_off = _dev(seq), _off(off)
        out_na = torch.full((seq.size,), 7, dtype=torch.uint8, device="cuda")
        f.query_batch_dev_noalloc(d_seq, d_off, out_na)
        out_ref = f.query(d_seq, d_off)
        torch.cuda.synchronize()
        got, ref = out_na.cpu().numpy(), out_ref.cpu().numpy()
        want = oracle.query(p, F, seq, off)
        assert np.array_equal(got, ref)
        assert np.array_equal(got, want)
        assert want[:half].sum() > 0
    f.close()


def test_noalloc_query_rejects_batches_above_its_scratch():
    from paper_2606_24417_amd import Filter, SBFError, SBF_E_INVAL

    f = Filter(31, 28, 16, 4, 1 << 20)
    n = (1 << 26) + 1
    seq = torch.zeros(n, dtype=torch.uint8, device="cuda")
    off = _off(np.array([0, n], dtype=np.uint64))
    out = torch.zeros(n, dtype=torch.uint8, device="cuda")
    with pytest.raises(SBFError) as e:
        f.query_batch_dev_noalloc(seq, off, out)
    assert e.value.code == SBF_E_INVAL
    f.close()
