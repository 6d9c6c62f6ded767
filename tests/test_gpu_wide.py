"""GPU parity of the wide-shard super-k-mer kernels (shards of 4, 8 and 16
words) against the oracle at the same shard geometry, bit for bit: record
batches with invalid bases and short records, lengths around the tile size
(256 lanes x 16 or 32 k-mers), both insert strategies, persistent launches,
heavy shard contention, the tile-length setting and the shard-geometry
autotuner."""

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


def dev(x):
    return torch.from_numpy(np.array(x, copy=True)).cuda()


def doff(off):
    return dev(np.asarray(off, dtype=np.uint64).view(np.int64))


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError("%s differ at %d of %d positions, first %s: got %s want %s" % (
            what, bad.size, got.size, bad[:5].tolist(), got[bad[:5]].tolist(), want[bad[:5]].tolist()))


def batch(rng, nrec, mean_len, p_invalid=0.0, short_every=7):
    lens = rng.integers(1, 2 * mean_len, size=nrec)
    lens[::short_every] = rng.integers(0, 40, size=lens[::short_every].size)  # records shorter than k
    off = np.concatenate(([0], np.cumsum(lens))).astype(np.uint64)
    seq = synth.uniform_acgt(int(off[-1]), int(rng.integers(1 << 30))).copy()
    if p_invalid:
        bad = rng.random(seq.size) < p_invalid
        seq[bad] = rng.choice(np.frombuffer(b"NnX-.", dtype=np.uint8), bad.sum())
    lw = rng.random(seq.size) < 0.01
    seq[lw] |= 0x20
    return seq, off


def wide_filter(k, s, m, H, bits, S, tile=0, mode=0, launch=None):
    from paper_2606_24417_amd import VARIANT_WIDE, Filter

    f = Filter(k, s, m, H, bits, shard_words=S)
    f.variant = VARIANT_WIDE
    assert f.variant == VARIANT_WIDE
    if tile:
        f.set_tile(tile, tile)
    f.set_insert_mode(mode)
    if launch is not None:
        f.set_launch(*launch)
    return f


def run_both(params, S, ins, q, **kw):
    k, s, m, H, bits = params
    p = oracle.Params(k, s, m, H, bits, shard_words=S)
    F = oracle.insert(p, p.empty(), *ins)
    want = oracle.query(p, F, *q)
    f = wide_filter(k, s, m, H, bits, S, **kw)
    f.insert(dev(ins[0]), doff(ins[1]))
    ans = f.query(dev(q[0]), doff(q[1]))
    torch.cuda.synchronize()
    got_bits, got_ans = f.get_bits(), ans.cpu().numpy()
    f.close()
    assert_same(got_bits, F, "filter words")
    assert_same(got_ans, want, "answers")
    return F, want


@pytest.mark.parametrize("S", [4, 8, 16])
@pytest.mark.parametrize("H", [4, 8])
@pytest.mark.parametrize("tile", [16, 32])
@pytest.mark.parametrize("mode", [0, 1])
def test_wide_matches_oracle(S, H, tile, mode):
    rng = np.random.default_rng(1000 * S + 100 * H + 10 * tile + mode)
    ins = batch(rng, 120, 1500, 0.001)
    q0 = batch(rng, 90, 900, 0.001)
    # half of the query records are inserted records: present k-mers occur
    qs = np.concatenate([ins[0][: int(ins[1][40])], q0[0]])
    qo = np.concatenate([ins[1][:41], q0[1][1:] + ins[1][40]])
    print("case wide S=%d H=%d tile=%d mode=%d" % (S, H, tile, mode), flush=True)
    _, want = run_both((31, 28, 16, H, 1 << 18), S, ins, (qs, qo), tile=tile, mode=mode)
    assert want.sum() > 0


@pytest.mark.parametrize("S", [4, 16])
@pytest.mark.parametrize("n", [31, 32, 4095 + 31, 4096 + 30, 4096 + 31, 3 * 4096 + 45, 8192 * 2 + 29])
def test_wide_lengths_around_tiles(S, n):
    seq = synth.uniform_acgt(n, n).copy()
    off = np.array([0, n], dtype=np.uint64)
    print("case wide length", S, n, flush=True)
    _, want = run_both((31, 28, 16, 4, 1 << 16), S, (seq, off), (seq, off))
    # the filter's own sequence: every k-mer is present
    assert want[: n - 30].all() and not want[n - 30:].any()


@pytest.mark.parametrize("S", [8, 16])
@pytest.mark.parametrize("alphabet", [b"AC", b"ACGT"])
def test_wide_contention(S, alphabet):
    """Few shards (2^10 bits: one or two shards) receive every segment of
    every workgroup: the plain read-modify-writes race constantly and the
    repair walk must restore every dropped bit."""
    rng = np.random.default_rng(S + len(alphabet))
    seq = np.frombuffer(alphabet, dtype=np.uint8)[rng.integers(0, len(alphabet), 400_000)].copy()
    off = np.array([0, seq.size], dtype=np.uint64)
    print("case wide contention", S, alphabet, flush=True)
    run_both((31, 28, 16, 4, 1 << 10), S, (seq, off), (seq[:50_000], np.array([0, 50_000], dtype=np.uint64)))


@pytest.mark.parametrize("S", [8, 16])
@pytest.mark.parametrize("wgs", [0, 1, 4])
def test_wide_persistent_launches(S, wgs):
    """Persistent grids smaller than the tile count (the 10 Mbp genome has
    about 2400 tiles of 4096 k-mers) give the oracle's results."""
    w = synth.in_cache_workload(scale=0.1)
    print("case wide persistent", S, wgs, flush=True)
    run_both((w["k"], w["s"], w["m"], w["H"], w["bits"]), S, w["insert"], w["query"], launch=(wgs, wgs))


def test_auto_variant_picks_wide_kernels_for_wide_shards():
    from paper_2606_24417_amd import VARIANT_GENERIC, VARIANT_PARAM, VARIANT_ROLLING, VARIANT_WIDE, Filter, SBFError

    for S in (8, 16):
        f = Filter(31, 28, 16, 4, 1 << 20, shard_words=S)
        assert f.variant == VARIANT_WIDE
        f.variant = VARIANT_ROLLING  # the super-k-mer kernels of this geometry
        assert f.variant == VARIANT_WIDE
        assert f.get_tile() == (16, 16)
        f.set_tile(32, 16)
        assert f.get_tile() == (32, 16)
        with pytest.raises(SBFError):
            f.set_tile(48, 16)
        f.variant = VARIANT_GENERIC
        assert f.get_tile() == (0, 0)
        with pytest.raises(SBFError):
            f.set_tile(16, 16)
        f.close()
    f = Filter(31, 28, 16, 4, 1 << 20)
    assert f.variant == VARIANT_ROLLING and f.get_tile() == (64, 48)
    f.set_tile(64, 32)
    assert f.get_tile() == (64, 32)
    with pytest.raises(SBFError):
        f.set_tile(16, 48)
    f.close()
    # no wide kernel for this parameter set: the run-time parameter kernels run
    f = Filter(31, 27, 16, 4, 1 << 20, shard_words=16)
    assert f.variant == VARIANT_PARAM
    with pytest.raises(SBFError):
        f.variant = VARIANT_WIDE
    f.close()
    # nor a run-time parameter kernel (H > 8): the generic kernels run
    f = Filter(31, 27, 16, 9, 1 << 20, shard_words=8)
    assert f.variant == VARIANT_GENERIC
    f.close()


@pytest.mark.parametrize("ltile,qtile", [(64, 32), (32, 32), (64, 48)])
def test_lane_kernel_tile_lengths(ltile, qtile):
    """The 4-word lane kernels at their non-default tile lengths."""
    from paper_2606_24417_amd import Filter

    w = synth.in_cache_workload(scale=0.02)
    params = (w["k"], w["s"], w["m"], w["H"], w["bits"])
    p = oracle.Params(*params)
    F = oracle.insert(p, p.empty(), *w["insert"])
    want = oracle.query(p, F, *w["query"])
    print("case lane tiles", ltile, qtile, flush=True)
    for mode in (0, 1):
        f = Filter(*params)
        f.set_tile(ltile, qtile)
        f.set_insert_mode(mode)
        f.insert(dev(w["insert"][0]), doff(w["insert"][1]))
        ans = f.query(dev(w["query"][0]), doff(w["query"][1]))
        torch.cuda.synchronize()
        assert_same(f.get_bits(), F, "filter words (insert mode %d)" % mode)
        assert_same(ans.cpu().numpy(), want, "answers")
        f.close()


def test_geometry_autotuner():
    """sbf_autotune_geometry reports every geometry, returns the fastest one
    within the FPR bound, and its FPR equals the oracle's count at that
    geometry; an impossible bound returns the lowest-FPR geometry."""
    from paper_2606_24417_amd import autotune_geometry

    w = synth.in_cache_workload(scale=0.02)
    k, s, m, H, bits = w["k"], w["s"], w["m"], w["H"], w["bits"] // 4  # 5.4 bits per k-mer: visible FPR
    ins, ioff = w["insert"]
    qs, qoff = w["query"]
    nneg = (qoff.size - 1) // 2
    neg = qs[int(qoff[nneg]):]
    noff = qoff[nneg:] - qoff[nneg]
    args = (k, s, m, H, bits, dev(ins), doff(ioff), dev(qs), doff(qoff), dev(neg), doff(noff))
    fprs = {}
    for S in (4, 8, 16):
        p = oracle.Params(k, s, m, H, bits, shard_words=S)
        F = oracle.insert(p, p.empty(), ins, ioff)
        a = oracle.query(p, F, neg, noff)
        full = oracle.query(p, np.full(p.nwords, np.iinfo(np.uint64).max, dtype=np.uint64), neg, noff)
        fprs[S] = a.sum() / full.sum()
    print("oracle FPR by shard words:", fprs, flush=True)
    res = autotune_geometry(*args, max_fpr=1.0)
    print(res["report"], flush=True)
    for S in (4, 8, 16):
        assert ("shard %2d words" % S) in res["report"]
    assert res["shard_words"] in (4, 8, 16)
    assert res["fpr"] == pytest.approx(fprs[res["shard_words"]], rel=1e-12)
    res = autotune_geometry(*args, max_fpr=0.0)
    best = min(fprs, key=lambda S: fprs[S])
    assert res["shard_words"] == best and res["fpr"] == pytest.approx(fprs[best], rel=1e-12)
    assert "no geometry meets the FPR bound" in res["report"]
