"""GPU parity of the run-time parameter super-k-mer kernels (any (k, s, m, H)
with m <= k <= 32, s <= k, H <= 8; shards of 4, 8 and 16 words) against the
oracle at the same parameters, bit for bit: the corners and interior of the
(s, m, H) grid of the paper's parameter study at k = 31, other k down to 1
and up to 32, record batches with invalid bases and short records, lengths
around the tile (256 lanes x 8 or 16 k-mers), both insert strategies,
persistent launches, heavy shard contention, and the family's selection."""

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


def param_filter(k, s, m, H, bits, S, tile=0, mode=0, launch=None):
    from paper_2606_24417_amd import VARIANT_PARAM, Filter

    f = Filter(k, s, m, H, bits, shard_words=S)
    f.variant = VARIANT_PARAM
    assert f.variant == VARIANT_PARAM
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
    f = param_filter(k, s, m, H, bits, S, **kw)
    f.insert(dev(ins[0]), doff(ins[1]))
    ans = f.query(dev(q[0]), doff(q[1]))
    torch.cuda.synchronize()
    got_bits, got_ans = f.get_bits(), ans.cpu().numpy()
    f.close()
    assert_same(got_bits, F, "filter words")
    assert_same(got_ans, want, "answers")
    return F, want


def mixed(rng, mean_len=1200):
    ins = batch(rng, 80, mean_len, 0.001)
    q0 = batch(rng, 60, mean_len, 0.001)
    # half of the query records are inserted records: present k-mers occur
    qs = np.concatenate([ins[0][: int(ins[1][30])], q0[0]])
    qo = np.concatenate([ins[1][:31], q0[1][1:] + ins[1][30]])
    return ins, (qs, qo)


# corners and interior points of s in 24..31, m in 12..20, H in 1..8 at k = 31
GRID = [(24, 12, 1), (24, 20, 8), (31, 12, 8), (31, 20, 1), (27, 15, 3), (29, 17, 5), (26, 19, 6), (25, 13, 7),
        (30, 14, 2), (28, 16, 4), (28, 16, 8), (31, 16, 4)]


@pytest.mark.parametrize("s,m,H", GRID)
@pytest.mark.parametrize("mode", [0, 1])
def test_grid_points_match_oracle(s, m, H, mode):
    rng = np.random.default_rng(10000 * s + 100 * m + 10 * H + mode)
    ins, q = mixed(rng)
    print("case param grid s=%d m=%d H=%d mode=%d" % (s, m, H, mode), flush=True)
    _, want = run_both((31, s, m, H, 1 << 17), 4, ins, q, mode=mode)
    assert want.sum() > 0


# other k: m = k (one m-mer), s = k (one s-mer), m = 1 (w = 32), k = 1, tiny k
OTHER_K = [(32, 32, 32, 1), (32, 20, 1, 3), (32, 26, 17, 8), (21, 15, 11, 4), (16, 16, 16, 8), (16, 9, 16, 2),
           (9, 6, 5, 2), (5, 3, 2, 2), (1, 1, 1, 1), (17, 1, 1, 6)]


@pytest.mark.parametrize("k,s,m,H", OTHER_K)
def test_other_k_match_oracle(k, s, m, H):
    rng = np.random.default_rng(1000 * k + 100 * s + 10 * m + H)
    ins, q = mixed(rng, 700)
    print("case param k=%d s=%d m=%d H=%d" % (k, s, m, H), flush=True)
    run_both((k, s, m, H, 1 << 16), 4, ins, q)


@pytest.mark.parametrize("S", [8, 16])
@pytest.mark.parametrize("s,m,H", [(24, 12, 1), (27, 15, 3), (29, 17, 5), (25, 20, 8)])
def test_wide_shards_match_oracle(S, s, m, H):
    rng = np.random.default_rng(100 * S + 10 * s + H)
    ins, q = mixed(rng)
    print("case param S=%d s=%d m=%d H=%d" % (S, s, m, H), flush=True)
    for mode in (0, 1):
        run_both((31, s, m, H, 1 << 18), S, ins, q, mode=mode)


@pytest.mark.parametrize("tile", [8, 16])
@pytest.mark.parametrize("n", [31, 32, 2048 + 30, 2048 + 31, 4096 + 30, 4096 + 31, 3 * 4096 + 45])
def test_lengths_around_tiles(tile, n):
    seq = synth.uniform_acgt(n, n).copy()
    off = np.array([0, n], dtype=np.uint64)
    print("case param length", tile, n, flush=True)
    _, want = run_both((31, 25, 14, 3, 1 << 16), 4, (seq, off), (seq, off), tile=tile)
    # the filter's own sequence: every k-mer is present
    assert want[: n - 30].all() and not want[n - 30:].any()


@pytest.mark.parametrize("S", [4, 16])
@pytest.mark.parametrize("alphabet", [b"AC", b"ACGT"])
def test_contention(S, alphabet):
    """Few shards (2^10 bits) receive every run of every workgroup: the
    store pass's read-modify-writes race constantly and the repair walk must
    restore every dropped bit."""
    rng = np.random.default_rng(S + len(alphabet))
    seq = np.frombuffer(alphabet, dtype=np.uint8)[rng.integers(0, len(alphabet), 300_000)].copy()
    off = np.array([0, seq.size], dtype=np.uint64)
    print("case param contention", S, alphabet, flush=True)
    run_both((31, 26, 13, 5, 1 << 10), S, (seq, off), (seq[:40_000], np.array([0, 40_000], dtype=np.uint64)))


@pytest.mark.parametrize("S", [4, 8])
@pytest.mark.parametrize("wgs", [0, 1, 4])
def test_persistent_launches(S, wgs):
    """Persistent grids smaller than the tile count give the oracle's
    results (the 2 Mbp genome is about 1000 tiles of 2048 k-mers)."""
    w = synth.in_cache_workload(scale=0.02)
    print("case param persistent", S, wgs, flush=True)
    run_both((w["k"], 26, 18, 6, w["bits"] // 4), S, w["insert"], w["query"], launch=(wgs, wgs))


def test_family_selection_and_tiles():
    from paper_2606_24417_amd import VARIANT_GENERIC, VARIANT_PARAM, VARIANT_ROLLING, Filter, SBFError

    f = Filter(31, 25, 14, 3, 1 << 20)
    assert f.variant == VARIANT_PARAM  # no compiled kernel for this set
    assert f.get_tile() == (8, 8)
    f.set_tile(16, 8)
    assert f.get_tile() == (16, 8)
    with pytest.raises(SBFError):
        f.set_tile(32, 8)
    f.variant = VARIANT_ROLLING  # the super-k-mer kernels of this set
    assert f.variant == VARIANT_PARAM
    f.variant = VARIANT_GENERIC
    assert f.variant == VARIANT_GENERIC
    f.close()
    # compiled sets keep their lane kernels unless asked
    f = Filter(31, 28, 16, 4, 1 << 20)
    assert f.variant == VARIANT_ROLLING
    f.variant = VARIANT_PARAM
    assert f.variant == VARIANT_PARAM and f.get_tile() == (8, 8)
    f.close()
    # H > 8: no run-time parameter kernel
    f = Filter(31, 28, 16, 9, 1 << 20)
    assert f.variant == VARIANT_GENERIC
    with pytest.raises(SBFError):
        f.variant = VARIANT_PARAM
    f.close()


def test_autotuner_covers_tile_lengths():
    from paper_2606_24417_amd import VARIANT_PARAM, Filter

    w = synth.in_cache_workload(scale=0.01)
    params = (w["k"], 27, 15, 5, w["bits"])
    p = oracle.Params(*params)
    F = oracle.insert(p, p.empty(), *w["insert"])
    f = Filter(*params)
    assert f.variant == VARIANT_PARAM
    f.insert(dev(w["insert"][0]), doff(w["insert"][1]))
    report = f.autotune(dev(w["insert"][0]), doff(w["insert"][1]), dev(w["query"][0]), doff(w["query"][1]))
    print(report, flush=True)
    assert " 8 k-mers/lane" in report and "16 k-mers/lane" in report and "param" in report
    # the tuned filter still holds exactly the inserted k-mers
    assert_same(f.get_bits(), F, "filter words after autotuning")
    f.close()


@pytest.mark.parametrize("S", [4, 16])
def test_unaligned_input_and_output_and_host_path(S):
    """Sequence and answer buffers at odd device addresses (byte loads and
    byte stores instead of 16- and 8-byte ones), a single sequence (no
    record starts), and the host entry points (pinned staging, chunked)."""
    rng = np.random.default_rng(500 + S)
    params = (31, 25, 15, 6, 1 << 17)
    ins, q = mixed(rng, 900)
    p = oracle.Params(*params, shard_words=S)
    F = oracle.insert(p, p.empty(), *ins)
    want = oracle.query(p, F, *q)
    f = param_filter(*params, S)
    # insert from an odd address
    buf = torch.zeros(ins[0].size + 3, dtype=torch.uint8, device="cuda")
    buf[3:] = dev(ins[0])
    f.insert(buf[3:], doff(ins[1]))
    torch.cuda.synchronize()
    assert_same(f.get_bits(), F, "filter words (unaligned sequence)")
    # answers into an odd address
    qs = torch.zeros(q[0].size + 5, dtype=torch.uint8, device="cuda")
    qs[5:] = dev(q[0])
    out = torch.full((q[0].size + 1,), 9, dtype=torch.uint8, device="cuda")
    print("case param unaligned", S, flush=True)
    f.query(qs[5:], doff(q[1]), out=out[1:])
    torch.cuda.synchronize()
    assert_same(out[1:].cpu().numpy(), want, "answers (unaligned output)")
    assert int(out[0].item()) == 9
    # a single sequence: len - k + 1 answers
    one = q[0][: int(q[1][1])]
    if one.size >= params[0]:
        got1 = f.query(dev(one)).cpu().numpy()
        assert_same(got1, oracle.query(p, F, one)[: one.size - params[0] + 1], "single-sequence answers")
    # host entry points, staging in small chunks
    f.set_staging_bytes(1 << 16)
    got_h = f.query(q[0], q[1])
    assert_same(np.asarray(got_h), want, "answers (host path)")
    f.close()
