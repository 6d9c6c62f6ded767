"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Every test builds the same seeded inputs for both sides, runs the library
through its C ABI (ctypes binding), and compares the whole filter bit array
and every query answer with the oracle.  Sizes span several workgroup tiles
(8192 k-mers per insert tile, 4096 per query tile, 1024 per generic tile)
with ragged tails.
"""

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
    import paper_2606_24417_amd

    paper_2606_24417_amd.lib()
    print("GPU:", torch.cuda.get_device_name(0), flush=True)


def Filter(*a, **kw):
    from paper_2606_24417_amd import Filter as F

    return F(*a, **kw)


VARIANTS = {"rolling": 1, "generic": 2}


def dev(x):
    return torch.from_numpy(np.array(x, copy=True)).cuda()


def gpu_run(params, inserts, query, variant="auto", path="dev", staging=None):
    """inserts: list of (seq, off|None); query: (seq, off|None).  Returns the
    filter words and the answers."""
    k, s, m, H, bits = params
    f = Filter(k, s, m, H, bits)
    if variant != "auto":
        f.variant = VARIANTS[variant]
    if staging:
        f.set_staging_bytes(staging)
    for seq, off in inserts:
        if path == "dev":
            f.insert(dev(seq), None if off is None else dev(off.astype(np.uint64).view(np.int64)))
        else:
            f.insert(seq, off)
    ans = None
    if query is not None:
        qs, qo = query
        if path == "dev":
            ans = f.query(dev(qs), None if qo is None else dev(qo.astype(np.uint64).view(np.int64)))
            torch.cuda.synchronize()
            ans = ans.cpu().numpy()
        else:
            ans = f.query(qs, qo)
    torch.cuda.synchronize()
    bits = f.get_bits()
    f.close()
    return bits, ans


def oracle_run(params, inserts, query):
    k, s, m, H, bits = params
    p = oracle.Params(k, s, m, H, bits)
    F = p.empty()
    for seq, off in inserts:
        oracle.insert(p, F, seq, off)
    ans = None
    if query is not None:
        ans = oracle.query(p, F, query[0], query[1])
    return F, ans


def assert_same(got, want, what):
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError("%s differ at %d of %d positions, first %s: got %s want %s" % (
            what, bad.size, got.size, bad[:5].tolist(), got[bad[:5]].tolist(), want[bad[:5]].tolist()))


def check(params, inserts, query, **kw):
    gb, ga = gpu_run(params, inserts, query, **kw)
    ob, oa = oracle_run(params, inserts, query)
    assert_same(gb, ob, "filter words")
    if query is not None:
        assert ga.shape == oa.shape
        assert_same(ga, oa, "answers")
    return ob, oa


def noisy(rng, n, p_invalid=0.0, lower=0.0):
    seq = synth.uniform_acgt(n, int(rng.integers(1 << 30))).copy()
    if p_invalid:
        bad = rng.random(n) < p_invalid
        seq[bad] = rng.choice(np.frombuffer(b"NnX-\x00\xff.RY", dtype=np.uint8), bad.sum())
    if lower:
        lw = rng.random(n) < lower
        seq[lw] |= 0x20
    return seq


HOT = (31, 28, 16, 4)


@pytest.mark.parametrize("variant", ["rolling", "generic"])
@pytest.mark.parametrize("path", ["dev", "host"])
def test_tiny_workload(variant, path):
    """1 Mbp into 2^24 bits; query a 500 kbp substring plus 500 kbp fresh."""
    w = synth.tiny_workload()
    print("case tiny", variant, path, flush=True)
    params = (w["k"], w["s"], w["m"], w["H"], w["bits"])
    _, ans = check(params, [w["insert"]], w["query"], variant=variant, path=path)
    n_pos = 500_000 - 30
    assert ans[:n_pos].sum() == n_pos  # no false negatives


# Lengths at k-mer counts around one lane of the lane query (48 k-mers), the
# two-phase query tile (4096), the insert tile (8192) and one and two lane
# query tiles (12288, 24576): n = k-mers + 30.
@pytest.mark.parametrize("n", [0, 1, 30, 31, 32, 33, 64, 77, 78, 79, 4126, 4127, 4128, 8222, 8223, 8224, 12345,
                               12317, 12318, 12319, 24605, 24606, 24607, 50_000])
def test_lengths_around_tiles(n):
    rng = np.random.default_rng(n)
    seq = noisy(rng, n, 0.002, 0.1)
    print("case length", n, flush=True)
    for variant in ("rolling", "generic"):
        check(HOT + (1 << 14,), [(seq, None)], (seq, None), variant=variant)


# Base offsets, relative to the first base of a lane, where an invalid base
# or a record start decides k-mer validity across the seam between a lane's
# two 64-base validity windows (k-mers 0..31 judged on bases 0..63, k-mers
# 32..47 on bases 32..95: an invalid base at 61 ends k-mer 31, at 62 only
# k-mers from 32 on) and where lanes of 32 or 48 k-mers end.
SEAM_OFFSETS = [1, 30, 31, 32, 33, 47, 48, 61, 62, 63, 64, 77, 78]


@pytest.mark.parametrize("lane", [32, 48])
def test_validity_at_lane_window_seams(lane):
    """One invalid base in every fourth lane and one record start in every
    fourth lane (another phase), each at a seam offset, cycling through them."""
    rng = np.random.default_rng(700 + lane)
    n = 200_000
    seq = noisy(rng, n, 0.0, 0.05)
    nl = n // lane - 2
    for j, li in enumerate(range(0, nl, 4)):
        seq[li * lane + SEAM_OFFSETS[j % len(SEAM_OFFSETS)]] = ord("N")
    starts = sorted({li * lane + SEAM_OFFSETS[j % len(SEAM_OFFSETS)] for j, li in enumerate(range(2, nl, 4))})
    off = np.array([0] + starts + [n], dtype=np.uint64)
    print("case seams", lane, flush=True)
    _, ans = check(HOT + (1 << 24,), [(seq, off)], (seq, off))
    assert ans.sum() > n // 2  # most k-mers stay valid, so the seams decide


@pytest.mark.parametrize("bits", [1, 256, 257, 4096, 1 << 20, 1 << 30])
@pytest.mark.parametrize("p_invalid", [0.0, 0.01, 0.2])
def test_filter_sizes_and_invalid_bases(bits, p_invalid):
    rng = np.random.default_rng(bits % 1000 + int(p_invalid * 100))
    ins = noisy(rng, 30_000, p_invalid, 0.05)
    q = np.concatenate([ins[5000:15000], noisy(rng, 20_000, p_invalid)])
    print("case bits", bits, p_invalid, flush=True)
    check(HOT + (bits,), [(ins, None)], (q, None))


@pytest.mark.parametrize("k,s,m,H", [(31, 28, 16, 1), (31, 28, 16, 8), (31, 24, 12, 4), (31, 31, 16, 4),
                                     (32, 32, 32, 1), (32, 20, 10, 3), (21, 19, 11, 16), (21, 17, 9, 11),
                                     (9, 6, 5, 2), (1, 1, 1, 1), (16, 16, 8, 5), (31, 28, 20, 4)])
def test_generic_parameters(k, s, m, H):
    rng = np.random.default_rng(k * 100 + s * 10 + H)
    ins = noisy(rng, 20_000, 0.003)
    q = np.concatenate([ins[:7000], noisy(rng, 7000, 0.003)])
    print("case params", k, s, m, H, flush=True)
    check((k, s, m, H, 1 << 16), [(ins, None)], (q, None), variant="generic")


def random_batch(rng, nrec, maxlen, p_invalid=0.0):
    lens = rng.integers(0, maxlen + 1, nrec)
    lens[rng.random(nrec) < 0.1] = 0
    off = np.zeros(nrec + 1, dtype=np.uint64)
    off[1:] = np.cumsum(lens)
    return noisy(rng, int(off[-1]), p_invalid), off


ROLLING_SETS = [(31, 27, 16, 4), (31, 30, 16, 4), (31, 31, 16, 4), (31, 28, 18, 4), (31, 28, 16, 8)]


@pytest.mark.parametrize("k,s,m,H", ROLLING_SETS)
def test_rolling_parameter_sets(k, s, m, H):
    """The other compiled rolling parameter sets: every insert strategy and
    query kernel against the oracle on a record batch spanning several tiles
    with invalid bases and a ragged tail."""
    rng = np.random.default_rng(k * 1000 + s * 100 + m * 10 + H)
    ins = random_batch(rng, 60, 4000, 0.002)
    q = random_batch(rng, 80, 3000, 0.002)
    qs = np.concatenate([ins[0][: int(ins[1][20])], q[0]])
    qo = np.concatenate([ins[1][:21], q[1][1:] + ins[1][20]])
    params = (k, s, m, H, 1 << 15)
    F, oa = oracle_run(params, [ins], (qs, qo))
    print("case rolling set", k, s, m, H, flush=True)
    for imode in (0, 1):
        f = Filter(*params)
        f.variant = VARIANTS["rolling"]
        f.set_insert_mode(imode)
        f.insert(dev(ins[0]), dev(ins[1].astype(np.uint64).view(np.int64)))
        torch.cuda.synchronize()
        assert_same(f.get_bits(), F, "filter words (insert mode %d)" % imode)
        for qmode in (0, 1, 2):
            f.set_query_mode(qmode)
            ans = f.query(dev(qs), dev(qo.astype(np.uint64).view(np.int64)))
            torch.cuda.synchronize()
            assert_same(ans.cpu().numpy(), oa, "answers (query mode %d)" % qmode)
        f.close()


@pytest.mark.parametrize("S,H", [(8, 1), (8, 4), (8, 8), (8, 9), (16, 4), (16, 8)])
def test_shard_geometry(S, H):
    """Shards of 8 and 16 words (the geometry extension) against the oracle at
    the same geometry, on a record batch with invalid bases: the generic
    kernels for every H, and the super-k-mer kernels where they exist: the
    wide-shard kernels where they are compiled (H = 4, 8), the run-time
    parameter kernels for the other H up to 8."""
    from paper_2606_24417_amd import VARIANT_GENERIC, VARIANT_PARAM, VARIANT_ROLLING, VARIANT_WIDE, SBFError

    rng = np.random.default_rng(S * 100 + H)
    ins = random_batch(rng, 80, 3000, 0.002)
    q = random_batch(rng, 60, 2000, 0.002)
    qs = np.concatenate([ins[0][: int(ins[1][30])], q[0]])
    qo = np.concatenate([ins[1][:31], q[1][1:] + ins[1][30]])
    bits = 1 << 17
    p = oracle.Params(31, 28, 16, H, bits, shard_words=S)
    F = oracle.insert(p, p.empty(), ins[0], ins[1])
    want = oracle.query(p, F, qs, qo)
    tiled = VARIANT_WIDE if H in (4, 8) else VARIANT_PARAM if H <= 8 else None
    for variant in ([VARIANT_GENERIC, VARIANT_ROLLING] if tiled else [VARIANT_GENERIC]):
        print("case geometry", S, H, variant, flush=True)
        f = Filter(31, 28, 16, H, bits, shard_words=S)
        assert f.num_bits == p.nshards * S * 64
        if not tiled:
            with pytest.raises(SBFError):
                f.variant = VARIANT_ROLLING  # no super-k-mer kernel for this H
        f.variant = variant
        assert f.variant == (tiled if variant == VARIANT_ROLLING else VARIANT_GENERIC)
        f.insert(dev(ins[0]), dev(ins[1].astype(np.uint64).view(np.int64)))
        ans = f.query(dev(qs), dev(qo.astype(np.uint64).view(np.int64)))
        torch.cuda.synchronize()
        assert_same(f.get_bits(), F, "filter words")
        assert_same(ans.cpu().numpy(), want, "answers")
        f.close()


@pytest.mark.parametrize("variant", ["rolling", "generic"])
@pytest.mark.parametrize("path", ["dev", "host"])
def test_record_batches(variant, path):
    rng = np.random.default_rng(5)
    ins = random_batch(rng, 700, 400, 0.002)
    q = random_batch(rng, 600, 300)
    # some query records are copies of inserted records
    qs = np.concatenate([ins[0][: int(ins[1][50])], q[0]])
    qo = np.concatenate([ins[1][:51], q[1][1:] + ins[1][50]])
    print("case batch", variant, path, flush=True)
    check(HOT + (1 << 16,), [ins], (qs, qo), variant=variant, path=path)


def test_host_chunking_with_small_staging():
    rng = np.random.default_rng(6)
    ins = random_batch(rng, 300, 2000, 0.001)
    single = noisy(rng, 50_000, 0.001)
    q = random_batch(rng, 200, 1000)
    print("case chunking", flush=True)
    check(HOT + (1 << 16,), [ins, (single, None)], q, path="host", staging=4096)
    check(HOT + (1 << 16,), [(single, None)], (single, None), path="host", staging=5000)


@pytest.mark.parametrize("pin_in,pin_out", [(True, True), (True, False), (False, True)])
def test_host_pipeline_with_pinned_buffers(pin_in, pin_out):
    """Host entry points over many small chunks, with the caller's buffers in
    pinned memory (sent directly) or pageable memory (staged), both ways."""
    rng = np.random.default_rng(16)
    ins = random_batch(rng, 400, 1500, 0.001)
    single = noisy(rng, 60_000, 0.001)
    q = random_batch(rng, 300, 900)
    params = HOT + (1 << 16,)

    def host(x):
        t = torch.from_numpy(np.array(x, copy=True))
        return t.pin_memory() if pin_in else t

    def out_buf(n):
        t = torch.full((n,), 7, dtype=torch.uint8)
        return t.pin_memory() if pin_out else t

    print("case host pipeline", pin_in, pin_out, flush=True)
    f = Filter(*params)
    f.set_staging_bytes(6000)
    f.insert(host(ins[0]), ins[1])
    f.insert(host(single))
    qa = f.query(host(q[0]), q[1], out=out_buf(q[0].size))
    sa = f.query(host(single), out=out_buf(single.size - 30))
    bits = f.get_bits()
    f.close()
    F, oa = oracle_run(params, [ins, (single, None)], q)
    assert_same(bits, F, "filter words")
    assert_same(qa.numpy(), oa, "batch answers")
    assert_same(sa.numpy(), oracle.query(oracle.Params(*params), F, single), "single-sequence answers")


def test_unaligned_device_pointers():
    rng = np.random.default_rng(7)
    base = noisy(rng, 40_000, 0.001)
    p = oracle.Params(*HOT, 1 << 16)
    for shift in (1, 3, 8, 15):
        t = dev(base)
        f = Filter(*HOT, 1 << 16)
        f.insert(t[shift:])
        ans = f.query(t[shift + 5:])
        torch.cuda.synchronize()
        F = oracle.insert(p, p.empty(), base[shift:])
        assert_same(f.get_bits(), F, "filter words (shift %d)" % shift)
        assert_same(ans.cpu().numpy(), oracle.query(p, F, base[shift + 5:]), "answers (shift %d)" % shift)
        f.close()


@pytest.mark.parametrize("qmode", [0, 1, 2])
def test_unaligned_output_pointers(qmode):
    """Answers written through output views at every offset mod 16."""
    rng = np.random.default_rng(17)
    ins = noisy(rng, 30_000, 0.001)
    q = random_batch(rng, 120, 400)
    params = HOT + (1 << 16,)
    F, oa = oracle_run(params, [(ins, None)], q)
    f = Filter(*params)
    f.set_query_mode(qmode)
    f.insert(dev(ins))
    d_q = dev(q[0])
    d_off = dev(q[1].astype(np.uint64).view(np.int64))
    print("case unaligned out", qmode, flush=True)
    for shift in (1, 5, 8, 13):
        buf = torch.full((q[0].size + 32,), 9, dtype=torch.uint8, device="cuda")
        f.query(d_q, d_off, out=buf[shift:shift + q[0].size])
        torch.cuda.synchronize()
        got = buf.cpu().numpy()
        assert_same(got[shift:shift + q[0].size], oa, "answers (shift %d)" % shift)
        assert (got[:shift] == 9).all() and (got[shift + q[0].size:] == 9).all()
    f.close()


def test_nondefault_stream_and_state_roundtrip():
    rng = np.random.default_rng(8)
    a, b = noisy(rng, 30_000), noisy(rng, 30_000)
    p = oracle.Params(*HOT, 1 << 16)
    FA = oracle.insert(p, p.empty(), a)
    FAB = oracle.insert(p, FA.copy(), b)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        f = Filter(*HOT, 1 << 16)
        da, db = dev(a), dev(b)
        f.insert(da)
        f.insert(da)  # idempotent
    s.synchronize()
    assert_same(f.get_bits(), FA, "after repeated insert")
    with torch.cuda.stream(s):
        f.insert(db)
        ans = f.query(db)
    s.synchronize()
    assert_same(f.get_bits(), FAB, "after second insert")
    assert ans.cpu().numpy().all()
    snap = f.get_bits()
    g = Filter(*HOT, 1 << 16)
    g.set_bits(snap)
    assert_same(g.query(a), oracle.query(p, FAB, a), "restored filter answers")
    f.clear()
    torch.cuda.synchronize()
    assert not f.get_bits().any()
    f.close()
    g.close()


@pytest.mark.parametrize("qmode", [0, 1])
def test_concurrent_streams(qmode):
    """One filter, three streams: a record-batch insert on one, then two query
    batches on two others ordered after it by an event and free to overlap
    each other (each stream has its own record-start and work-queue
    scratch).  Every answer against the oracle."""
    rng = np.random.default_rng(31 + qmode)
    ins = random_batch(rng, 200, 3000, 0.002)
    qa = random_batch(rng, 300, 2000, 0.002)
    qb = random_batch(rng, 150, 5000, 0.002)
    params = HOT + (1 << 18,)
    F, oa = oracle_run(params, [ins], qa)
    ob = oracle.query(oracle.Params(*params), F, qb[0], qb[1])
    print("case streams", qmode, flush=True)
    f = Filter(*params)
    f.set_query_mode(qmode)
    s_ins, s_a, s_b = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    d_ins, d_ioff = dev(ins[0]), dev(ins[1].astype(np.uint64).view(np.int64))
    d_qa, d_qao = dev(qa[0]), dev(qa[1].astype(np.uint64).view(np.int64))
    d_qb, d_qbo = dev(qb[0]), dev(qb[1].astype(np.uint64).view(np.int64))
    out_a = torch.full((qa[0].size,), 7, dtype=torch.uint8, device="cuda")
    out_b = torch.full((qb[0].size,), 7, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    done = torch.cuda.Event()
    f.insert(d_ins, d_ioff, stream=s_ins)
    done.record(s_ins)
    s_a.wait_event(done)
    s_b.wait_event(done)
    for _ in range(3):  # repeated, so that the two query streams interleave
        f.query(d_qa, d_qao, out=out_a, stream=s_a)
        f.query(d_qb, d_qbo, out=out_b, stream=s_b)
    torch.cuda.synchronize()
    assert_same(f.get_bits(), F, "filter words")
    assert_same(out_a.cpu().numpy(), oa, "answers on stream a")
    assert_same(out_b.cpu().numpy(), ob, "answers on stream b")
    f.close()


@pytest.mark.parametrize("H", [1, 2, 4, 8])
def test_all_A_closed_form(H):
    f = Filter(31, 28, 16, H, 1 << 20)
    f.insert(dev(np.full(100_000, ord("A"), dtype=np.uint8)))
    ans = f.query(dev(np.frombuffer(b"A" * 40 + b"C" + b"A" * 40, dtype=np.uint8)))
    torch.cuda.synchronize()
    w = f.get_bits()
    expect = np.zeros_like(w)
    expect[: min(H, 4)] = 1
    assert_same(w, expect, "all-A filter")
    a = ans.cpu().numpy()
    assert a[:10].all() and a.size == 51
    f.close()


@pytest.mark.parametrize("alphabet", [b"A", b"AC", b"ACGT"])
def test_colliding_shards_stress(alphabet):
    """Low-complexity input sends most segments of every workgroup to a few
    shards: concurrent 64-bit atomic ORs on the same words across XCDs."""
    rng = np.random.default_rng(len(alphabet))
    if alphabet == b"ACGT":
        unit = synth.uniform_acgt(37, 1)
        seq = np.tile(unit, 60_000)
    else:
        seq = np.frombuffer(alphabet, dtype=np.uint8)[rng.integers(0, len(alphabet), 2_000_000)]
    print("case collide", alphabet, flush=True)
    check(HOT + (1 << 12,), [(seq, None)], (seq[:100_000], None))


def test_rolling_and_generic_agree_on_a_genome():
    w = synth.in_cache_workload(scale=0.02)  # 2 Mbp genome, 40k reads
    print("case genome 2 Mbp", flush=True)
    params = (w["k"], w["s"], w["m"], w["H"], w["bits"])
    gr = gpu_run(params, [w["insert"]], w["query"], variant="rolling")
    gg = gpu_run(params, [w["insert"]], w["query"], variant="generic")
    ob, oa = oracle_run(params, [w["insert"]], w["query"])
    assert_same(gr[0], ob, "rolling filter")
    assert_same(gg[0], ob, "generic filter")
    assert_same(gr[1], oa, "rolling answers")
    assert_same(gg[1], oa, "generic answers")


def test_marked_batch_entry_points_match_batch_form():
    """Marking record starts once and reusing them gives the batch results."""
    rng = np.random.default_rng(9)
    ins = random_batch(rng, 400, 500, 0.001)
    q = random_batch(rng, 300, 400)
    ob, oa = oracle_run(HOT + (1 << 16,), [ins], q)
    f = Filter(*HOT, 1 << 16)
    d_ins, d_ioff = dev(ins[0]), dev(ins[1].view(np.int64))
    d_q, d_qoff = dev(q[0]), dev(q[1].view(np.int64))
    st_i = f.mark_record_starts(d_ioff, ins[0].size)
    st_q = f.mark_record_starts(d_qoff, q[0].size)
    f.insert_marked(d_ins, st_i)
    f.insert_marked(d_ins, st_i)
    out = f.query_marked(d_q, st_q)
    torch.cuda.synchronize()
    assert_same(f.get_bits(), ob, "filter words")
    assert_same(out.cpu().numpy(), oa, "answers")
    f.close()


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("bits", [1 << 10, 1 << 16, 1 << 24])
def test_insert_modes_match_oracle(mode, bits):
    """Two-pass insert (plain read-modify-write, then atomic repair) and the
    one-atomic-per-word insert give the oracle's filter, also when many
    segments hit few shards (small filters force concurrent updates)."""
    rng = np.random.default_rng(bits + mode)
    ins = noisy(rng, 300_000, 0.001)
    p = oracle.Params(*HOT, bits)
    F = oracle.insert(p, p.empty(), ins)
    f = Filter(*HOT, bits)
    f.set_insert_mode(mode)
    f.insert(dev(ins))
    torch.cuda.synchronize()
    assert_same(f.get_bits(), F, "filter words (mode %d)" % mode)
    f.close()


@pytest.mark.parametrize("qmode", [0, 1, 2])
def test_query_modes_match_oracle(qmode):
    w = synth.in_cache_workload(scale=0.01)
    params = (w["k"], w["s"], w["m"], w["H"], w["bits"])
    ob, oa = oracle_run(params, [w["insert"]], w["query"])
    f = Filter(*params)
    f.set_query_mode(qmode)
    f.insert(dev(w["insert"][0]), dev(w["insert"][1].view(np.int64)))
    out = f.query(dev(w["query"][0]), dev(w["query"][1].view(np.int64)))
    torch.cuda.synchronize()
    assert_same(out.cpu().numpy(), oa, "answers (query mode %d)" % qmode)
    f.close()


@pytest.mark.parametrize("wgs", [0, 1, 4])
def test_persistent_launch_shapes_match_oracle(wgs):
    """Persistent grids taking tiles from the device work queue give the
    same filter and answers as one workgroup per tile.  The batches have
    more tiles than the persistent grids have workgroups (1220 insert and
    2441 query tiles against 256 and 1024), so workgroups take several
    tiles from the queue."""
    w = synth.in_cache_workload(scale=0.1)
    params = (w["k"], w["s"], w["m"], w["H"], w["bits"])
    ob, oa = oracle_run(params, [w["insert"]], w["query"])
    for qmode in (0, 1, 2):
        f = Filter(*params)
        f.set_launch(wgs, wgs)
        f.set_query_mode(qmode)
        f.insert(dev(w["insert"][0]), dev(w["insert"][1].view(np.int64)))
        out = f.query(dev(w["query"][0]), dev(w["query"][1].view(np.int64)))
        torch.cuda.synchronize()
        assert_same(f.get_bits(), ob, "filter words (wgs %d)" % wgs)
        assert_same(out.cpu().numpy(), oa, "answers (wgs %d, query mode %d)" % (wgs, qmode))
        f.close()


def test_graph_replays_match_eager_and_oracle():
    """A captured graph (clear, mark, insert, query) replayed several times,
    with eager work and synchronisation between replays, gives the oracle's
    filter and answers every time."""
    from paper_2606_24417_amd import Graph

    w = synth.in_cache_workload(scale=0.01)
    params = (w["k"], w["s"], w["m"], w["H"], w["bits"])
    ob, oa = oracle_run(params, [w["insert"]], w["query"])
    f = Filter(*params)
    f.set_launch(2, 2)
    ins, ioff = dev(w["insert"][0]), dev(w["insert"][1].view(np.int64))
    q, qoff = dev(w["query"][0]), dev(w["query"][1].view(np.int64))
    out = torch.zeros(q.numel(), dtype=torch.uint8, device=q.device)
    g = Graph(f, ins, ioff, q, qoff, out, clear_first=True)
    for rep in range(3):
        out.zero_()
        f.insert(dev(synth.uniform_acgt(5000, rep)))  # eager work that the graph's clear undoes
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        assert_same(f.get_bits(), ob, "filter words after replay %d" % rep)
        assert_same(out.cpu().numpy(), oa, "answers after replay %d" % rep)
    g.close()
    f.close()


def test_autotune_picks_settings_and_keeps_results():
    w = synth.in_cache_workload(scale=0.01)
    params = (w["k"], w["s"], w["m"], w["H"], w["bits"])
    ob, oa = oracle_run(params, [w["insert"]], w["query"])
    f = Filter(*params)
    ins, ioff = dev(w["insert"][0]), dev(w["insert"][1].view(np.int64))
    q, qoff = dev(w["query"][0]), dev(w["query"][1].view(np.int64))
    report = f.autotune(ins, ioff, q, qoff)
    print(report)
    assert "best insert" in report and "best query" in report
    assert not f.get_bits().any()  # tuning inserts into a scratch filter
    f.insert(ins, ioff)
    out = f.query(q, qoff)
    torch.cuda.synchronize()
    assert_same(f.get_bits(), ob, "filter words after autotune")
    assert_same(out.cpu().numpy(), oa, "answers after autotune")
    f.close()
