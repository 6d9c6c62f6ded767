"""Served form: continuous batching over a resident filter.

Each request's answers must be identical whether it runs alone (one slot, one
request at a time) or mixed with many others admitted into shared batches on
several streams, and equal to the oracle.
"""

import threading
import time

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


def make_requests(genome, goff, n, seed, max_reads=300):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n):
        nreads = int(np.exp(rng.uniform(0, np.log(max_reads))))
        lens = synth.lognormal_lengths(nreads, seed * 1000 + i, median=400, lo=20, hi=3000)
        if i % 2 == 0:
            seq, off = synth.sample_reads(genome, goff, nreads, lens, seed * 1000 + i)
        else:
            seq, off = synth.random_reads(nreads, lens, seed * 1000 + i)
        pinned = torch.from_numpy(seq).pin_memory()
        out = torch.zeros(seq.size, dtype=torch.uint8).pin_memory()
        reqs.append((seq, off, pinned, out))
    return reqs


@pytest.fixture(scope="module")
def served():
    from paper_2606_24417_amd import Filter

    w = synth.in_cache_workload(scale=0.02)
    params = (w["k"], w["s"], w["m"], w["H"], w["bits"])
    f = Filter(*params)
    ins, ioff = w["insert"]
    f.insert(torch.from_numpy(ins).cuda(), torch.from_numpy(ioff.view(np.int64)).cuda())
    torch.cuda.synchronize()
    bits = f.get_bits()
    p = oracle.Params(*params)
    yield f, p, bits, ins, ioff
    f.close()


def test_server_alone_and_in_mix_match_oracle(served):
    from paper_2606_24417_amd import Server

    f, p, bits, ins, ioff = served
    reqs = make_requests(ins, ioff, 60, 7)
    # alone: one slot, one request in flight at a time
    sv = Server(f, slots=1, slot_bases=1 << 21, slot_records=1 << 12)
    alone = []
    for seq, off, pin, out in reqs:
        out.zero_()
        t = sv.submit(pin, off, out)
        sv.wait(t)
        alone.append(out.numpy().copy())
    assert sv.stats()["max_batch_requests"] == 1
    sv.close()
    # in the mix: four slots, requests submitted from two threads with jitter;
    # a 2 ms batching window makes requests that arrive close together share
    # a batch while earlier batches are still on the device
    sv = Server(f, slots=4, slot_bases=1 << 21, slot_records=1 << 12)
    sv.set_batch_window(2000)
    for _, _, _, out in reqs:
        out.fill_(7)
    tickets = [None] * len(reqs)

    def submit(idx):
        rng = np.random.default_rng(idx[0])
        for i in idx:
            tickets[i] = sv.submit(reqs[i][2], reqs[i][1], reqs[i][3])
            time.sleep(float(rng.uniform(0, 2e-4)))

    th = [threading.Thread(target=submit, args=(list(range(j, len(reqs), 2)),)) for j in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for t in tickets:
        sv.wait(t)
    st = sv.stats()
    print("server stats", st, flush=True)
    assert st["requests"] == len(reqs) and st["max_batch_requests"] > 1
    sv.close()
    for i, (seq, off, pin, out) in enumerate(reqs):
        mixed = out.numpy()
        assert np.array_equal(mixed, alone[i]), "request %d differs alone vs in the mix" % i
        assert np.array_equal(mixed, oracle.query(p, bits, seq, off)), "request %d differs from the oracle" % i


def test_server_admission_and_busy(served):
    from paper_2606_24417_amd import SBF_E_BUSY, SBF_E_INVAL, SBFError, Server

    f, p, bits, ins, ioff = served
    sv = Server(f, slots=1, slot_bases=4096, slot_records=8, max_pending=2)
    big = torch.zeros(5000, dtype=torch.uint8).pin_memory()
    with pytest.raises(SBFError) as e:
        sv.submit(big, [0, 5000], torch.zeros(5000, dtype=torch.uint8))
    assert e.value.code == SBF_E_INVAL
    with pytest.raises(SBFError) as e:
        sv.submit(big[:100], list(range(0, 100, 10)), torch.zeros(100, dtype=torch.uint8))  # 9 records > 8
    assert e.value.code == SBF_E_INVAL
    # flood: more pending requests than allowed gives SBF_E_BUSY, never a hang
    seq = torch.from_numpy(synth.uniform_acgt(4000, 3)).pin_memory()
    outs, tickets, busy = [], [], 0
    for _ in range(200):
        o = torch.zeros(4000, dtype=torch.uint8).pin_memory()
        try:
            tickets.append(sv.submit(seq, [0, 4000], o))
            outs.append(o)
        except SBFError as err:
            assert err.code == SBF_E_BUSY
            busy += 1
    for t in tickets:
        sv.wait(t)
    sv.close()
    assert busy > 0
    want = oracle.query(p, bits, seq.numpy(), [0, 4000])
    for o in outs:
        assert np.array_equal(o.numpy(), want)


@pytest.mark.parametrize("window_us", [0, 3000])
def test_server_mixed_buffer_kinds(served, window_us):
    """Requests whose buffers the server's copy kernels move (16-byte aligned
    pinned memory) share batches with requests it copies through the runtime
    (pageable arrays, pinned views at odd offsets); every answer equals the
    oracle's, and bytes around each output view stay untouched."""
    from paper_2606_24417_amd import Server

    f, p, bits, ins, ioff = served
    reqs = make_requests(ins, ioff, 40, 11, max_reads=200)
    sv = Server(f, slots=3, slot_bases=1 << 21, slot_records=1 << 12)
    if window_us:
        sv.set_batch_window(window_us)
    jobs = []
    for i, (seq, off, pin, out) in enumerate(reqs):
        kind = i % 4
        n = seq.size
        if kind == 0:  # aligned pinned in and out
            s_buf, o_buf, o_view = pin, out, out
        elif kind == 1:  # pageable in and out
            s_buf = np.ascontiguousarray(seq)
            o_buf = np.full(n, 7, dtype=np.uint8)
            o_view = o_buf
        elif kind == 2:  # pinned views at odd offsets
            s_big = torch.zeros(n + 8, dtype=torch.uint8).pin_memory()
            s_big[3:3 + n] = torch.from_numpy(seq)
            o_big = torch.full((n + 8,), 9, dtype=torch.uint8).pin_memory()
            s_buf, o_buf, o_view = s_big[3:3 + n], o_big, o_big[5:5 + n]
        else:  # aligned pinned in, pageable out
            s_buf = pin
            o_buf = np.full(n, 7, dtype=np.uint8)
            o_view = o_buf
        jobs.append((i, kind, o_buf, o_view, sv.submit(s_buf, off, o_view), s_buf))
    for i, kind, o_buf, o_view, t, _ in jobs:
        sv.wait(t)
    st = sv.stats()
    sv.close()
    assert st["requests"] == len(reqs)
    for i, kind, o_buf, o_view, t, _ in jobs:
        seq, off = reqs[i][0], reqs[i][1]
        got = o_view.numpy() if hasattr(o_view, "numpy") else o_view
        assert np.array_equal(got, oracle.query(p, bits, seq, off)), "request %d (kind %d)" % (i, kind)
        if kind == 2:
            whole = o_buf.numpy()
            assert (whole[:5] == 9).all() and (whole[5 + seq.size:] == 9).all(), "bytes outside request %d" % i
