"""ctypes binding of ``libsbf.so`` (declared in include/sbf.h).

Argument marshalling only: every step of insert and query runs in the HIP
kernels of the library.  PyTorch is used for device buffers and streams; CPU
inputs go through the library's host entry points, CUDA tensors through its
stream-ordered device entry points on the current torch stream.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsbf.so")

SBF_OK = 0
SBF_E_INVAL = -1
SBF_E_NOMEM = -2
SBF_E_DEVICE = -3
SBF_E_BUSY = -4
VARIANT_AUTO = 0
VARIANT_ROLLING = 1
VARIANT_GENERIC = 2
VARIANT_WIDE = 3
VARIANT_PARAM = 4
INSERT_TWO_PASS = 0
INSERT_ATOMIC = 1
QUERY_LANE = 0
QUERY_LEADER = 1
QUERY_DIRECT = 2

# every function declared in include/sbf.h, with its ctypes signature
_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_int = ctypes.c_int
SIGNATURES = {
    "sbf_create": (_vp, [_u32, _u32, _u32, _u32, _u64]),
    "sbf_create_ex": (_vp, [_u32, _u32, _u32, _u32, _u64, _u32]),
    "sbf_destroy": (None, [_vp]),
    "sbf_insert_seq": (_int, [_vp, _vp, _u64]),
    "sbf_query_seq": (_int, [_vp, _vp, _u64, _vp]),
    "sbf_last_error": (_int, [ctypes.POINTER(ctypes.c_char_p)]),
    "sbf_num_shards": (_u64, [_vp]),
    "sbf_num_bits": (_u64, [_vp]),
    "sbf_num_words": (_u64, [_vp]),
    "sbf_get_bits": (_int, [_vp, _vp, _u64]),
    "sbf_set_bits": (_int, [_vp, _vp, _u64]),
    "sbf_clear": (_int, [_vp, _vp]),
    "sbf_device_words": (_vp, [_vp]),
    "sbf_estimate_fpr": (_int, [_vp, _vp, _vp]),
    "sbf_insert_seq_dev": (_int, [_vp, _vp, _u64, _vp]),
    "sbf_query_seq_dev": (_int, [_vp, _vp, _u64, _vp, _vp]),
    "sbf_insert_batch": (_int, [_vp, _vp, _vp, _u64]),
    "sbf_query_batch": (_int, [_vp, _vp, _vp, _u64, _vp]),
    "sbf_insert_batch_dev": (_int, [_vp, _vp, _u64, _vp, _u64, _vp]),
    "sbf_query_batch_dev": (_int, [_vp, _vp, _u64, _vp, _u64, _vp, _vp]),
    "sbf_query_batch_dev_noalloc": (_int, [_vp, _vp, _u64, _vp, _u64, _vp, _vp]),
    "sbf_mark_record_starts_dev": (_int, [_vp, _u64, _u64, _vp, _vp]),
    "sbf_insert_marked_dev": (_int, [_vp, _vp, _u64, _vp, _vp]),
    "sbf_query_marked_dev": (_int, [_vp, _vp, _u64, _vp, _vp, _vp]),
    "sbf_set_variant": (_int, [_vp, _int]),
    "sbf_get_variant": (_int, [_vp]),
    "sbf_set_insert_mode": (_int, [_vp, _int]),
    "sbf_set_query_mode": (_int, [_vp, _int]),
    "sbf_set_staging_bytes": (_int, [_vp, _u64]),
    "sbf_set_launch": (_int, [_vp, _u32, _u32]),
    "sbf_get_launch": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "sbf_graph_create": (_vp, [_vp, _int, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _u64, _vp]),
    "sbf_graph_launch": (_int, [_vp, _vp]),
    "sbf_graph_destroy": (None, [_vp]),
    "sbf_autotune": (_int, [_vp, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _u64]),
    "sbf_autotune_geometry": (_int, [_u32, _u32, _u32, _u32, _u64, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _u64, _vp,
                                     _u64, _vp, _u64, ctypes.c_double, _vp, _vp, _vp, _vp, _vp, _u64]),
    "sbf_set_tile": (_int, [_vp, _u32, _u32]),
    "sbf_get_tile": (_int, [_vp, _vp, _vp]),
    "sbf_server_create": (_vp, [_vp, _u32, _u64, _u64, _u32]),
    "sbf_server_set_batch_window": (_int, [_vp, _u64]),
    "sbf_server_submit": (_int, [_vp, _vp, _vp, _u64, _vp, _vp]),
    "sbf_server_poll": (_int, [_vp, _u64]),
    "sbf_server_wait": (_int, [_vp, _u64, _vp, _vp]),
    "sbf_server_stats": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "sbf_server_destroy": (None, [_vp]),
}

_lib = None


class SBFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sbf error %d: %s" % (code, msg))
        self.code = code


def lib() -> ctypes.CDLL:
    """Load libsbf.so; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsbf.so is not built (run paper_2606_24417_amd/build.py or "
                              "__graft_entry__.build()); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def last_error():
    msg = ctypes.c_char_p()
    code = lib().sbf_last_error(ctypes.byref(msg))
    return code, (msg.value or b"").decode()


def _check(rc):
    if rc != SBF_OK:
        code, msg = last_error()
        raise SBFError(rc, msg)


def _is_cuda(x) -> bool:
    return hasattr(x, "is_cuda") and x.is_cuda


def _host_u8(seq) -> np.ndarray:
    if isinstance(seq, (bytes, bytearray)):
        return np.frombuffer(bytes(seq), dtype=np.uint8)
    if isinstance(seq, str):
        return np.frombuffer(seq.encode("ascii"), dtype=np.uint8)
    if hasattr(seq, "numpy"):
        seq = seq.numpy()
    return np.ascontiguousarray(seq, dtype=np.uint8)


def _stream_handle(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Filter:
    """A Super Bloom filter on the current GPU (owns its device bit array)."""

    def __init__(self, k=31, s=28, m=16, H=4, bits=1 << 24, shard_words=4):
        self.k, self.s, self.m, self.H = int(k), int(s), int(m), int(H)
        self.shard_words = int(shard_words)
        h = lib().sbf_create_ex(self.k, self.s, self.m, self.H, int(bits), self.shard_words)
        if not h:
            code, msg = last_error()
            raise SBFError(code, msg)
        self._h = ctypes.c_void_p(h)

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().sbf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- geometry and state ------------------------------------------------------
    @property
    def handle(self):
        return self._h

    @property
    def num_shards(self) -> int:
        return lib().sbf_num_shards(self._h)

    @property
    def num_bits(self) -> int:
        return lib().sbf_num_bits(self._h)

    @property
    def num_words(self) -> int:
        return lib().sbf_num_words(self._h)

    @property
    def device_words_ptr(self) -> int:
        return lib().sbf_device_words(self._h)

    @property
    def variant(self) -> int:
        return lib().sbf_get_variant(self._h)

    @variant.setter
    def variant(self, v: int):
        _check(lib().sbf_set_variant(self._h, int(v)))

    def set_insert_mode(self, mode: int):
        _check(lib().sbf_set_insert_mode(self._h, int(mode)))

    def set_query_mode(self, mode: int):
        _check(lib().sbf_set_query_mode(self._h, int(mode)))

    def set_launch(self, insert_wgs_per_cu: int = 0, query_wgs_per_cu: int = 0):
        """0 = one workgroup per tile; n > 0 = persistent grid of n workgroups per CU."""
        _check(lib().sbf_set_launch(self._h, int(insert_wgs_per_cu), int(query_wgs_per_cu)))

    def get_launch(self) -> dict:
        iw, qw = ctypes.c_uint32(), ctypes.c_uint32()
        im, qm = ctypes.c_int(), ctypes.c_int()
        _check(lib().sbf_get_launch(self._h, ctypes.byref(iw), ctypes.byref(qw), ctypes.byref(im), ctypes.byref(qm)))
        return {"insert_wgs_per_cu": iw.value, "query_wgs_per_cu": qw.value, "insert_mode": im.value,
                "query_mode": qm.value}

    def set_tile(self, insert_kmers_per_lane: int = 0, query_kmers_per_lane: int = 0):
        """k-mers per lane of the insert and query tiles (0 = default)."""
        _check(lib().sbf_set_tile(self._h, int(insert_kmers_per_lane), int(query_kmers_per_lane)))

    def get_tile(self) -> tuple:
        i, q = ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().sbf_get_tile(self._h, ctypes.byref(i), ctypes.byref(q)))
        return i.value, q.value

    def autotune(self, ins, ins_off, q, q_off) -> str:
        """Time launch shapes and kernel organisations on device batches and keep
        the fastest (sbf_autotune).  Returns the timing report."""
        buf = ctypes.create_string_buffer(8192)
        _check(lib().sbf_autotune(self._h, ctypes.c_void_p(ins.data_ptr()), ins.numel(),
                                  ctypes.c_void_p(ins_off.data_ptr()), ins_off.numel() - 1,
                                  ctypes.c_void_p(q.data_ptr()), q.numel(), ctypes.c_void_p(q_off.data_ptr()),
                                  q_off.numel() - 1, buf, len(buf)))
        return buf.value.decode()

    def set_staging_bytes(self, n: int):
        _check(lib().sbf_set_staging_bytes(self._h, int(n)))

    def get_bits(self) -> np.ndarray:
        out = np.empty(self.num_words, dtype=np.uint64)
        _check(lib().sbf_get_bits(self._h, out.ctypes.data_as(ctypes.c_void_p), out.size))
        return out

    def set_bits(self, words):
        a = np.ascontiguousarray(words, dtype=np.uint64)
        _check(lib().sbf_set_bits(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size))

    def estimate_fpr(self):
        """(expected FPR of absent uniformly sharded k-mers, set bits) from the
        filter's sector popcounts (sbf_estimate_fpr)."""
        fpr, nb = ctypes.c_double(), ctypes.c_uint64()
        _check(lib().sbf_estimate_fpr(self._h, ctypes.byref(fpr), ctypes.byref(nb)))
        return fpr.value, nb.value

    def clear(self, stream=None):
        _check(lib().sbf_clear(self._h, _stream_handle(stream)))

    # -- insert / query ------------------------------------------------------------
    def insert(self, seq, offsets=None, stream=None):
        """Insert a sequence (or a record batch with ``offsets``).  CUDA tensors
        run stream-ordered on ``stream`` (default: torch's current stream)."""
        L = lib()
        if _is_cuda(seq):
            st = _stream_handle(stream)
            if offsets is None:
                _check(L.sbf_insert_seq_dev(self._h, ctypes.c_void_p(seq.data_ptr()), seq.numel(), st))
            else:
                _check(L.sbf_insert_batch_dev(self._h, ctypes.c_void_p(seq.data_ptr()), seq.numel(),
                                              ctypes.c_void_p(offsets.data_ptr()), offsets.numel() - 1, st))
            return
        a = _host_u8(seq)
        if offsets is None:
            _check(L.sbf_insert_seq(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size))
        else:
            off = np.ascontiguousarray(offsets, dtype=np.uint64)
            _check(L.sbf_insert_batch(self._h, a.ctypes.data_as(ctypes.c_void_p),
                                      off.ctypes.data_as(ctypes.c_void_p), off.size - 1))

    # -- record batches in two steps (device tensors) ----------------------------
    @staticmethod
    def mark_record_starts(offsets, length, starts=None, stream=None):
        """Record-start bits of a device batch (int32 tensor of ceil(len/32)
        words, reused by insert_marked / query_marked)."""
        import torch

        if starts is None:
            starts = torch.empty((int(length) + 31) // 32, dtype=torch.int32, device=offsets.device)
        _check(lib().sbf_mark_record_starts_dev(ctypes.c_void_p(offsets.data_ptr()), offsets.numel() - 1,
                                                int(length), ctypes.c_void_p(starts.data_ptr()),
                                                _stream_handle(stream)))
        return starts

    def insert_marked(self, seq, starts=None, stream=None):
        _check(lib().sbf_insert_marked_dev(self._h, ctypes.c_void_p(seq.data_ptr()), seq.numel(),
                                           ctypes.c_void_p(starts.data_ptr() if starts is not None else None),
                                           _stream_handle(stream)))

    def query_marked(self, seq, starts=None, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty(seq.numel(), dtype=torch.uint8, device=seq.device)
        _check(lib().sbf_query_marked_dev(self._h, ctypes.c_void_p(seq.data_ptr()), seq.numel(),
                                          ctypes.c_void_p(starts.data_ptr() if starts is not None else None),
                                          ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out

    def query(self, seq, offsets=None, out=None, stream=None):
        """Answers as uint8 0/1.  A single sequence gives len-k+1 answers; a
        record batch gives one answer per base position (len of the batch)."""
        L = lib()
        if _is_cuda(seq):
            import torch

            st = _stream_handle(stream)
            n = seq.numel() if offsets is not None else max(0, seq.numel() - self.k + 1)
            if out is None:
                out = torch.empty(n, dtype=torch.uint8, device=seq.device)
            if offsets is None:
                _check(L.sbf_query_seq_dev(self._h, ctypes.c_void_p(seq.data_ptr()), seq.numel(),
                                           ctypes.c_void_p(out.data_ptr()), st))
            else:
                _check(L.sbf_query_batch_dev(self._h, ctypes.c_void_p(seq.data_ptr()), seq.numel(),
                                             ctypes.c_void_p(offsets.data_ptr()), offsets.numel() - 1,
                                             ctypes.c_void_p(out.data_ptr()), st))
            return out
        # host buffers (numpy arrays or CPU tensors; pinned tensors are copied
        # without an extra staging copy)
        a = _host_u8(seq)
        n = max(0, a.size - self.k + 1) if offsets is None else a.size
        res = np.zeros(n, dtype=np.uint8) if out is None else out
        if hasattr(res, "data_ptr"):
            if res.numel() < n or not res.is_contiguous():
                raise ValueError("out must be a contiguous buffer of at least %d bytes" % n)
            res_p = ctypes.c_void_p(res.data_ptr())
        else:
            if res.size < n or not res.flags.c_contiguous:
                raise ValueError("out must be a contiguous buffer of at least %d bytes" % n)
            res_p = res.ctypes.data_as(ctypes.c_void_p)
        if offsets is None:
            if n:
                _check(L.sbf_query_seq(self._h, a.ctypes.data_as(ctypes.c_void_p), a.size, res_p))
            return res
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        _check(L.sbf_query_batch(self._h, a.ctypes.data_as(ctypes.c_void_p), off.ctypes.data_as(ctypes.c_void_p),
                                 off.size - 1, res_p))
        return res


    def query_batch_dev_noalloc(self, seq, offsets, out, stream=None):
        """Query a device record batch without any device allocation
        (sbf_query_batch_dev_noalloc: fixed per-GPU scratch, at most 2^26
        bases per call, calls on one GPU must not overlap).  ``out`` is a
        caller-allocated uint8 device tensor of len(seq) bytes."""
        _check(lib().sbf_query_batch_dev_noalloc(self._h, ctypes.c_void_p(seq.data_ptr()), seq.numel(),
                                                 ctypes.c_void_p(offsets.data_ptr()), offsets.numel() - 1,
                                                 ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)))
        return out


def autotune_geometry(k, s, m, H, bits, ins, ins_off, q, q_off, neg, neg_off, max_fpr):
    """Shard-geometry autotuner (sbf_autotune_geometry) on device batches:
    returns a dict with the chosen shard words, tile lengths, FPR and the
    report of every trial."""
    def p(t):
        return ctypes.c_void_p(t.data_ptr())

    S, il, ql = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    fpr = ctypes.c_double()
    buf = ctypes.create_string_buffer(65536)
    _check(lib().sbf_autotune_geometry(int(k), int(s), int(m), int(H), int(bits), p(ins), ins.numel(), p(ins_off),
                                       ins_off.numel() - 1, p(q), q.numel(), p(q_off), q_off.numel() - 1, p(neg),
                                       neg.numel(), p(neg_off), neg_off.numel() - 1, float(max_fpr),
                                       ctypes.byref(S), ctypes.byref(il), ctypes.byref(ql), ctypes.byref(fpr), buf,
                                       len(buf)))
    return {"shard_words": S.value, "insert_kmers_per_lane": il.value, "query_kmers_per_lane": ql.value,
            "fpr": fpr.value, "report": buf.value.decode()}


class Graph:
    """A captured HIP graph of one insert batch and/or one query batch on a
    filter (sbf_graph_create).  Device tensors; the caller keeps them alive."""

    def __init__(self, f: Filter, ins=None, ins_off=None, q=None, q_off=None, out=None, clear_first=False):
        def ptr(t):
            return ctypes.c_void_p(t.data_ptr()) if t is not None else None

        h = lib().sbf_graph_create(f.handle, int(bool(clear_first)), ptr(ins), ins.numel() if ins is not None else 0,
                                   ptr(ins_off), ins_off.numel() - 1 if ins_off is not None else 0, ptr(q),
                                   q.numel() if q is not None else 0, ptr(q_off),
                                   q_off.numel() - 1 if q_off is not None else 0, ptr(out))
        if not h:
            code, msg = last_error()
            raise SBFError(code, msg)
        self._h = ctypes.c_void_p(h)
        self._keep = (f, ins, ins_off, q, q_off, out)

    def launch(self, stream=None):
        _check(lib().sbf_graph_launch(self._h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().sbf_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching query server over a resident filter
    (sbf_server_create).  Requests are host record batches; pinned buffers
    (torch ``pin_memory=True``) let the copies run asynchronously."""

    def __init__(self, f: Filter, slots=4, slot_bases=1 << 24, slot_records=1 << 16, max_pending=1 << 16):
        h = lib().sbf_server_create(f.handle, int(slots), int(slot_bases), int(slot_records), int(max_pending))
        if not h:
            code, msg = last_error()
            raise SBFError(code, msg)
        self._h = ctypes.c_void_p(h)
        self._f = f
        self._keep = {}

    @staticmethod
    def _ptr(x):
        if x is None:
            return None
        if hasattr(x, "data_ptr"):
            return ctypes.c_void_p(x.data_ptr())
        return x.ctypes.data_as(ctypes.c_void_p)

    def set_batch_window(self, microseconds: int):
        """Hold a free slot up to this long for more requests to join a batch."""
        _check(lib().sbf_server_set_batch_window(self._h, int(microseconds)))

    def submit(self, seq, offsets, out) -> int:
        """Queue a query of a host record batch; out receives len(seq) bytes.
        The three buffers stay referenced until wait()."""
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        t = ctypes.c_uint64()
        _check(lib().sbf_server_submit(self._h, self._ptr(seq), off.ctypes.data_as(ctypes.c_void_p), off.size - 1,
                                       self._ptr(out), ctypes.byref(t)))
        self._keep[t.value] = (seq, off, out)
        return t.value

    def poll(self, ticket: int) -> bool:
        rc = lib().sbf_server_poll(self._h, int(ticket))
        if rc < 0:
            _check(rc)
        return rc == 1

    def wait(self, ticket: int):
        """Block until the request is done; returns (latency_ms, queue_ms)."""
        lat, que = ctypes.c_double(), ctypes.c_double()
        rc = lib().sbf_server_wait(self._h, int(ticket), ctypes.byref(lat), ctypes.byref(que))
        self._keep.pop(int(ticket), None)
        _check(rc)
        return lat.value, que.value

    def stats(self) -> dict:
        v = [ctypes.c_uint64() for _ in range(4)]
        _check(lib().sbf_server_stats(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(["batches", "requests", "bases", "max_batch_requests"], [x.value for x in v]))

    def close(self):
        if getattr(self, "_h", None):
            lib().sbf_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
