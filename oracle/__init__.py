"""CPU oracle of the Super Bloom filter insert/query path (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``sbf_oracle.c`` (plain C, one
k-mer at a time, Algorithms 1 and 2 of the paper) through ctypes and shares no
code with the GPU library.

Inputs are numpy arrays: sequences are ``uint8`` ASCII, record offsets are
``uint64`` with ``nrec + 1`` entries, filters are ``uint64`` words laid out as
``shard * shard_words + word``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sbf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64


_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
# gcc flags of the checked build: AddressSanitizer and UndefinedBehaviorSanitizer,
# any finding fatal (the process aborts, so the calling test fails)
SANITIZE_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=all"]


def sanitized() -> bool:
    """True when this process is to load the sanitizer build (environment
    variable SBF_ORACLE_SANITIZE=1; the sanitizer runtimes must then be
    preloaded, since the Python interpreter is not built with them)."""
    return os.environ.get("SBF_ORACLE_SANITIZE") == "1"


def build(force: bool = True, sanitize: bool | None = None) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc, or with
    ``sanitize`` into ``oracle/liboracle_san.so`` under ASan and UBSan."""
    if sanitize is None:
        sanitize = sanitized()
    out = _LIB_SAN if sanitize else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp%d" % os.getpid()
        flags = SANITIZE_FLAGS if sanitize else ["-O2"]
        subprocess.check_call(["gcc"] + flags + ["-std=c99", "-Wall", "-Werror", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, out)
    return out


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build(force=False))
        L.orc_base_code.argtypes = [ctypes.c_ubyte]
        L.orc_base_code.restype = ctypes.c_int
        L.orc_hash_minimizer.argtypes = [_u64]
        L.orc_hash_minimizer.restype = _u64
        L.orc_hash_smer.argtypes = [_u64]
        L.orc_hash_smer.restype = _u64
        L.orc_bit_address.argtypes = [_u64, _u32, _u32]
        L.orc_bit_address.restype = _u32
        L.orc_word_index.argtypes = [_u64, _u32, _u32, _u32]
        L.orc_word_index.restype = _u32
        L.orc_num_shards.argtypes = [_u64, _u32]
        L.orc_num_shards.restype = _u64
        L.orc_subwindow.argtypes = [_u64, _u32, _u32, _u32]
        L.orc_subwindow.restype = _u64
        L.orc_min_hash.argtypes = [_u64, _u32, _u32]
        L.orc_min_hash.restype = _u64
        L.orc_insert_records.argtypes = [_u32, _u32, _u32, _u32, _u32, _u64, _u64p, _u8p, _u64p, _u64]
        L.orc_insert_records.restype = None
        L.orc_insert_records_shared.argtypes = L.orc_insert_records.argtypes
        L.orc_insert_records_shared.restype = None
        L.orc_query_records.argtypes = [_u32, _u32, _u32, _u32, _u32, _u64, _u64p, _u8p, _u64p, _u64, _u8p]
        L.orc_query_records.restype = None
        L.orc_kmer_shards.argtypes = [_u32, _u32, _u64, _u8p, _u64, _u64p]
        L.orc_kmer_shards.restype = None
        L.orc_kmer_min_hashes.argtypes = [_u32, _u32, _u8p, _u64, _u64p, _u8p]
        L.orc_kmer_min_hashes.restype = None
        L.orc_count_runs.argtypes = [_u64p, _u8p, _u64]
        L.orc_count_runs.restype = _u64
        L.orc_count_segments.argtypes = [_u32, _u32, _u64, _u8p, _u64p, _u64, _u32p, _u64]
        L.orc_count_segments.restype = _u64
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _u8(seq) -> np.ndarray:
    if isinstance(seq, (bytes, bytearray)):
        return np.frombuffer(bytes(seq), dtype=np.uint8)
    if isinstance(seq, str):
        return np.frombuffer(seq.encode("ascii"), dtype=np.uint8)
    a = np.ascontiguousarray(seq, dtype=np.uint8)
    return a


def _offsets(seq: np.ndarray, offsets) -> np.ndarray:
    if offsets is None:
        return np.array([0, seq.size], dtype=np.uint64)
    return np.ascontiguousarray(offsets, dtype=np.uint64)


# --- scalar definitions -----------------------------------------------------

def base_code(c: int) -> int:
    return lib().orc_base_code(c)


def hash_minimizer(y: int) -> int:
    return lib().orc_hash_minimizer(y)


def hash_smer(v: int) -> int:
    return lib().orc_hash_smer(v)


def bit_address(g: int, t: int, H: int) -> int:
    return lib().orc_bit_address(g, t, H)


def word_index(g: int, t: int, H: int, shard_words: int = 4) -> int:
    return lib().orc_word_index(g, t, H, shard_words)


def num_shards(bits: int, shard_words: int = 4) -> int:
    return lib().orc_num_shards(bits, shard_words)


def subwindow(K: int, k: int, L: int, j: int) -> int:
    return lib().orc_subwindow(K, k, L, j)


def min_hash(K: int, k: int, m: int) -> int:
    return lib().orc_min_hash(K, k, m)


# --- filters ----------------------------------------------------------------

class Params:
    def __init__(self, k=31, s=28, m=16, H=4, bits=1 << 24, shard_words=4):
        self.k, self.s, self.m, self.H = int(k), int(s), int(m), int(H)
        self.shard_words = int(shard_words)
        self.nshards = num_shards(int(bits), self.shard_words)

    @property
    def nwords(self) -> int:
        return self.nshards * self.shard_words

    def empty(self) -> np.ndarray:
        return np.zeros(self.nwords, dtype=np.uint64)


def insert(p: Params, F: np.ndarray, seq, offsets=None) -> np.ndarray:
    """OR every valid k-mer of every record into F (in place); returns F."""
    s = _u8(seq)
    off = _offsets(s, offsets)
    assert F.dtype == np.uint64 and F.flags.c_contiguous and F.size == p.nwords
    lib().orc_insert_records(p.k, p.s, p.m, p.H, p.shard_words, p.nshards, _p(F, _u64p),
                             _p(s, _u8p), _p(off, _u64p), off.size - 1)
    return F


def pieces(off: np.ndarray, total: int, n: int, k: int):
    """Split bases [0, total) of a record batch into at most n ranges whose
    k-mer starts partition [0, total - k + 1): (a, b, e, local offsets), where
    the range holds bases [a, e) with e = min(total, b + k - 1) and its record
    starts as offsets local to a.  Every k-mer starting in [a, b) lies inside
    the range, so a range inserts or answers exactly those k-mers."""
    off = np.asarray(off, dtype=np.uint64)
    cuts = np.unique(np.linspace(0, max(total - k + 1, 0), n + 1).astype(np.int64))
    out = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        a, b = int(a), int(b)
        e = min(total, b + k - 1)
        inner = off[(off > a) & (off < e)].astype(np.int64) - a
        loc = np.concatenate(([0], inner, [e - a])).astype(np.uint64)
        out.append((a, b, e, loc))
    return out


def _threads(threads) -> int:
    return max(1, int(threads or os.cpu_count() or 1))


def insert_parallel(p: Params, F: np.ndarray, seq, offsets=None, threads: int | None = None) -> np.ndarray:
    """insert() on several threads into the one filter F: the batch is cut
    into k-1-overlapping pieces (pieces()) that insert with atomic ORs
    (orc_insert_records_shared); the result equals insert()."""
    from concurrent.futures import ThreadPoolExecutor

    s = _u8(seq)
    off = _offsets(s, offsets)
    assert F.dtype == np.uint64 and F.flags.c_contiguous and F.size == p.nwords
    nt = _threads(threads)
    L = lib()

    def run(job):
        a, _, e, loc = job
        part = s[a:e]
        L.orc_insert_records_shared(p.k, p.s, p.m, p.H, p.shard_words, p.nshards, _p(F, _u64p),
                                    _p(part, _u8p), _p(loc, _u64p), loc.size - 1)

    jobs = pieces(off, s.size, 4 * nt, p.k)
    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(run, jobs))
    return F


def query_parallel(p: Params, F: np.ndarray, seq, offsets, threads: int | None = None) -> np.ndarray:
    """query() of a record batch on several threads (answers per base
    position, length offsets[-1]); equal to query(p, F, seq, offsets)."""
    from concurrent.futures import ThreadPoolExecutor

    s = _u8(seq)
    off = _offsets(s, offsets)
    F = np.ascontiguousarray(F)
    assert F.dtype == np.uint64 and F.size == p.nwords
    out = np.zeros(s.size, dtype=np.uint8)
    nt = _threads(threads)
    L = lib()

    def run(job):
        a, b, e, loc = job
        part = s[a:e]
        res = np.zeros(e - a, dtype=np.uint8)
        L.orc_query_records(p.k, p.s, p.m, p.H, p.shard_words, p.nshards, _p(F, _u64p), _p(part, _u8p),
                            _p(loc, _u64p), loc.size - 1, _p(res, _u8p))
        out[a:b] = res[:b - a]

    jobs = pieces(off, s.size, 4 * nt, p.k)
    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(run, jobs))
    return out


def query(p: Params, F: np.ndarray, seq, offsets=None, per_base: bool | None = None) -> np.ndarray:
    """Answers per k-mer.  With offsets (a record batch) the result is indexed
    by base position (length ``offsets[-1]``); for a single sequence it has
    ``len - k + 1`` entries (empty when ``len < k``)."""
    s = _u8(seq)
    single = offsets is None
    off = _offsets(s, offsets)
    out = np.zeros(s.size, dtype=np.uint8)
    assert F.dtype == np.uint64 and F.size == p.nwords
    F = np.ascontiguousarray(F)
    lib().orc_query_records(p.k, p.s, p.m, p.H, p.shard_words, p.nshards, _p(F, _u64p),
                            _p(s, _u8p), _p(off, _u64p), off.size - 1, _p(out, _u8p))
    if single if per_base is None else not per_base:
        return out[: max(0, s.size - p.k + 1)]
    return out


def kmer_shards(p: Params, seq) -> np.ndarray:
    s = _u8(seq)
    n = max(0, s.size - p.k + 1)
    out = np.zeros(n, dtype=np.uint64)
    if n:
        lib().orc_kmer_shards(p.k, p.m, p.nshards, _p(s, _u8p), s.size, _p(out, _u64p))
    return out


def kmer_min_hashes(k: int, m: int, seq):
    s = _u8(seq)
    n = max(0, s.size - k + 1)
    mu = np.zeros(n, dtype=np.uint64)
    valid = np.zeros(n, dtype=np.uint8)
    if n:
        lib().orc_kmer_min_hashes(k, m, _p(s, _u8p), s.size, _p(mu, _u64p), _p(valid, _u8p))
    return mu, valid.astype(bool)


def count_runs(shards, active) -> int:
    sh = np.ascontiguousarray(shards, dtype=np.uint64)
    ac = np.ascontiguousarray(active, dtype=np.uint8)
    return lib().orc_count_runs(_p(sh, _u64p), _p(ac, _u8p), sh.size)


def count_segments(p: Params, seq, offsets=None, with_lengths: bool = False):
    s = _u8(seq)
    off = _offsets(s, offsets)
    if not with_lengths:
        return lib().orc_count_segments(p.k, p.m, p.nshards, _p(s, _u8p), _p(off, _u64p),
                                        off.size - 1, None, 0)
    cap = max(1, s.size)
    lengths = np.zeros(cap, dtype=np.uint32)
    n = lib().orc_count_segments(p.k, p.m, p.nshards, _p(s, _u8p), _p(off, _u64p),
                                 off.size - 1, _p(lengths, _u32p), cap)
    return n, lengths[:n].copy()
