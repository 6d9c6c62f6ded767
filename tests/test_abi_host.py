"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/sbf.h declares, and rejects bad arguments before it
touches a device."""

import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "sbf.h")
PROBE_HEADER = os.path.join(ROOT, "include", "sbf_probe.h")


def header_functions(path=HEADER):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sbf_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2606_24417_amd import sbf

    if not os.path.exists(sbf.LIB_PATH):
        pytest.skip("libsbf.so not built")
    return sbf.lib()


def test_header_declares_the_core_abi():
    names = header_functions()
    for core in ("sbf_create", "sbf_insert_seq", "sbf_query_seq", "sbf_destroy"):
        assert core in names


def test_library_exports_every_declared_function(L):
    from paper_2606_24417_amd import sbf

    names = header_functions()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(sbf.SIGNATURES) == names


@pytest.mark.parametrize("k,s,m,H,bits", [
    (0, 1, 1, 1, 256), (33, 28, 16, 4, 256), (31, 32, 16, 4, 256), (31, 0, 16, 4, 256), (31, 28, 0, 4, 256),
    (31, 28, 32, 4, 256), (31, 28, 16, 0, 256), (31, 28, 16, 17, 256), (31, 28, 16, 4, 0),
    (31, 28, 16, 4, (1 << 40) + 1)])
def test_create_rejects_bad_parameters(L, k, s, m, H, bits):
    from paper_2606_24417_amd import sbf

    assert L.sbf_create(k, s, m, H, bits) is None
    code, msg = sbf.last_error()
    assert code == sbf.SBF_E_INVAL and "invalid parameters" in msg


@pytest.mark.parametrize("H,S", [(4, 5), (4, 0), (4, 32), (10, 8), (9, 16), (16, 8)])
def test_create_ex_rejects_bad_geometry(L, H, S):
    from paper_2606_24417_amd import sbf

    assert L.sbf_create_ex(31, 28, 16, H, 1 << 20, S) is None
    code, msg = sbf.last_error()
    assert code == sbf.SBF_E_INVAL and "shard geometry" in msg


def test_null_filter_calls_fail_cleanly(L):
    from paper_2606_24417_amd import sbf

    L.sbf_destroy(None)
    assert L.sbf_num_shards(None) == 0 and L.sbf_num_bits(None) == 0 and L.sbf_num_words(None) == 0
    buf = ctypes.create_string_buffer(64)
    for rc in (L.sbf_insert_seq(None, buf, 64), L.sbf_query_seq(None, buf, 64, buf),
               L.sbf_get_bits(None, buf, 1), L.sbf_set_bits(None, buf, 1), L.sbf_clear(None, None),
               L.sbf_insert_seq_dev(None, buf, 64, None), L.sbf_query_batch(None, buf, buf, 1, buf),
               L.sbf_set_variant(None, 0), L.sbf_set_staging_bytes(None, 1 << 20)):
        assert rc == sbf.SBF_E_INVAL
        assert sbf.last_error()[0] == sbf.SBF_E_INVAL


def test_server_rejects_bad_arguments_without_a_device(L):
    from paper_2606_24417_amd import sbf

    assert L.sbf_server_create(None, 1, 1 << 20, 16, 16) is None
    assert sbf.last_error()[0] == sbf.SBF_E_INVAL
    t = ctypes.c_uint64()
    assert L.sbf_server_submit(None, None, None, 0, None, ctypes.byref(t)) == sbf.SBF_E_INVAL
    assert L.sbf_server_poll(None, 1) == sbf.SBF_E_INVAL
    assert L.sbf_server_set_batch_window(None, 10) == sbf.SBF_E_INVAL
    assert L.sbf_server_wait(None, 1, None, None) == sbf.SBF_E_INVAL
    L.sbf_server_destroy(None)
    assert L.sbf_graph_launch(None, None) == sbf.SBF_E_INVAL
    L.sbf_graph_destroy(None)


def test_probe_library_exports_its_header():
    from paper_2606_24417_amd import build

    if not os.path.exists(build.PROBE_LIB):
        pytest.skip("libsbf_probe.so not built")
    L = ctypes.CDLL(build.PROBE_LIB)
    names = header_functions(PROBE_HEADER)
    assert names == ["sbf_probe_random_access", "sbf_probe_valu"]
    for n in names:
        assert hasattr(L, n)
    v = L.sbf_probe_valu
    v.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    c, d = ctypes.c_double(), ctypes.c_double()
    assert v(6, ctypes.byref(c), ctypes.byref(d)) == -1  # bad op
    assert v(-1, ctypes.byref(c), ctypes.byref(d)) == -1
    assert v(0, None, None) == -1
    # argument checks happen before any device call
    fn = L.sbf_probe_random_access
    fn.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    a, b = ctypes.c_double(), ctypes.c_double()
    ra, rb = ctypes.byref(a), ctypes.byref(b)
    assert fn(3 << 20, 0, 32, 8, 4, 1 << 20, ra, rb) == -1  # not a power of two
    assert fn(1 << 20, 9, 32, 8, 4, 1 << 20, ra, rb) == -1  # bad mode
    assert fn(1 << 20, 0, 32, 8, 4, 1 << 20, None, None) == -1
    assert fn(1 << 20, 0, 48, 8, 4, 1 << 20, ra, rb) == -1  # shard size
    assert fn(1 << 20, 1, 32, 3, 4, 1 << 20, ra, rb) == -1  # in-flight depth not compiled
    assert fn(1 << 20, 1, 128, 8, 4, 1 << 20, ra, rb) == -1
    assert fn(1 << 20, 0, 32, 8, 0, 1 << 20, ra, rb) == -1  # workgroups per CU
    assert fn(1 << 20, 0, 32, 8, 17, 1 << 20, ra, rb) == -1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2606_24417_amd import sbf

    monkeypatch.setattr(sbf, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sbf, "_lib", None)
    with pytest.raises(ImportError):
        sbf.lib()
