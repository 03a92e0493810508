"""The C-ABI library loads on a machine without a GPU, exports every entry
point ``include/hoszp.h`` declares, and its host-only functions agree with the
oracle (no kernel launches here)."""
import os
import re

import numpy as np
import pytest

import paper_2408_11971_amd as hz
from oracle import ref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hoszp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hoszp_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hz.LIB_PATH):
        from paper_2408_11971_amd import build
        build.build()
    return hz._lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(hz.exported_symbols())


def test_result_record_is_64_bytes():
    assert hz.result_struct_size() == 64 == hz.RESULT_BYTES


@pytest.mark.parametrize("L", [32, 64, 128, 256])
def test_compress_bound_matches_oracle(lib, L):
    for n in [1, 2, 31, 32, 33, 1000, 8191, 8192, 8193, 123457, 1 << 20, 2**32 - 1]:
        assert hz.compress_bound(n, L) == ref.bound(n, L)


def test_compress_bound_rejects_bad_args(lib):
    assert hz.compress_bound(0, 32) == 0
    assert hz.compress_bound(10, 16) == 0
    assert hz.compress_bound(10, 512) == 0
    assert hz.compress_bound(2**32, 32) == 0


@pytest.mark.parametrize("L", [32, 64, 128, 256])
def test_parse_header_matches_oracle(lib, L):
    x = np.random.default_rng(L).normal(0, 1, 5000).astype(np.float32)
    c = ref.compress(x, 0.01, L)
    info = ref.info(c)
    h = hz.parse_header(c[:64].tobytes())
    assert h["n"] == info["n"] and h["block"] == L and h["eb"] == info["eb"]
    assert h["payload_bytes"] == info["payload_bytes"]
    assert h["total_bytes"] == info["total_bytes"] == c.size


def test_parse_header_rejects_corruption(lib):
    c = ref.compress(np.zeros(100, np.float32), 0.5, 32)
    for off, val in [(0, 0), (4, 2), (6, 1), (8, 48), (32, 9), (40, 5)]:
        bad = c.copy()
        bad[off] = val
        with pytest.raises(hz.HoszpError) as e:
            hz.parse_header(bad[:64].tobytes())
        assert e.value.code == hz.ERR_FORMAT


def test_status_precedence(lib):
    bit = lambda code: 1 << code
    assert hz.status_code(0) == hz.OK
    assert hz.status_code(bit(hz.ERR_RANGE) | bit(hz.ERR_NONFINITE)) == hz.ERR_NONFINITE
    assert hz.status_code(bit(hz.ERR_RANGE) | bit(hz.ERR_FORMAT)) == hz.ERR_FORMAT
    assert hz.status_code(bit(hz.ERR_CAPACITY) | bit(hz.ERR_MISMATCH)) == hz.ERR_MISMATCH
    assert hz.status_code(bit(hz.ERR_RANGE)) == hz.ERR_RANGE
    # a look-back that gave up outranks what its invalid prefix caused
    assert hz.status_code(bit(hz.ERR_TIMEOUT) | bit(hz.ERR_FORMAT) | bit(hz.ERR_ARG)) == hz.ERR_TIMEOUT
    assert b"poll limit" in hz._lib().hoszp_strerror(hz.ERR_TIMEOUT)


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(hz, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(hz, "_LIB", None)
    with pytest.raises(hz.HoszpUnavailable):
        hz.compress_bound(10, 32)


def test_batch_structs_match_header(lib):
    import ctypes
    assert ctypes.sizeof(hz.Field) == 48
    assert ctypes.sizeof(hz.FieldResult) == 64
    assert ctypes.sizeof(hz.BatchInfo) == 40


def test_batch_create_rejects_null_context(lib):
    import ctypes
    h = ctypes.c_void_p()
    table = (hz.Field * 1)()
    assert lib.hoszp_batch_create(None, table, 1, 0, None, ctypes.byref(h), None) == hz.ERR_ARG
    assert lib.hoszp_batch_launch(None, None) == hz.ERR_ARG
    assert lib.hoszp_batch_destroy(None) == hz.OK
    assert lib.hoszp_batch_device_results(None) is None


def test_batch_out_cap_covers_every_block(lib):
    for n in [1, 31, 33, 1000, 8193, 1 << 20]:
        cap = hz.batch_out_cap(n)
        assert cap == max(ref.bound(n, L) for L in (32, 64, 128))
        assert hz.batch_out_cap(n, 64) == ref.bound(n, 64)


def test_server_structs_match_header(lib):
    import ctypes
    req, cpl = hz._np_dtypes()
    assert req.itemsize == 80 and cpl.itemsize == 64
    assert ctypes.sizeof(hz.ServerConfig) == 24
    assert ctypes.sizeof(hz.ServerStats) == 56


def test_server_rejects_bad_config_without_device(lib):
    import ctypes
    h = ctypes.c_void_p()
    bad = [hz.ServerConfig(0, 0, 1 << 20, 0.0), hz.ServerConfig(65, 0, 1 << 20, 0.0),
           hz.ServerConfig(4, 0, 0, 0.0), hz.ServerConfig(4, 2, 1 << 20, 0.0),
           hz.ServerConfig(4, 0, 1 << 20, -1.0)]
    for cfg in bad:
        assert lib.hoszp_server_create(0, ctypes.byref(cfg), ctypes.byref(h)) == hz.ERR_ARG
    assert lib.hoszp_server_create(0, None, ctypes.byref(h)) == hz.ERR_ARG
    assert lib.hoszp_server_submit(None, None) == hz.ERR_ARG
    assert lib.hoszp_server_pending(None) == 0
    assert lib.hoszp_server_destroy(None) == hz.OK
