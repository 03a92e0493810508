"""Error paths of the oracle: every failure the ABI documents, forced from
host-side inputs (no GPU)."""
import ctypes

import numpy as np
import pytest

from oracle import ref


def good_stream(n=100, L=32, eb=0.01, seed=0):
    x = np.random.default_rng(seed).normal(0, 1, n).astype(np.float32)
    return ref.compress(x, eb, L)


def code_of(fn, *args):
    with pytest.raises(ref.RefError) as e:
        fn(*args)
    return e.value.code


def test_nonfinite_inputs():
    for bad in (np.nan, np.inf, -np.inf):
        x = np.array([0.0, bad, 1.0], dtype=np.float32)
        assert code_of(ref.compress, x, 0.1, 32) == ref.ERR_NONFINITE
        assert code_of(ref.quantize, x, 0.1) == ref.ERR_NONFINITE


def test_nonfinite_wins_over_range():
    x = np.array([3e38, np.nan], dtype=np.float32)
    assert code_of(ref.compress, x, 1e-3, 32) == ref.ERR_NONFINITE


def test_bin_overflow_is_range_error():
    # (1e6 + 1e-4) / 2e-4 ~ 5e9 > 2^31 - 1
    x = np.array([0.0, 1e6], dtype=np.float32)
    assert code_of(ref.compress, x, 1e-4, 32) == ref.ERR_RANGE
    # the largest representable bin is fine: 2^31 - 1
    eb = 0.5
    x = np.array([2147483520.0], dtype=np.float32)   # float32 below 2^31
    q = ref.quantize(x, eb)
    assert q[0] == 2147483520


def test_bad_arguments():
    x = np.zeros(10, dtype=np.float32)
    for eb in (0.0, -1.0, np.inf, np.nan):
        assert code_of(ref.compress, x, eb, 32) == ref.ERR_ARG
    for L in (0, 16, 48, 512, 33):
        assert code_of(ref.compress, x, 0.1, L) == ref.ERR_ARG
    assert ref.bound(0, 32) == 0
    assert ref.bound(10, 48) == 0
    out = np.zeros(1024, dtype=np.uint8)
    nb = ctypes.c_size_t()
    xp = x.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    op = out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    assert ref.raw("hoszp_ref_compress", xp, 0, 0.1, 32, op, out.size, ctypes.byref(nb)) == ref.ERR_ARG


def test_capacity():
    x = np.zeros(1000, dtype=np.float32)
    need = ref.bound(1000, 32)
    out = np.zeros(need - 1, dtype=np.uint8)
    nb = ctypes.c_size_t()
    rc = ref.raw("hoszp_ref_compress", x.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), 1000, 0.1,
                 32, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), out.size, ctypes.byref(nb))
    assert rc == ref.ERR_CAPACITY


def corrupt(c, offset, value):
    d = c.copy()
    d[offset] = value
    return d


@pytest.mark.parametrize("op", ["decode_bins", "decompress", "negate", "mean", "variance"])
def test_malformed_streams(op):
    c = good_stream()
    fn = getattr(ref, op)
    cases = [
        corrupt(c, 0, ord("X")),          # magic
        corrupt(c, 4, 2),                 # version
        corrupt(c, 6, 1),                 # flags
        corrupt(c, 8, 48),                # block size
        corrupt(c, 32, c[32] + 1),        # block count
        corrupt(c, 64, 33),               # width > 32
        corrupt(c, 64, (int(c[64]) + 1) % 33),  # widths no longer fill the payload
        c[:-1],                           # truncated
        c[:40],                           # shorter than a header
    ]
    for bad in cases:
        with pytest.raises(ref.RefError) as e:
            fn(bad)
        assert e.value.code == ref.ERR_FORMAT


def test_outlier_out_of_range_is_format_error():
    c = good_stream()
    d = c.copy()
    d[80:84] = np.array([0x80000000], dtype=np.uint32).view(np.uint8)   # INT32_MIN
    assert code_of(ref.decode_bins, d) == ref.ERR_FORMAT
    assert code_of(ref.mean, d) == ref.ERR_FORMAT


def test_add_mismatch():
    a = good_stream(100, 32, 0.01)
    assert code_of(ref.add, a, good_stream(101, 32, 0.01)) == ref.ERR_MISMATCH
    assert code_of(ref.add, a, good_stream(100, 64, 0.01)) == ref.ERR_MISMATCH
    assert code_of(ref.add, a, good_stream(100, 32, 0.01 * (1 + 2**-52))) == ref.ERR_MISMATCH


def test_add_overflow_is_range_error():
    q = np.array([2**31 - 1, 2**31 - 1], dtype=np.int32)
    a = ref.encode_bins(q, 0.5, 32)
    assert code_of(ref.add, a, a) == ref.ERR_RANGE


def test_mul_errors():
    c = good_stream()
    assert code_of(ref.mul, c, np.inf) == ref.ERR_ARG
    assert code_of(ref.mul, c, np.nan) == ref.ERR_ARG
    big = ref.encode_bins(np.array([1 << 20, 3], dtype=np.int32), 0.5, 32)
    assert code_of(ref.mul, big, 4096.0) == ref.ERR_RANGE


def test_encode_rejects_int32_min():
    with pytest.raises(ref.RefError) as e:
        ref.encode_bins(np.array([-(2**31)], dtype=np.int32), 0.5, 32)
    assert e.value.code == ref.ERR_RANGE
