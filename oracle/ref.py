"""ctypes binding of the CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module.  Arrays are numpy arrays on the host; compressed streams are
``numpy.uint8`` arrays whose length is the stream's total size.
"""
import ctypes
import os

import numpy as np

from . import build as _build

OK, ERR_ARG, ERR_NONFINITE, ERR_RANGE, ERR_FORMAT, ERR_MISMATCH, ERR_CAPACITY = range(7)
_NAMES = {OK: "ok", ERR_ARG: "bad argument", ERR_NONFINITE: "non-finite input",
          ERR_RANGE: "bin out of range", ERR_FORMAT: "malformed stream",
          ERR_MISMATCH: "operand mismatch", ERR_CAPACITY: "output too small"}


class RefError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {_NAMES.get(code, code)} ({code})")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("HOSZP_REF_LIB")  # lets the mutation tests load a planted copy
        if not path:
            path = _build.LIB
            if not os.path.exists(path):
                _build.build()
        L = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        f32p = ctypes.POINTER(ctypes.c_float)
        i32p = ctypes.POINTER(ctypes.c_int32)
        sz, u64, u32, dbl = ctypes.c_size_t, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        P = ctypes.POINTER
        sig = {
            "hoszp_ref_bound": (sz, [u64, u32]),
            "hoszp_ref_quantize": (ctypes.c_int, [f32p, u64, dbl, i32p]),
            "hoszp_ref_compress": (ctypes.c_int, [f32p, u64, dbl, u32, u8p, sz, P(sz)]),
            "hoszp_ref_encode_bins": (ctypes.c_int, [i32p, u64, dbl, u32, u8p, sz, P(sz)]),
            "hoszp_ref_info": (ctypes.c_int, [u8p, sz, P(u64), P(u32), P(dbl), P(u64), P(u64)]),
            "hoszp_ref_decode_bins": (ctypes.c_int, [u8p, sz, i32p, u64]),
            "hoszp_ref_decompress": (ctypes.c_int, [u8p, sz, f32p, u64]),
            "hoszp_ref_negate": (ctypes.c_int, [u8p, sz, u8p, sz, P(sz)]),
            "hoszp_ref_add": (ctypes.c_int, [u8p, sz, u8p, sz, u8p, sz, P(sz)]),
            "hoszp_ref_mul": (ctypes.c_int, [u8p, sz, dbl, u8p, sz, P(sz)]),
            "hoszp_ref_sums": (ctypes.c_int, [u8p, sz, P(ctypes.c_int64), P(u64), P(u64)]),
            "hoszp_ref_mean": (ctypes.c_int, [u8p, sz, P(dbl)]),
            "hoszp_ref_variance": (ctypes.c_int, [u8p, sz, P(dbl)]),
            "hoszp_ref_scalar_add": (ctypes.c_int, [u8p, sz, dbl, u8p, sz, P(sz)]),
            "hoszp_ref_scalar_sub": (ctypes.c_int, [u8p, sz, dbl, u8p, sz, P(sz)]),
            "hoszp_ref_std": (ctypes.c_int, [u8p, sz, P(dbl)]),
            "hoszp_ref_sub": (ctypes.c_int, [u8p, sz, u8p, sz, u8p, sz, P(sz)]),
            "hoszp_ref_hadamard": (ctypes.c_int, [u8p, sz, u8p, sz, u8p, sz, P(sz)]),
            "hoszp_ref_covariance": (ctypes.c_int, [u8p, sz, u8p, sz, P(dbl)]),
            "hoszp_ref_block_means": (ctypes.c_int, [u8p, sz, P(dbl), u64, P(u64)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _check(rc, where):
    if rc != OK:
        raise RefError(rc, where)


def bound(n: int, block: int) -> int:
    return lib().hoszp_ref_bound(n, block)


def quantize(x: np.ndarray, eb: float) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    q = np.empty(x.size, dtype=np.int32)
    _check(lib().hoszp_ref_quantize(_ptr(x, ctypes.c_float), x.size, eb, _ptr(q, ctypes.c_int32)),
           "quantize")
    return q


def _stream_out(n, block):
    cap = bound(n, block)
    if cap == 0:
        raise RefError(ERR_ARG, "bound")
    return np.zeros(cap, dtype=np.uint8), ctypes.c_size_t(0)


def compress(x: np.ndarray, eb: float, block: int = 32) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32).ravel()
    out, nbytes = _stream_out(max(x.size, 1), block)
    rc = lib().hoszp_ref_compress(_ptr(x, ctypes.c_float), x.size, eb, block,
                                  _ptr(out, ctypes.c_uint8), out.size, ctypes.byref(nbytes))
    _check(rc, "compress")
    return out[:nbytes.value].copy()


def encode_bins(q: np.ndarray, eb: float, block: int = 32) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.int32).ravel()
    out, nbytes = _stream_out(max(q.size, 1), block)
    rc = lib().hoszp_ref_encode_bins(_ptr(q, ctypes.c_int32), q.size, eb, block,
                                     _ptr(out, ctypes.c_uint8), out.size, ctypes.byref(nbytes))
    _check(rc, "encode_bins")
    return out[:nbytes.value].copy()


def _u8(c):
    c = np.ascontiguousarray(c, dtype=np.uint8)
    return c, _ptr(c, ctypes.c_uint8)


def info(c: np.ndarray) -> dict:
    c, p = _u8(c)
    n, blk, eb = ctypes.c_uint64(), ctypes.c_uint32(), ctypes.c_double()
    pay, tot = ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().hoszp_ref_info(p, c.size, ctypes.byref(n), ctypes.byref(blk), ctypes.byref(eb),
                                ctypes.byref(pay), ctypes.byref(tot)), "info")
    return {"n": n.value, "block": blk.value, "eb": eb.value,
            "payload_bytes": pay.value, "total_bytes": tot.value}


def decode_bins(c: np.ndarray) -> np.ndarray:
    c, p = _u8(c)
    n = info(c)["n"]
    q = np.empty(n, dtype=np.int32)
    _check(lib().hoszp_ref_decode_bins(p, c.size, _ptr(q, ctypes.c_int32), n), "decode_bins")
    return q


def decompress(c: np.ndarray) -> np.ndarray:
    c, p = _u8(c)
    n = info(c)["n"]
    x = np.empty(n, dtype=np.float32)
    _check(lib().hoszp_ref_decompress(p, c.size, _ptr(x, ctypes.c_float), n), "decompress")
    return x


def negate(c: np.ndarray) -> np.ndarray:
    c, p = _u8(c)
    out = np.zeros(c.size, dtype=np.uint8)
    nbytes = ctypes.c_size_t(0)
    _check(lib().hoszp_ref_negate(p, c.size, _ptr(out, ctypes.c_uint8), out.size,
                                  ctypes.byref(nbytes)), "negate")
    return out[:nbytes.value].copy()


def add(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a, pa = _u8(a)
    b, pb = _u8(b)
    ia = info(a)
    out, nbytes = _stream_out(ia["n"], ia["block"])
    _check(lib().hoszp_ref_add(pa, a.size, pb, b.size, _ptr(out, ctypes.c_uint8), out.size,
                               ctypes.byref(nbytes)), "add")
    return out[:nbytes.value].copy()


def mul(c: np.ndarray, s: float) -> np.ndarray:
    c, p = _u8(c)
    ic = info(c)
    out, nbytes = _stream_out(ic["n"], ic["block"])
    _check(lib().hoszp_ref_mul(p, c.size, float(s), _ptr(out, ctypes.c_uint8), out.size,
                               ctypes.byref(nbytes)), "mul")
    return out[:nbytes.value].copy()


def sums(c: np.ndarray):
    """Exact (S, Q) of the bins as Python ints."""
    c, p = _u8(c)
    s, lo, hi = ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(lib().hoszp_ref_sums(p, c.size, ctypes.byref(s), ctypes.byref(lo), ctypes.byref(hi)),
           "sums")
    return s.value, (hi.value << 64) | lo.value


def mean(c: np.ndarray) -> float:
    c, p = _u8(c)
    r = ctypes.c_double()
    _check(lib().hoszp_ref_mean(p, c.size, ctypes.byref(r)), "mean")
    return r.value


def variance(c: np.ndarray) -> float:
    c, p = _u8(c)
    r = ctypes.c_double()
    _check(lib().hoszp_ref_variance(p, c.size, ctypes.byref(r)), "variance")
    return r.value


def _shift(fn, c, s):
    c, p = _u8(c)
    out = np.zeros(c.size, dtype=np.uint8)
    nbytes = ctypes.c_size_t(0)
    _check(fn(p, c.size, float(s), _ptr(out, ctypes.c_uint8), out.size, ctypes.byref(nbytes)),
           fn.__name__)
    return out[:nbytes.value].copy()


def scalar_add(c: np.ndarray, s: float) -> np.ndarray:
    return _shift(lib().hoszp_ref_scalar_add, c, s)


def scalar_sub(c: np.ndarray, s: float) -> np.ndarray:
    return _shift(lib().hoszp_ref_scalar_sub, c, s)


def std(c: np.ndarray) -> float:
    c, p = _u8(c)
    r = ctypes.c_double()
    _check(lib().hoszp_ref_std(p, c.size, ctypes.byref(r)), "std")
    return r.value


def _bivariate(fn, a, b):
    a, pa = _u8(a)
    b, pb = _u8(b)
    ia = info(a)
    out, nbytes = _stream_out(ia["n"], ia["block"])
    _check(fn(pa, a.size, pb, b.size, _ptr(out, ctypes.c_uint8), out.size, ctypes.byref(nbytes)),
           fn.__name__)
    return out[:nbytes.value].copy()


def sub(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return _bivariate(lib().hoszp_ref_sub, a, b)


def hadamard(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return _bivariate(lib().hoszp_ref_hadamard, a, b)


def covariance(a: np.ndarray, b: np.ndarray) -> float:
    a, pa = _u8(a)
    b, pb = _u8(b)
    r = ctypes.c_double()
    _check(lib().hoszp_ref_covariance(pa, a.size, pb, b.size, ctypes.byref(r)), "covariance")
    return r.value


def block_means(c: np.ndarray):
    """(per-block means as float64, number of constant blocks)."""
    c, p = _u8(c)
    ic = info(c)
    nb = (ic["n"] + ic["block"] - 1) // ic["block"]
    m = np.empty(nb, dtype=np.float64)
    k = ctypes.c_uint64()
    _check(lib().hoszp_ref_block_means(p, c.size, _ptr(m, ctypes.c_double), nb, ctypes.byref(k)),
           "block_means")
    return m, k.value


def raw(fn_name: str, *args):
    """Direct access to a C entry point for error-path tests."""
    return getattr(lib(), fn_name)(*args)
