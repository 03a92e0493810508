"""HoSZp on MI355X: error-bounded compression and homomorphic operations on the
compressed stream (Agarwal et al., arXiv 2408.11971), as gfx950 HIP kernels
behind the C ABI of ``include/hoszp.h``.

This module is argument marshalling only: torch supplies device memory and
streams, every step of compression, decompression and the homomorphic
operations runs in ``libhoszp.so``.  Importing works anywhere; the first call
that needs the library raises ``HoszpUnavailable`` if it has not been built
(``python -m paper_2408_11971_amd.build``) -- there is no CPU fallback.
"""
import ctypes
import os
import struct

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhoszp.so")

OK, ERR_ARG, ERR_NONFINITE, ERR_RANGE, ERR_FORMAT, ERR_MISMATCH, ERR_CAPACITY, ERR_DEVICE, \
    ERR_NOMEM, ERR_LIMIT, ERR_TIMEOUT = range(11)
NOALLOC_MAX_N = 1 << 28
DEFAULT_WAIT_LIMIT = 1 << 24
RESULT_BYTES = 64


class HoszpUnavailable(RuntimeError):
    pass


class HoszpError(RuntimeError):
    def __init__(self, code, where):
        msg = _lib().hoszp_strerror(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_uint32), ("reserved0", ctypes.c_uint32),
                ("out_bytes", ctypes.c_uint64), ("value", ctypes.c_double),
                ("count", ctypes.c_uint64), ("reserved", ctypes.c_uint64 * 4)]


class Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("block", ctypes.c_uint32), ("version", ctypes.c_uint32),
                ("eb", ctypes.c_double), ("nb", ctypes.c_uint64),
                ("payload_bytes", ctypes.c_uint64), ("total_bytes", ctypes.c_uint64)]


class Field(ctypes.Structure):
    _fields_ = [("d_x", ctypes.c_void_p), ("n", ctypes.c_uint64), ("eb", ctypes.c_double),
                ("block", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("d_out", ctypes.c_void_p), ("out_cap", ctypes.c_uint64)]


class FieldResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_uint32), ("block", ctypes.c_uint32),
                ("out_bytes", ctypes.c_uint64), ("mean", ctypes.c_double),
                ("variance", ctypes.c_double), ("reserved", ctypes.c_uint64 * 4)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("fields", ctypes.c_uint64), ("total_tiles", ctypes.c_uint64),
                ("raw_bytes", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
                ("grid", ctypes.c_uint32), ("threads", ctypes.c_uint32)]


BATCH_TUNE_GRID = 1

OP_MEAN, OP_VARIANCE, OP_NEGATE, OP_ADD, OP_MUL = range(5)
PATH_HOMOMORPHIC, PATH_TRADITIONAL = 0, 1
OPS = {"mean": OP_MEAN, "variance": OP_VARIANCE, "negate": OP_NEGATE, "add": OP_ADD,
       "mul": OP_MUL}


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint32), ("keep_outputs", ctypes.c_uint32),
                ("pool_bytes", ctypes.c_uint64), ("starve_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "admitted", "completed", "failed",
                                               "pool_bytes", "pool_peak", "queue_peak")]


def _np_dtypes():
    import numpy as np
    req = np.dtype([("op", "<u4"), ("path", "<u4"), ("d_a", "<u8"), ("a_bytes", "<u8"),
                    ("d_b", "<u8"), ("b_bytes", "<u8"), ("n", "<u8"), ("block", "<u4"),
                    ("reserved", "<u4"), ("eb", "<f8"), ("scalar", "<f8"), ("tag", "<u8")])
    cpl = np.dtype([("tag", "<u8"), ("code", "<i4"), ("op", "<u4"), ("value", "<f8"),
                    ("d_out", "<u8"), ("out_bytes", "<u8"), ("submit_s", "<f8"),
                    ("admit_s", "<f8"), ("done_s", "<f8")])
    return req, cpl

_LIB = None
_VP, _SZ, _U64, _U32, _DBL, _INT = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64,
                                    ctypes.c_uint32, ctypes.c_double, ctypes.c_int)
_SIGNATURES = {
    "hoszp_ctx_create": (_INT, [_INT, ctypes.POINTER(_VP)]),
    "hoszp_ctx_destroy": (_INT, [_VP]),
    "hoszp_set_wait_limit": (_INT, [_VP, _U32]),
    "hoszp_compress_bound": (_SZ, [_U64, _U32]),
    "hoszp_parse_header": (_INT, [_VP, _SZ, ctypes.POINTER(Info)]),
    "hoszp_status_code": (_INT, [_U32]),
    "hoszp_strerror": (ctypes.c_char_p, [_INT]),
    "hoszp_compress": (_INT, [_VP, _VP, _U64, _DBL, _U32, _VP, _SZ, ctypes.POINTER(_SZ), _VP]),
    "hoszp_compress_async": (_INT, [_VP, _VP, _U64, _DBL, _U32, _VP, _SZ, _VP, _VP]),
    "hoszp_decompress": (_INT, [_VP, _VP, _SZ, _VP, _U64, _VP]),
    "hoszp_decompress_async": (_INT, [_VP, _VP, _SZ, _VP, _U64, _VP, _VP]),
    "hoszp_negate": (_INT, [_VP, _VP, _SZ, _VP, _SZ, ctypes.POINTER(_SZ), _VP]),
    "hoszp_negate_async": (_INT, [_VP, _VP, _SZ, _VP, _SZ, _VP, _VP]),
    "hoszp_add": (_INT, [_VP, _VP, _SZ, _VP, _SZ, _VP, _SZ, ctypes.POINTER(_SZ), _VP]),
    "hoszp_add_async": (_INT, [_VP, _VP, _SZ, _VP, _SZ, _VP, _SZ, _VP, _VP]),
    "hoszp_mul": (_INT, [_VP, _VP, _SZ, _DBL, _VP, _SZ, ctypes.POINTER(_SZ), _VP]),
    "hoszp_mul_async": (_INT, [_VP, _VP, _SZ, _DBL, _VP, _SZ, _VP, _VP]),
    "hoszp_mul_bins": (_INT, [_DBL, _VP, _VP, _U64]),
    "hoszp_bin_range": (_INT, [_DBL, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "hoszp_sub": (_INT, [_VP, _VP, _SZ, _VP, _SZ, _VP, _SZ, ctypes.POINTER(_SZ), _VP]),
    "hoszp_sub_async": (_INT, [_VP, _VP, _SZ, _VP, _SZ, _VP, _SZ, _VP, _VP]),
    "hoszp_scalar_add": (_INT, [_VP, _VP, _SZ, _DBL, _VP, _SZ, ctypes.POINTER(_SZ), _VP]),
    "hoszp_scalar_add_async": (_INT, [_VP, _VP, _SZ, _DBL, _VP, _SZ, _VP, _VP]),
    "hoszp_scalar_sub": (_INT, [_VP, _VP, _SZ, _DBL, _VP, _SZ, ctypes.POINTER(_SZ), _VP]),
    "hoszp_scalar_sub_async": (_INT, [_VP, _VP, _SZ, _DBL, _VP, _SZ, _VP, _VP]),
    "hoszp_std": (_INT, [_VP, _VP, _SZ, ctypes.POINTER(_DBL), _VP]),
    "hoszp_hadamard": (_INT, [_VP, _VP, _SZ, _VP, _SZ, _VP, _SZ, ctypes.POINTER(_SZ), _VP]),
    "hoszp_hadamard_async": (_INT, [_VP, _VP, _SZ, _VP, _SZ, _VP, _SZ, _VP, _VP]),
    "hoszp_covariance": (_INT, [_VP, _VP, _SZ, _VP, _SZ, ctypes.POINTER(_DBL), _VP]),
    "hoszp_covariance_async": (_INT, [_VP, _VP, _SZ, _VP, _SZ, _VP, _VP]),
    "hoszp_block_means": (_INT, [_VP, _VP, _SZ, _VP, _U64, ctypes.POINTER(_U64), _VP]),
    "hoszp_block_means_async": (_INT, [_VP, _VP, _SZ, _VP, _U64, _VP, _VP]),
    "hoszp_mean": (_INT, [_VP, _VP, _SZ, ctypes.POINTER(_DBL), _VP]),
    "hoszp_mean_async": (_INT, [_VP, _VP, _SZ, _VP, _VP]),
    "hoszp_variance": (_INT, [_VP, _VP, _SZ, ctypes.POINTER(_DBL), _VP]),
    "hoszp_variance_async": (_INT, [_VP, _VP, _SZ, _VP, _VP]),
    "hoszp_f32_negate_async": (_INT, [_VP, _VP, _VP, _U64, _VP]),
    "hoszp_f32_add_async": (_INT, [_VP, _VP, _VP, _VP, _U64, _VP]),
    "hoszp_f32_mul_async": (_INT, [_VP, _VP, _DBL, _VP, _U64, _VP]),
    "hoszp_f32_sub_async": (_INT, [_VP, _VP, _VP, _VP, _U64, _VP]),
    "hoszp_f32_scalar_add_async": (_INT, [_VP, _VP, _DBL, _VP, _U64, _VP]),
    "hoszp_f32_hadamard_async": (_INT, [_VP, _VP, _VP, _VP, _U64, _VP]),
    "hoszp_f32_mean_async": (_INT, [_VP, _VP, _U64, _VP, _VP]),
    "hoszp_f32_variance_async": (_INT, [_VP, _VP, _U64, _VP, _VP]),
    "hoszp_result_wait": (_INT, [_VP, _VP, ctypes.POINTER(Result), _VP]),
    "hoszp_compress_noalloc": (_INT, [_VP, _U64, _DBL, _U32, _VP, _SZ, _VP, _VP]),
    "hoszp_batch_create": (_INT, [_VP, ctypes.POINTER(Field), _U64, _U32, _VP, ctypes.POINTER(_VP),
                                  ctypes.POINTER(_U64)]),
    "hoszp_batch_launch": (_INT, [_VP, _VP]),
    "hoszp_batch_results": (_INT, [_VP, ctypes.POINTER(FieldResult), _VP]),
    "hoszp_batch_device_results": (_VP, [_VP]),
    "hoszp_batch_info_get": (_INT, [_VP, ctypes.POINTER(BatchInfo)]),
    "hoszp_batch_destroy": (_INT, [_VP]),
    "hoszp_server_create": (_INT, [_INT, ctypes.POINTER(ServerConfig), ctypes.POINTER(_VP)]),
    "hoszp_server_submit": (_INT, [_VP, _VP]),
    "hoszp_server_poll": (_INT, [_VP, _VP, _U32, ctypes.POINTER(_U32)]),
    "hoszp_server_pending": (_U64, [_VP]),
    "hoszp_server_release": (_INT, [_VP, _VP]),
    "hoszp_server_replay": (_INT, [_VP, _VP, _VP, _U64, _VP, ctypes.POINTER(_DBL)]),
    "hoszp_server_stats_get": (_INT, [_VP, ctypes.POINTER(ServerStats)]),
    "hoszp_server_destroy": (_INT, [_VP]),
}


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise HoszpUnavailable(
                f"{LIB_PATH} is missing: build it with `python -m paper_2408_11971_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def exported_symbols():
    """Names of the C entry points this binding wraps (all must be exported)."""
    return sorted(_SIGNATURES)


def _check(rc, where):
    if rc != OK:
        raise HoszpError(rc, where)


# ---------------------------------------------------------------- host-only

def compress_bound(n: int, block: int = 32) -> int:
    return _lib().hoszp_compress_bound(n, block)


def parse_header(header: bytes) -> dict:
    buf = ctypes.create_string_buffer(bytes(header[:64]), 64)
    info = Info()
    _check(_lib().hoszp_parse_header(ctypes.cast(buf, _VP), len(header), ctypes.byref(info)),
           "parse_header")
    return {k: getattr(info, k) for k, _ in Info._fields_}


def status_code(mask: int) -> int:
    return _lib().hoszp_status_code(mask)


def bin_range(eb):
    """(lo, hi): the float32 inputs whose bin at error bound eb is in range
    (see hoszp_bin_range)."""
    lo, hi = ctypes.c_float(0.0), ctypes.c_float(0.0)
    _check(_lib().hoszp_bin_range(float(eb), ctypes.byref(lo), ctypes.byref(hi)), "bin_range")
    return lo.value, hi.value


def mul_bins(s: float, q):
    """floor(s q + 1/2) exactly for an int32 numpy array q, by the rounding
    function the scalar-multiplication kernel uses (host code, no device).
    Returns (code, results); out-of-range results are 0 with code ERR_RANGE."""
    import numpy as np

    q = np.ascontiguousarray(q, dtype=np.int32)
    out = np.empty_like(q)
    rc = _lib().hoszp_mul_bins(float(s), _VP(q.ctypes.data), _VP(out.ctypes.data), q.size)
    return rc, out


# ---------------------------------------------------------------- contexts

class Context:
    """A library context on one device (owns the kernels' scratch)."""

    def __init__(self, device: int = 0):
        self.device = device
        h = _VP()
        _check(_lib().hoszp_ctx_create(device, ctypes.byref(h)), "ctx_create")
        self.handle = h

    def set_wait_limit(self, polls: int):
        """Poll limit of this context's encoder look-back waits (0: give up at once)."""
        _check(_lib().hoszp_set_wait_limit(self.handle, int(polls)), "set_wait_limit")

    def close(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.hoszp_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_CTX = {}


def context(device=None) -> Context:
    import torch

    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _CTX:
        _CTX[dev] = Context(dev)
    return _CTX[dev]


def _stream(stream=None):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return _VP(s.cuda_stream)


def _ptr(t):
    return _VP(t.data_ptr())


def _nbytes(t):
    return t.numel() * t.element_size()


def new_result(device=None):
    """A device-resident result record for the *_async calls."""
    import torch

    return torch.zeros(RESULT_BYTES // 8, dtype=torch.int64, device=device or "cuda")


def read_result(res, ctx=None, stream=None) -> dict:
    """Wait for `stream` and return the record as a dict (status code decoded)."""
    ctx = ctx or context(res.device.index)
    r = Result()
    code = _lib().hoszp_result_wait(ctx.handle, _ptr(res), ctypes.byref(r), _stream(stream))
    return {"code": code, "status": r.status, "out_bytes": r.out_bytes, "value": r.value,
            "count": r.count}


def header_of(c) -> dict:
    """Parse the header of a device-resident stream (copies 64 bytes to host)."""
    return parse_header(bytes(c[:64].cpu().numpy().tobytes()))


def _out_stream(n, block, device):
    import torch

    cap = compress_bound(n, block)
    if cap == 0:
        raise HoszpError(ERR_ARG, "compress_bound")
    return torch.empty(cap, dtype=torch.uint8, device=device)


# ---------------------------------------------------------------- sync API

def compress(x, eb: float, block: int = 32, out=None, stream=None):
    """Compress a float32 CUDA tensor; returns the stream as a uint8 tensor
    (a view of `out` trimmed to the stream size)."""
    ctx = context(x.device.index)
    x = x.contiguous().view(-1)
    if out is None:
        out = _out_stream(x.numel(), block, x.device)
    nb = _SZ(0)
    _check(_lib().hoszp_compress(ctx.handle, _ptr(x), x.numel(), float(eb), block, _ptr(out),
                                 _nbytes(out), ctypes.byref(nb), _stream(stream)), "compress")
    return out[:nb.value]


def decompress(c, out=None, stream=None):
    import torch

    ctx = context(c.device.index)
    n = header_of(c)["n"]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=c.device)
    _check(_lib().hoszp_decompress(ctx.handle, _ptr(c), _nbytes(c), _ptr(out), out.numel(),
                                   _stream(stream)), "decompress")
    return out[:n]


def negate(c, out=None, stream=None):
    import torch

    ctx = context(c.device.index)
    if out is None:
        out = torch.empty_like(c)
    nb = _SZ(0)
    _check(_lib().hoszp_negate(ctx.handle, _ptr(c), _nbytes(c), _ptr(out), _nbytes(out),
                               ctypes.byref(nb), _stream(stream)), "negate")
    return out[:nb.value]


def add(a, b, out=None, stream=None):
    ctx = context(a.device.index)
    if out is None:
        h = header_of(a)
        out = _out_stream(h["n"], h["block"], a.device)
    nb = _SZ(0)
    _check(_lib().hoszp_add(ctx.handle, _ptr(a), _nbytes(a), _ptr(b), _nbytes(b), _ptr(out),
                            _nbytes(out), ctypes.byref(nb), _stream(stream)), "add")
    return out[:nb.value]


def mul(c, s: float, out=None, stream=None):
    ctx = context(c.device.index)
    if out is None:
        h = header_of(c)
        out = _out_stream(h["n"], h["block"], c.device)
    nb = _SZ(0)
    _check(_lib().hoszp_mul(ctx.handle, _ptr(c), _nbytes(c), float(s), _ptr(out), _nbytes(out),
                            ctypes.byref(nb), _stream(stream)), "mul")
    return out[:nb.value]


def sub(a, b, out=None, stream=None):
    """Element-wise subtraction a - b of two streams."""
    ctx = context(a.device.index)
    if out is None:
        h = header_of(a)
        out = _out_stream(h["n"], h["block"], a.device)
    nb = _SZ(0)
    _check(_lib().hoszp_sub(ctx.handle, _ptr(a), _nbytes(a), _ptr(b), _nbytes(b), _ptr(out),
                            _nbytes(out), ctypes.byref(nb), _stream(stream)), "sub")
    return out[:nb.value]


def _shift(fn, name, c, s, out, stream):
    import torch

    ctx = context(c.device.index)
    if out is None:
        out = torch.empty_like(c)
    nb = _SZ(0)
    _check(fn(ctx.handle, _ptr(c), _nbytes(c), float(s), _ptr(out), _nbytes(out),
              ctypes.byref(nb), _stream(stream)), name)
    return out[:nb.value]


def scalar_add(c, s: float, out=None, stream=None):
    """Add scalar s to every element (its Eq. 3 bin added to the outliers);
    out may be c itself."""
    return _shift(_lib().hoszp_scalar_add, "scalar_add", c, s, out, stream)


def scalar_sub(c, s: float, out=None, stream=None):
    return _shift(_lib().hoszp_scalar_sub, "scalar_sub", c, s, out, stream)


def hadamard(a, b, out=None, stream=None):
    """Element-wise product of two streams (same n, block size and eb)."""
    ctx = context(a.device.index)
    if out is None:
        h = header_of(a)
        out = _out_stream(h["n"], h["block"], a.device)
    nb = _SZ(0)
    _check(_lib().hoszp_hadamard(ctx.handle, _ptr(a), _nbytes(a), _ptr(b), _nbytes(b), _ptr(out),
                                 _nbytes(out), ctypes.byref(nb), _stream(stream)), "hadamard")
    return out[:nb.value]


def covariance(a, b, stream=None) -> float:
    ctx = context(a.device.index)
    v = _DBL(0.0)
    _check(_lib().hoszp_covariance(ctx.handle, _ptr(a), _nbytes(a), _ptr(b), _nbytes(b),
                                   ctypes.byref(v), _stream(stream)), "covariance")
    return v.value


def block_means(c, out=None, stream=None):
    """(float64 tensor of the per-block means, number of constant blocks)."""
    import torch

    ctx = context(c.device.index)
    h = header_of(c)
    if out is None:
        out = torch.empty(h["nb"], dtype=torch.float64, device=c.device)
    k = _U64(0)
    _check(_lib().hoszp_block_means(ctx.handle, _ptr(c), _nbytes(c), _ptr(out), out.numel(),
                                    ctypes.byref(k), _stream(stream)), "block_means")
    return out[:h["nb"]], k.value


def std(c, stream=None) -> float:
    ctx = context(c.device.index)
    v = _DBL(0.0)
    _check(_lib().hoszp_std(ctx.handle, _ptr(c), _nbytes(c), ctypes.byref(v), _stream(stream)),
           "std")
    return v.value


def mean(c, stream=None) -> float:
    ctx = context(c.device.index)
    v = _DBL(0.0)
    _check(_lib().hoszp_mean(ctx.handle, _ptr(c), _nbytes(c), ctypes.byref(v), _stream(stream)),
           "mean")
    return v.value


def variance(c, stream=None) -> float:
    ctx = context(c.device.index)
    v = _DBL(0.0)
    _check(_lib().hoszp_variance(ctx.handle, _ptr(c), _nbytes(c), ctypes.byref(v),
                                 _stream(stream)), "variance")
    return v.value


# ---------------------------------------------------------------- async API
# Enqueue only; outcomes land in a device result record (see new_result()).

def compress_async(x, eb, block, out, res, ctx=None, stream=None):
    ctx = ctx or context(x.device.index)
    _check(_lib().hoszp_compress_async(ctx.handle, _ptr(x), x.numel(), float(eb), block,
                                       _ptr(out), _nbytes(out), _ptr(res), _stream(stream)),
           "compress_async")


def compress_noalloc(x, eb, block, out, res, stream=None):
    """hoszp_compress_noalloc: compress float32 tensor x into `out` with no
    context and no device allocation (the library's fixed scratch array of
    the current device); the outcome lands in the device record `res`."""
    _check(_lib().hoszp_compress_noalloc(_ptr(x), x.numel(), float(eb), block, _ptr(out),
                                         _nbytes(out), _ptr(res), _stream(stream)),
           "compress_noalloc")


def decompress_async(c, out, res, ctx=None, stream=None, c_bytes=None):
    ctx = ctx or context(c.device.index)
    _check(_lib().hoszp_decompress_async(ctx.handle, _ptr(c), c_bytes or _nbytes(c), _ptr(out),
                                         out.numel(), _ptr(res), _stream(stream)),
           "decompress_async")


def negate_async(c, out, res, ctx=None, stream=None, c_bytes=None):
    ctx = ctx or context(c.device.index)
    _check(_lib().hoszp_negate_async(ctx.handle, _ptr(c), c_bytes or _nbytes(c), _ptr(out),
                                     _nbytes(out), _ptr(res), _stream(stream)), "negate_async")


def add_async(a, b, out, res, ctx=None, stream=None, a_bytes=None, b_bytes=None):
    ctx = ctx or context(a.device.index)
    _check(_lib().hoszp_add_async(ctx.handle, _ptr(a), a_bytes or _nbytes(a), _ptr(b),
                                  b_bytes or _nbytes(b), _ptr(out), _nbytes(out), _ptr(res),
                                  _stream(stream)), "add_async")


def mul_async(c, s, out, res, ctx=None, stream=None, c_bytes=None):
    ctx = ctx or context(c.device.index)
    _check(_lib().hoszp_mul_async(ctx.handle, _ptr(c), c_bytes or _nbytes(c), float(s), _ptr(out),
                                  _nbytes(out), _ptr(res), _stream(stream)), "mul_async")


def sub_async(a, b, out, res, ctx=None, stream=None, a_bytes=None, b_bytes=None):
    ctx = ctx or context(a.device.index)
    _check(_lib().hoszp_sub_async(ctx.handle, _ptr(a), a_bytes or _nbytes(a), _ptr(b),
                                  b_bytes or _nbytes(b), _ptr(out), _nbytes(out), _ptr(res),
                                  _stream(stream)), "sub_async")


def hadamard_async(a, b, out, res, ctx=None, stream=None, a_bytes=None, b_bytes=None):
    ctx = ctx or context(a.device.index)
    _check(_lib().hoszp_hadamard_async(ctx.handle, _ptr(a), a_bytes or _nbytes(a), _ptr(b),
                                       b_bytes or _nbytes(b), _ptr(out), _nbytes(out), _ptr(res),
                                       _stream(stream)), "hadamard_async")


def covariance_async(a, b, res, ctx=None, stream=None, a_bytes=None, b_bytes=None):
    ctx = ctx or context(a.device.index)
    _check(_lib().hoszp_covariance_async(ctx.handle, _ptr(a), a_bytes or _nbytes(a), _ptr(b),
                                         b_bytes or _nbytes(b), _ptr(res), _stream(stream)),
           "covariance_async")


def scalar_add_async(c, s, out, res, ctx=None, stream=None, c_bytes=None):
    ctx = ctx or context(c.device.index)
    _check(_lib().hoszp_scalar_add_async(ctx.handle, _ptr(c), c_bytes or _nbytes(c), float(s),
                                         _ptr(out), _nbytes(out), _ptr(res), _stream(stream)),
           "scalar_add_async")


def scalar_sub_async(c, s, out, res, ctx=None, stream=None, c_bytes=None):
    ctx = ctx or context(c.device.index)
    _check(_lib().hoszp_scalar_sub_async(ctx.handle, _ptr(c), c_bytes or _nbytes(c), float(s),
                                         _ptr(out), _nbytes(out), _ptr(res), _stream(stream)),
           "scalar_sub_async")


def block_means_async(c, out, res, ctx=None, stream=None, c_bytes=None):
    ctx = ctx or context(c.device.index)
    _check(_lib().hoszp_block_means_async(ctx.handle, _ptr(c), c_bytes or _nbytes(c), _ptr(out),
                                          out.numel(), _ptr(res), _stream(stream)),
           "block_means_async")


def mean_async(c, res, ctx=None, stream=None, c_bytes=None):
    ctx = ctx or context(c.device.index)
    _check(_lib().hoszp_mean_async(ctx.handle, _ptr(c), c_bytes or _nbytes(c), _ptr(res),
                                   _stream(stream)), "mean_async")


def variance_async(c, res, ctx=None, stream=None, c_bytes=None):
    ctx = ctx or context(c.device.index)
    _check(_lib().hoszp_variance_async(ctx.handle, _ptr(c), c_bytes or _nbytes(c), _ptr(res),
                                       _stream(stream)), "variance_async")


def f32_negate_async(x, y, ctx=None, stream=None):
    ctx = ctx or context(x.device.index)
    _check(_lib().hoszp_f32_negate_async(ctx.handle, _ptr(x), _ptr(y), x.numel(), _stream(stream)),
           "f32_negate_async")


def f32_add_async(a, b, y, ctx=None, stream=None):
    ctx = ctx or context(a.device.index)
    _check(_lib().hoszp_f32_add_async(ctx.handle, _ptr(a), _ptr(b), _ptr(y), a.numel(),
                                      _stream(stream)), "f32_add_async")


def f32_mul_async(x, s, y, ctx=None, stream=None):
    ctx = ctx or context(x.device.index)
    _check(_lib().hoszp_f32_mul_async(ctx.handle, _ptr(x), float(s), _ptr(y), x.numel(),
                                      _stream(stream)), "f32_mul_async")


def f32_sub_async(a, b, y, ctx=None, stream=None):
    ctx = ctx or context(a.device.index)
    _check(_lib().hoszp_f32_sub_async(ctx.handle, _ptr(a), _ptr(b), _ptr(y), a.numel(),
                                      _stream(stream)), "f32_sub_async")


def f32_scalar_add_async(x, s, y, ctx=None, stream=None):
    ctx = ctx or context(x.device.index)
    _check(_lib().hoszp_f32_scalar_add_async(ctx.handle, _ptr(x), float(s), _ptr(y), x.numel(),
                                             _stream(stream)), "f32_scalar_add_async")


def f32_hadamard_async(a, b, y, ctx=None, stream=None):
    ctx = ctx or context(a.device.index)
    _check(_lib().hoszp_f32_hadamard_async(ctx.handle, _ptr(a), _ptr(b), _ptr(y), a.numel(),
                                           _stream(stream)), "f32_hadamard_async")


def f32_mean_async(x, res, ctx=None, stream=None):
    ctx = ctx or context(x.device.index)
    _check(_lib().hoszp_f32_mean_async(ctx.handle, _ptr(x), x.numel(), _ptr(res),
                                       _stream(stream)), "f32_mean_async")


def f32_variance_async(x, res, ctx=None, stream=None):
    ctx = ctx or context(x.device.index)
    _check(_lib().hoszp_f32_variance_async(ctx.handle, _ptr(x), x.numel(), _ptr(res),
                                           _stream(stream)), "f32_variance_async")


# ---------------------------------------------------------------- batches

def batch_out_cap(n: int, block: int = 0) -> int:
    """Output capacity a batch field needs (block 0: the autotuned case)."""
    if block:
        return compress_bound(n, block)
    return max(compress_bound(n, b) for b in (32, 64, 128))


class Batch:
    """A planned batch: every field compressed, with its mean and variance,
    in one captured persistent launch (see hoszp_batch_create).

    fields: sequence of (x, eb, block, out) with x a contiguous float32 CUDA
    tensor, block 32/64/128 or 0 (autotuned) and out a uint8 CUDA tensor of at
    least batch_out_cap(x.numel(), block) bytes.  The tensors must outlive the
    plan."""

    def __init__(self, fields, tune_grid=False, ctx=None, stream=None):
        if not fields:
            raise HoszpError(ERR_ARG, "batch_create")
        x0 = fields[0][0]
        self.ctx = ctx or context(x0.device.index)
        self.count = len(fields)
        self._keep = [(x, out) for x, _, _, out in fields]
        table = (Field * self.count)()
        for i, (x, eb, block, out) in enumerate(fields):
            table[i] = Field(x.data_ptr(), x.numel(), float(eb), int(block), 0, out.data_ptr(),
                             _nbytes(out))
        h = _VP()
        bad = _U64(0)
        rc = _lib().hoszp_batch_create(self.ctx.handle, table, self.count,
                                       BATCH_TUNE_GRID if tune_grid else 0, _stream(stream),
                                       ctypes.byref(h), ctypes.byref(bad))
        if rc != OK:
            raise HoszpError(rc, f"batch_create (field {bad.value})")
        self.handle = h

    def launch(self, stream=None):
        _check(_lib().hoszp_batch_launch(self.handle, _stream(stream)), "batch_launch")

    def results(self, stream=None):
        """Per-field dicts: code, status, block, out_bytes, mean, variance."""
        arr = (FieldResult * self.count)()
        _lib().hoszp_batch_results(self.handle, arr, _stream(stream))
        return [{"code": status_code(r.status), "status": r.status, "block": r.block,
                 "out_bytes": r.out_bytes, "mean": r.mean, "variance": r.variance} for r in arr]

    def info(self) -> dict:
        bi = BatchInfo()
        _check(_lib().hoszp_batch_info_get(self.handle, ctypes.byref(bi)), "batch_info")
        return {k: getattr(bi, k) for k, _ in BatchInfo._fields_ if k != "reserved"}

    def close(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.hoszp_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- serving

class Server:
    """Continuous-batching query server (see hoszp_server_create).

    Requests are numpy records of ``request_dtype`` (build them with
    ``make_requests``); completions come back as records of
    ``completion_dtype``."""

    def __init__(self, device=0, slots=8, pool_bytes=1 << 30, keep_outputs=False, starve_s=0.0):
        self.request_dtype, self.completion_dtype = _np_dtypes()
        cfg = ServerConfig(slots, 1 if keep_outputs else 0, pool_bytes, starve_s)
        h = _VP()
        _check(_lib().hoszp_server_create(device, ctypes.byref(cfg), ctypes.byref(h)),
               "server_create")
        self.handle = h

    def make_requests(self, count):
        import numpy as np
        return np.zeros(count, dtype=self.request_dtype)

    def submit(self, reqs):
        import numpy as np
        reqs = np.ascontiguousarray(reqs, dtype=self.request_dtype).reshape(-1)
        for i in range(reqs.size):
            _check(_lib().hoszp_server_submit(self.handle, reqs[i:i + 1].ctypes.data),
                   "server_submit")

    def poll(self, max_out=256):
        import numpy as np
        out = np.zeros(max_out, dtype=self.completion_dtype)
        n = _U32(0)
        _check(_lib().hoszp_server_poll(self.handle, out.ctypes.data, max_out, ctypes.byref(n)),
               "server_poll")
        return out[:n.value]

    def pending(self) -> int:
        return _lib().hoszp_server_pending(self.handle)

    def drain(self):
        """Poll until nothing is queued or running; returns every completion."""
        import numpy as np
        got = []
        while True:
            c = self.poll()
            if c.size:
                got.append(c)
            elif self.pending() == 0:
                break
        return np.concatenate(got) if got else np.zeros(0, dtype=self.completion_dtype)

    def replay(self, reqs, arrival_s):
        """Open-loop replay; returns (completions in request order, start time)."""
        import numpy as np
        reqs = np.ascontiguousarray(reqs, dtype=self.request_dtype).reshape(-1)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64).reshape(-1)
        out = np.zeros(reqs.size, dtype=self.completion_dtype)
        start = _DBL(0.0)
        _check(_lib().hoszp_server_replay(self.handle, reqs.ctypes.data, arr.ctypes.data, reqs.size,
                                          out.ctypes.data, ctypes.byref(start)), "server_replay")
        return out, start.value

    def release(self, d_out):
        _check(_lib().hoszp_server_release(self.handle, _VP(int(d_out))), "server_release")

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib().hoszp_server_stats_get(self.handle, ctypes.byref(st)), "server_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None) and _LIB is not None:
            _LIB.hoszp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fill_request(rec, op, a, b=None, scalar=0.0, path=PATH_HOMOMORPHIC, tag=0, info=None):
    """Fill one request record for stream tensor `a` (and `b` for add);
    `info` is a parsed header of `a` (read from the device when omitted)."""
    h = info or header_of(a)
    rec["op"] = OPS[op] if isinstance(op, str) else op
    rec["path"] = path
    rec["d_a"] = a.data_ptr()
    rec["a_bytes"] = h["total_bytes"]
    if b is not None:
        rec["d_b"] = b.data_ptr()
        rec["b_bytes"] = h["total_bytes"] if b is a else header_of(b)["total_bytes"]
    rec["n"] = h["n"]
    rec["block"] = h["block"]
    rec["eb"] = h["eb"]
    rec["scalar"] = scalar
    rec["tag"] = tag


def result_struct_size() -> int:
    return ctypes.sizeof(Result)

