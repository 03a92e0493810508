"""The allocation-free compression entry point (hoszp_compress_noalloc, for
callers that cannot allocate device memory) against the context-based
hoszp_compress_async on the same inputs: identical streams and result
records on two calls in a row (the second smaller, so leftovers of the first
call in the shared scratch array would show), both equal to the oracle; a
size above the stated maximum is refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import ref

torch = pytest.importorskip("torch")
import paper_2408_11971_amd as hz  # noqa: E402

pytestmark = pytest.mark.gpu


def both(x, eb, L, dev):
    gx = torch.from_numpy(x).to(dev)
    cap = hz.compress_bound(x.size, L)
    out_a = torch.full((cap,), 0xAB, dtype=torch.uint8, device=dev)
    out_b = torch.full((cap,), 0xCD, dtype=torch.uint8, device=dev)
    ra, rb = hz.new_result(dev), hz.new_result(dev)
    hz.compress_async(gx, eb, L, out_a, ra)
    hz.compress_noalloc(gx, eb, L, out_b, rb)
    a, b = hz.read_result(ra), hz.read_result(rb)
    return a, b, out_a, out_b


@pytest.mark.parametrize("L", [32, 128])
def test_noalloc_matches_compress_async(L):
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    dev = torch.device("cuda:0")
    big = synth.sinusoid_1d(3_000_001, seed=11)          # 92 encoder tiles, ragged tail
    small = synth.sinusoid_1d(70_001, seed=12)           # 3 tiles: the first call's
    for x in (big, small):                               # later tiles must not leak in
        print(f"case noalloc n={x.size} L={L}", flush=True)
        eb = synth.rel_eb(x, 1e-3)
        a, b, out_a, out_b = both(x, eb, L, dev)
        assert a["code"] == b["code"] == hz.OK
        assert a["out_bytes"] == b["out_bytes"]
        n = b["out_bytes"]
        got = out_b[:n].cpu().numpy()
        assert np.array_equal(got, out_a[:n].cpu().numpy())
        assert np.array_equal(got, ref.compress(x, eb, L))


def test_noalloc_reports_device_errors_and_recovers():
    dev = torch.device("cuda:0")
    x = synth.sinusoid_1d(100_000, seed=13)
    eb = synth.rel_eb(x, 1e-3)
    bad = x.copy()
    bad[54321] = np.nan
    a, b, _, _ = both(bad, eb, 32, dev)
    assert a["code"] == b["code"] == hz.ERR_NONFINITE
    a, b, out_a, out_b = both(x, eb, 32, dev)  # the next call starts clean
    assert a["code"] == b["code"] == hz.OK
    n = b["out_bytes"]
    assert np.array_equal(out_b[:n].cpu().numpy(), ref.compress(x, eb, 32))


def test_noalloc_limit_is_refused_on_the_host():
    dev = torch.device("cuda:0")
    x = torch.zeros(1024, dtype=torch.float32, device=dev)
    out = torch.zeros(4096, dtype=torch.uint8, device=dev)
    res = hz.new_result(dev)
    lib = hz._lib()
    rc = lib.hoszp_compress_noalloc(ctypes.c_void_p(x.data_ptr()), hz.NOALLOC_MAX_N + 1, 0.1, 32,
                                    ctypes.c_void_p(out.data_ptr()), 1 << 62,
                                    ctypes.c_void_p(res.data_ptr()), None)
    assert rc == hz.ERR_LIMIT
    assert "2^28" in lib.hoszp_strerror(hz.ERR_LIMIT).decode()
    # too small an output is CAPACITY, a bad block size ARG (nothing launched)
    with pytest.raises(hz.HoszpError) as e:
        hz.compress_noalloc(x, 0.1, 32, out[:100], res)
    assert e.value.code == hz.ERR_CAPACITY
    with pytest.raises(hz.HoszpError) as e:
        hz.compress_noalloc(x, 0.1, 48, out, res)
    assert e.value.code == hz.ERR_ARG
    torch.cuda.synchronize()
    assert int(res.cpu().view(torch.uint8)[:4].view(torch.int32)[0]) == 0
