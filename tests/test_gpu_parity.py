"""Parity of the gfx950 library (through the C ABI) with the CPU oracle.

Streams and quantized values must be byte-identical, mean and variance equal
to 1e-12 relative (they are computed from exact integer sums on both sides
and are expected to be bit-identical).  Sizes span several 8192-slot tiles
with ragged tails, every block size, and the degenerate cases of the method
(constant blocks, single elements, partial blocks, extreme widths and bins).
"""
import math

import numpy as np
import pytest

import synth
from oracle import ref

torch = pytest.importorskip("torch")
import paper_2408_11971_amd as hz  # noqa: E402

pytestmark = pytest.mark.gpu

BLOCKS = [32, 64, 128, 256]
REL = 1e-12


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def gpu(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gaussian(n, seed, scale=1.0):
    return np.random.default_rng(seed).normal(0.0, scale, n).astype(np.float32)


def close(a, b, rel=REL):
    return a == b or abs(a - b) <= rel * max(abs(a), abs(b))


def check_all_ops(x, y, eb, L, dev, scalars=(3.14, -0.37)):
    """compress/decompress/mean/variance/negate/add/mul parity for one case."""
    xc = ref.compress(x, eb, L)
    gx = gpu(x, dev)
    c = hz.compress(gx, eb, L)
    got = host(c)
    assert got.size == xc.size
    assert np.array_equal(got, xc), f"compress differs (n={x.size}, L={L}, eb={eb})"
    assert np.array_equal(host(hz.decompress(c)), ref.decompress(xc))
    assert close(hz.mean(c), ref.mean(xc))
    assert close(hz.variance(c), ref.variance(xc))
    assert np.array_equal(host(hz.negate(c)), ref.negate(xc))
    if y is not None:
        yc = ref.compress(y, eb, L)
        cy = hz.compress(gpu(y, dev), eb, L)
        assert np.array_equal(host(cy), yc)
        assert np.array_equal(host(hz.add(c, cy)), ref.add(xc, yc))
    for s in scalars:
        assert np.array_equal(host(hz.mul(c, s)), ref.mul(xc, s)), f"mul by {s}"
    return c, xc


@pytest.mark.parametrize("L", BLOCKS)
@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 63, 100, 255, 256, 257, 1000])
def test_small_fields(dev, n, L):
    print(f"case small n={n} L={L}", flush=True)
    check_all_ops(gaussian(n, n), gaussian(n, n + 1), 0.01, L, dev)


@pytest.mark.parametrize("L", BLOCKS)
@pytest.mark.parametrize("n", [8191, 8192, 8193, 3 * 8192 + 77, (1 << 16) + 5, 200003])
def test_multi_tile_ragged(dev, n, L):
    print(f"case ragged n={n} L={L}", flush=True)
    x = synth.sinusoid_1d(n, seed=1)
    y = synth.sinusoid_1d(n, seed=2)
    check_all_ops(x, y, synth.rel_eb(x, 1e-3), L, dev)


@pytest.mark.parametrize("n", [64 * 4096 * 32, 64 * 4096 * 32 + 1])
def test_direct_chunk_boundary(dev, n):
    """Streams of up to 64 chunks of 64 wave tiles (2^23 values at 32 slots a
    segment) get their chunk offsets from the consumers' own scan, larger
    ones from the width pre-pass's scan: both sides of the boundary (and of
    it at every block size, as segments do not depend on L) match the
    oracle."""
    x = synth.sinusoid_1d(n, seed=5)
    y = synth.sinusoid_1d(n, seed=6)
    eb = synth.rel_eb(x, 1e-3)
    for L in (32, 256):
        print(f"case direct-chunk boundary n={n} L={L}", flush=True)
        check_all_ops(x, y, eb, L, dev, scalars=(3.14,))


@pytest.mark.parametrize("rel", [1e-2, 1e-3, 1e-4])
def test_config_1d_full(dev, rel):
    """2^20-element sum of 8 sinusoids plus noise, block 32."""
    x = synth.sinusoid_1d(1 << 20, seed=1)
    y = synth.sinusoid_1d(1 << 20, seed=2)
    check_all_ops(x, y, synth.rel_eb(x, rel), 32, dev)


@pytest.mark.parametrize("L", BLOCKS)
def test_wide_fields(dev, L):
    """Tiny bound: widths up to 30 bits (the 128-bit variance path)."""
    x = gaussian(50000, 7)
    y = gaussian(50000, 8)
    c, xc = check_all_ops(x, y, 1e-8, L, dev, scalars=(0.5, -1.0))
    widths = xc[64:64 + ref.info(xc)["n"] // L]
    assert widths.max() >= 27


@pytest.mark.parametrize("L", BLOCKS)
def test_extreme_bins(dev, L):
    """Bins near +-2^30 and deltas near 2^31: exact-range paths."""
    rng = np.random.default_rng(11)
    x = rng.uniform(-2.0**30, 2.0**30, 20000).astype(np.float32)
    check_all_ops(x, None, 0.5, L, dev, scalars=(1.0, -1.0, 0.75))


@pytest.mark.parametrize("L", BLOCKS)
def test_constant_and_zero_fields(dev, L):
    for x in (np.zeros(30000, np.float32), np.full(30000, 3.0, np.float32)):
        c, xc = check_all_ops(x, x, 0.25, L, dev)
        assert ref.info(xc)["payload_bytes"] == 0


@pytest.mark.parametrize("L", BLOCKS)
def test_climate_like_steps(dev, L):
    steps = list(synth.climate_steps(2, 180, 360))
    eb = synth.rel_eb(steps[0], 1e-4)
    check_all_ops(steps[0], steps[1], eb, L, dev, scalars=(1.7320508, -0.5))


def test_grf_3d_small(dev):
    x = synth.grf_3d(48, seed=3)
    y = synth.grf_3d(48, seed=4)
    for rel in (1e-2, 1e-4):
        check_all_ops(x.ravel(), y.ravel(), synth.rel_eb(x, rel), 32, dev)


def test_add_negated_cancels(dev):
    x = synth.sinusoid_1d(100000, 3)
    c = hz.compress(gpu(x, dev), 1e-3, 32)
    z = host(hz.add(c, hz.negate(c)))
    info = ref.info(z)
    assert info["payload_bytes"] == 0
    assert np.all(ref.decode_bins(z) == 0)


def test_negate_in_place(dev):
    x = gaussian(70000, 5)
    xc = ref.compress(x, 0.01, 64)
    c = gpu(xc, dev)
    out = hz.negate(c, out=c)
    assert out.data_ptr() == c.data_ptr()
    assert np.array_equal(host(c), ref.negate(xc))


def test_repeatable_across_calls(dev):
    """Look-back generations change every call; results must not."""
    x = synth.sinusoid_1d(300000, 9)
    gx = gpu(x, dev)
    first = host(hz.compress(gx, 1e-3, 32))
    for _ in range(20):
        assert np.array_equal(host(hz.compress(gx, 1e-3, 32)), first)
    c = gpu(first, dev)
    means = {hz.mean(c) for _ in range(10)}
    assert len(means) == 1


# ------------------------------------------------------------------ errors

def err_of(fn, *a, **k):
    with pytest.raises(hz.HoszpError) as e:
        fn(*a, **k)
    return e.value.code


def test_nonfinite_and_range_errors(dev):
    for bad in (np.nan, np.inf, -np.inf):
        x = gaussian(20000, 1)
        x[12345] = bad
        assert err_of(hz.compress, gpu(x, dev), 0.01, 32) == hz.ERR_NONFINITE
    x = gaussian(20000, 1)
    x[777] = 1e6
    assert err_of(hz.compress, gpu(x, dev), 1e-4, 32) == hz.ERR_RANGE
    x[778] = np.nan
    assert err_of(hz.compress, gpu(x, dev), 1e-4, 32) == hz.ERR_NONFINITE


def test_bad_arguments(dev):
    x = gpu(gaussian(100, 1), dev)
    for eb in (0.0, -1.0, math.inf, math.nan):
        assert err_of(hz.compress, x, eb, 32) == hz.ERR_ARG
    assert err_of(hz.compress, x, 0.1, 48) == hz.ERR_ARG
    small = torch.empty(hz.compress_bound(100, 32) - 1, dtype=torch.uint8, device=dev)
    assert err_of(hz.compress, x, 0.1, 32, out=small) == hz.ERR_CAPACITY
    c = hz.compress(x, 0.1, 32)
    assert err_of(hz.mul, c, math.inf) == hz.ERR_ARG


def test_output_overlapping_an_input_is_rejected(dev):
    """add and mul refuse an output range that shares bytes with an input
    (a tile's output words could overwrite input words later tiles read);
    nothing is launched, so the buffer is left as it was."""
    x = synth.sinusoid_1d(40000, 3)
    xc = ref.compress(x, 1e-3, 32)
    cap = hz.compress_bound(x.size, 32)
    buf = torch.zeros(2 * cap + 4096, dtype=torch.uint8, device=dev)
    buf[:xc.size] = gpu(xc, dev)
    a = buf[:xc.size]
    before = host(buf).copy()
    for off in (0, 16, xc.size - 16):
        out = buf[off:off + cap]
        assert err_of(hz.mul, a, 2.0, out=out) == hz.ERR_ARG
        assert err_of(hz.add, a, a, out=out) == hz.ERR_ARG
    other = gpu(xc, dev)
    assert err_of(hz.add, other, a, out=buf[64:64 + cap]) == hz.ERR_ARG
    assert np.array_equal(host(buf), before)
    # disjoint ranges of the same allocation are fine
    start = (xc.size + 15) // 16 * 16
    out = buf[start:start + cap]
    assert np.array_equal(host(hz.mul(a, 2.0, out=out)), ref.mul(xc, 2.0))
    assert np.array_equal(host(hz.add(a, other, out=out)), ref.add(xc, xc))


def corruptions(c):
    out = []
    for off, val in [(0, ord("X")), (4, 2), (8, 48), (32, int(c[32]) + 1), (64, 33),
                     (64, (int(c[64]) + 1) % 33)]:
        d = c.copy()
        d[off] = val
        out.append(d)
    out.append(c[:-4].copy())
    return out


def test_malformed_streams(dev):
    x = synth.sinusoid_1d(50000, 4)
    c = ref.compress(x, 1e-3, 32)
    for bad in corruptions(c):
        g = gpu(bad, dev)
        assert err_of(hz.mean, g) == hz.ERR_FORMAT
        assert err_of(hz.variance, g) == hz.ERR_FORMAT
        assert err_of(hz.negate, g, out=torch.empty(c.size + 64, dtype=torch.uint8, device=dev)) \
            == hz.ERR_FORMAT
        out = torch.empty(hz.compress_bound(50000, 32), dtype=torch.uint8, device=dev)
        assert err_of(hz.mul, g, 2.0, out=out) == hz.ERR_FORMAT
        assert err_of(hz.add, g, gpu(c, dev), out=out) == hz.ERR_FORMAT
        # the second operand is indexed by the other half of the same launch
        assert err_of(hz.add, gpu(c, dev), g, out=out) == hz.ERR_FORMAT
        assert err_of(hz.hadamard, gpu(c, dev), g, out=out) == hz.ERR_FORMAT
        assert err_of(hz.covariance, gpu(c, dev), g) == hz.ERR_FORMAT
        xo = torch.empty(50000, dtype=torch.float32, device=dev)
        assert err_of(hz.decompress, g, out=xo) == hz.ERR_FORMAT


def test_width_above_32_is_format_error(dev):
    # n = 1000, L = 32: the width section is bytes 64..95; widths 16..19
    # become 0, 0, 0, 128
    c = ref.compress(gaussian(1000, 3), 0.01, 32)
    c[80:84] = np.array([0x80000000], dtype=np.uint32).view(np.uint8)
    g = gpu(c, dev)
    assert err_of(hz.mean, g) == hz.ERR_FORMAT
    assert err_of(hz.variance, g) == hz.ERR_FORMAT


def outlier_offset(n, L):
    nb = (n + L - 1) // L
    return ((64 + nb + 15) // 16) * 16


def test_outlier_edges(dev):
    """Blocks whose outlier and width let a bin reach the int32 limits take
    the decoders' exact per-slot check: bins at +-(2^31 - 1) decode like the
    oracle; an outlier raised so that one bin passes 2^31 - 1, or an outlier
    of -2^31, is a format error (for the oracle too)."""
    K = 2**31 - 1
    rng = np.random.default_rng(12)
    n = 5000
    q = rng.integers(-3, 4, n).astype(np.int64)
    ramp = np.array([0, 1, 2, 3, 4, 5, 5, 4, 3, 2, 1, 0] * 11)[:64]
    q[:64] = K - 5 + ramp                   # block 0 starts at K - 5 and touches K
    q[64:128] = -K + np.abs(q[64:128])      # blocks near -K, touching it
    q[100] = -K
    q = q.astype(np.int32)
    for L in (32, 64):
        c = ref.encode_bins(q, 0.5, L)
        g = gpu(c, dev)
        print(f"case outlier edges L={L}", flush=True)
        assert hz.mean(g) == ref.mean(c)
        assert hz.variance(g) == ref.variance(c)
        assert np.array_equal(host(hz.decompress(g)), ref.decompress(c))
        o = outlier_offset(n, L)
        up = c.copy()
        up[o:o + 4] = np.array([K - 4], dtype=np.int32).view(np.uint8)  # the bin K becomes K + 1
        low = c.copy()
        low[o:o + 4] = np.array([-2**31], dtype=np.int32).view(np.uint8)
        for bad in (up, low):
            with pytest.raises(ref.RefError):
                ref.mean(bad)
            gb = gpu(bad, dev)
            assert err_of(hz.mean, gb) == hz.ERR_FORMAT
            assert err_of(hz.variance, gb) == hz.ERR_FORMAT
            assert err_of(hz.decompress, gb) == hz.ERR_FORMAT


def test_add_mismatch_capacity_and_range(dev):
    a = gpu(ref.compress(gaussian(1000, 1), 0.01, 32), dev)
    for other in (ref.compress(gaussian(1001, 1), 0.01, 32), ref.compress(gaussian(1000, 1), 0.01, 64),
                  ref.compress(gaussian(1000, 1), 0.01 * (1 + 2**-52), 32)):
        assert err_of(hz.add, a, gpu(other, dev)) == hz.ERR_MISMATCH
    small = torch.empty(hz.compress_bound(1000, 32) - 1, dtype=torch.uint8, device=dev)
    assert err_of(hz.add, a, a, out=small) == hz.ERR_CAPACITY
    assert err_of(hz.mul, a, 2.0, out=small) == hz.ERR_CAPACITY
    big = gpu(ref.encode_bins(np.full(100, 2**31 - 1, np.int32), 0.5, 32), dev)
    assert err_of(hz.add, big, big) == hz.ERR_RANGE
    assert err_of(hz.mul, big, 1.5) == hz.ERR_RANGE
    assert err_of(hz.mul, big, 2.0**60) == hz.ERR_RANGE


# ------------------------------------------------- decompress-then-compute

def test_float32_workflow_ops(dev):
    x = synth.sinusoid_1d(100003, 1)
    y = synth.sinusoid_1d(100003, 2)
    gx, gy = gpu(x, dev), gpu(y, dev)
    out = torch.empty_like(gx)
    hz.f32_negate_async(gx, out)
    assert np.array_equal(host(out), -x)
    hz.f32_add_async(gx, gy, out)
    assert np.array_equal(host(out), x + y)
    hz.f32_mul_async(gx, 1.7, out)
    assert np.array_equal(host(out), (x.astype(np.float64) * 1.7).astype(np.float32))
    hz.f32_sub_async(gx, gy, out)
    assert np.array_equal(host(out), x - y)
    hz.f32_scalar_add_async(gx, -0.37, out)
    assert np.array_equal(host(out), (x.astype(np.float64) - 0.37).astype(np.float32))
    hz.f32_hadamard_async(gx, gy, out)
    assert np.array_equal(host(out), x * y)
    res = hz.new_result(dev)
    hz.f32_mean_async(gx, res)
    m = hz.read_result(res)["value"]
    assert close(m, float(np.mean(x.astype(np.float64))), 1e-12)
    hz.f32_variance_async(gx, res)
    v = hz.read_result(res)["value"]
    assert close(v, float(np.var(x.astype(np.float64))), 1e-12)


def test_traditional_equals_homomorphic(dev):
    """Theorem 1 on the GPU: decompress + float32 op + compress gives the
    same stream as the homomorphic op (negate, add), bins far below 2^24."""
    x = synth.sinusoid_1d(1 << 18, 1)
    y = synth.sinusoid_1d(1 << 18, 2)
    eb = synth.rel_eb(x, 1e-3)
    cx = hz.compress(gpu(x, dev), eb, 32)
    cy = hz.compress(gpu(y, dev), eb, 32)
    dx, dy = hz.decompress(cx), hz.decompress(cy)
    t = torch.empty_like(dx)
    hz.f32_add_async(dx, dy, t)
    assert np.array_equal(host(hz.compress(t, eb, 32)), host(hz.add(cx, cy)))
    hz.f32_negate_async(dx, t)
    trad = host(hz.compress(t, eb, 32))
    assert np.array_equal(ref.decode_bins(trad), ref.decode_bins(host(hz.negate(cx))))
    hz.f32_sub_async(dx, dy, t)
    assert np.array_equal(host(hz.compress(t, eb, 32)), host(hz.sub(cx, cy)))


# ------------------------------------------------------------ async chain

def test_async_chain_matches_sync(dev):
    x = synth.sinusoid_1d(1 << 18, 5)
    gx = gpu(x, dev)
    eb = synth.rel_eb(x, 1e-3)
    cap = hz.compress_bound(x.size, 32)
    c = torch.empty(cap, dtype=torch.uint8, device=dev)
    z = torch.empty(cap, dtype=torch.uint8, device=dev)
    r1, r2, r3 = hz.new_result(dev), hz.new_result(dev), hz.new_result(dev)
    hz.compress_async(gx, eb, 32, c, r1)
    hz.mean_async(c, r2)
    hz.add_async(c, c, z, r3)
    a1, a2, a3 = hz.read_result(r1), hz.read_result(r2), hz.read_result(r3)
    assert a1["code"] == a2["code"] == a3["code"] == 0
    xc = ref.compress(x, eb, 32)
    assert a1["out_bytes"] == xc.size
    assert np.array_equal(host(c)[:xc.size], xc)
    assert a2["value"] == ref.mean(xc)
    zc = ref.add(xc, xc)
    assert a3["out_bytes"] == zc.size
    assert np.array_equal(host(z)[:zc.size], zc)


@pytest.mark.parametrize("s", [0.5, 1.5, -2.5, 1.0 / 3.0, 0.1, 3 * 2.0**-20, 1e-5, 123.456,
                               -0.7499999999999999, 2.0**51 * 1.5, 2.0**-101, 1.1, 0.55,
                               0.49999999999999994, 0.24999999999999997,
                               -0.49999999999999994])
def test_mul_rounding_ties(dev, s):
    """Integer-valued fields at eb = 1/2 (bins equal the values): scalars that
    put s q exactly on, or one ulp beside, half-integers must round like the
    exact definition."""
    print(f"case mul ties s={s}", flush=True)
    rng = np.random.default_rng(17)
    q = rng.integers(-200000, 200001, 40000)
    q[::7] = rng.integers(-3, 4, q[::7].size)
    q[5::11] = rng.choice([465, -465, 930, -930, 150000, -150000, 1, 2, 4], q[5::11].size)
    x = q.astype(np.float32)
    xc = ref.compress(x, 0.5, 32)
    c = hz.compress(gpu(x, dev), 0.5, 32)
    assert np.array_equal(host(c), xc)
    try:
        want = ref.mul(xc, s)
    except ref.RefError as e:
        with pytest.raises(hz.HoszpError) as g:
            hz.mul(c, s)
        assert g.value.code == e.code
        return
    assert np.array_equal(host(hz.mul(c, s)), want), f"mul by {s!r}"


def test_mul_exact_rounding_classes(dev):
    """Scalar multiplication on the GPU on every near-tie class of
    floor(s q + 1/2) (s q within a few ulps of a half-integer, including
    y = 1/2 - 2^-54 and y = 2^k - 1/2 + ulp(y)): the stream equals the
    oracle's, and the decoded bins equal exact rational arithmetic."""
    from mul_cases import exact_mul_bins, tie_cases

    rng = np.random.default_rng(31)
    cases = tie_cases()
    print(f"case mul tie classes: {len(cases)} scalars", flush=True)
    for i, (s, q) in enumerate(cases):
        fill = rng.integers(-50, 51, 97).astype(np.int32)
        field = np.concatenate([fill[: i % 40], q, fill, q[::-1]]).astype(np.int32)
        xc = ref.encode_bins(field, 0.5, 32)
        c = gpu(xc, dev)
        want = exact_mul_bins(s, field)
        if any(w is None for w in want):
            with pytest.raises(hz.HoszpError) as g:
                hz.mul(c, s)
            assert g.value.code == hz.ERR_RANGE, s
            continue
        got = host(hz.mul(c, s))
        assert np.array_equal(got, ref.mul(xc, s)), f"mul stream differs for s={s!r}"
        assert np.array_equal(ref.decode_bins(got).astype(np.int64),
                              np.array(want, dtype=np.int64)), f"mul bins differ for s={s!r}"


def wave_width_field(L, seed):
    """Float field whose waves (64 consecutive segments of 32 slots) have
    widest block widths 1, 2, ..., 23 in turn (twice over), the other
    blocks of each wave narrower.  Slots alternate between a block base and
    base + m_j, so every delta is +-m_j and a block's width is the bit length
    of its largest m_j; all bins stay below 2^24 in magnitude, so with
    eps = 1/2 each value is its own (exact) bin."""
    rng = np.random.default_rng(seed)
    blocks_per_wave = 64 // (L // 32)
    out = []
    for wave in range(2 * 23):
        W = 1 + wave % 23
        for b in range(blocks_per_wave):
            wb = W if b == (wave * 7) % blocks_per_wave else int(rng.integers(0, W + 1))
            m = rng.integers(0, 1 << wb, L)
            m[int(rng.integers(1, L))] = (1 << wb) - 1
            base = int(rng.integers(-(1 << 22), 1 << 22))
            q = base + np.where(np.arange(L) % 2 == 1, m, 0)
            out.append(q)
    q = np.concatenate(out)
    x = q.astype(np.float32)
    assert np.array_equal(x.astype(np.int64), q)
    return x


def wave_max_widths(c, L):
    """Widest block width of every wave of a stream (oracle stream)."""
    nb = ref.info(c)["n"] // L
    w = c[64:64 + nb].astype(np.int64)
    per = 64 // (L // 32)
    return [int(w[k:k + per].max()) for k in range(0, nb, per)]


@pytest.mark.parametrize("L", BLOCKS)
def test_every_wave_max_width(dev, L):
    """Encoders pack 1 to 4 fields per step depending on the widest width in
    a wave (64 segments); this field gives every wave-widest width 1..23, so
    every step size and every last, shorter group is exercised."""
    x = wave_width_field(L, 100 + L)
    xc = ref.compress(x, 0.5, L)
    assert wave_max_widths(xc, L) == [1 + k % 23 for k in range(2 * 23)]
    print(f"case wave widths L={L} n={x.size}", flush=True)
    check_all_ops(x, x[::-1].copy(), 0.5, L, dev, scalars=(1.0, -0.5))


@pytest.mark.parametrize("eb", [1e-3, 0.5, 7.3e-6])
def test_range_interval_ends(dev, eb):
    """Inputs at both ends of the accepted interval (bins +-(2^31-1) or the
    nearest) compress exactly like the oracle; the next float beyond either
    end is RANGE.  The kernels test ranges against a bound derived from this
    interval, so its ends are where a mistake would show."""
    lo, hi = hz.bin_range(eb)
    x = gaussian(70000, 3, scale=100 * eb)
    for k, pos in enumerate((5, 40, 31, 32, 33, 1023, 32768, 65535, 69999)):
        x[pos] = hi if k % 2 == 0 else lo
    print(f"case range ends eb={eb} lo={lo} hi={hi}", flush=True)
    for L in BLOCKS:
        xc = ref.compress(x, eb, L)
        assert np.array_equal(host(hz.compress(gpu(x, dev), eb, L)), xc), L
    for beyond in (np.nextafter(np.float32(hi), np.float32(np.inf)),
                   np.nextafter(np.float32(lo), np.float32(-np.inf))):
        y = x.copy()
        y[40000] = beyond
        assert err_of(hz.compress, gpu(y, dev), eb, 32) == hz.ERR_RANGE
