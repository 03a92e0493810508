"""GPU parity (through the C ABI) of the remaining Table II operations with
the CPU oracle: scalar addition and subtraction (Sec. V-A, workflow 1),
element-wise subtraction and the Hadamard product (Sec. V-C), standard
deviation and block-wise means with constant-block counts (Sec. V-B),
covariance (Sec. V-D).

Streams must be byte-identical to the oracle's, doubles equal to 1e-12
relative; sizes span several 32768-slot encoder tiles with ragged tails and
every block size; the degenerate cases are constant blocks, single elements,
in-place calls, non-canonical (negated) inputs, and bins at the edge of the
range where the kernel's exact slow path decides.
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
BIN_MAX = 2**31 - 1


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def gpu(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def err_of(fn, *a, **k):
    with pytest.raises(hz.HoszpError) as e:
        fn(*a, **k)
    return e.value.code


def walk(n, seed, scale=1.0):
    return np.cumsum(np.random.default_rng(seed).normal(0.0, scale, n)).astype(np.float32)


CASES = [(1, 32), (31, 64), (5000, 32), (70001, 64), (262147, 128), (1000003, 256),
         (2500000, 32)]


@pytest.mark.parametrize("n,L", CASES)
def test_scalar_add_sub(dev, n, L):
    print(f"case scalar add/sub n={n} L={L}", flush=True)
    x = walk(n, n % 97)
    x[n // 3:n // 3 + 5 * L] = 3.5          # constant blocks
    eb = synth.rel_eb(x, 1e-3)
    xc = ref.compress(x, eb, L)
    c = gpu(xc, dev)
    for s in (0.0, 2.75, -13.125, 1000.0 * eb, -eb, 1e-9, 123456.789):
        assert np.array_equal(host(hz.scalar_add(c, s)), ref.scalar_add(xc, s)), s
        assert np.array_equal(host(hz.scalar_sub(c, s)), ref.scalar_sub(xc, s)), s
    # in place, and on a negated (non-canonical) stream
    d = c.clone()
    hz.scalar_add(d, 7.5, out=d)
    assert np.array_equal(host(d), ref.scalar_add(xc, 7.5))
    hz.scalar_sub(d, 7.5, out=d)
    assert np.array_equal(host(d), xc)
    nc = ref.negate(xc)
    assert np.array_equal(host(hz.scalar_add(gpu(nc, dev), -4.0)), ref.scalar_add(nc, -4.0))


def test_scalar_shift_range_slow_path(dev):
    """Blocks whose outlier and width cannot rule out an out-of-range bin are
    decoded by the kernel; the decision must equal the oracle's."""
    for L in BLOCKS:
        print(f"case scalar shift range L={L}", flush=True)
        rng = np.random.default_rng(L)
        q = rng.integers(-1000, 1000, 40 * L).astype(np.int32)
        wide = np.zeros(4 * L, np.int32)        # widths 31/32, bins within +-2^30
        wide[1::2] = 1 << 30
        wide[2::4] = -(1 << 30)
        q[7 * L:11 * L] = wide
        c = ref.encode_bins(q, 0.5, L)           # eps 1/2: the scalar's bin is floor(s + 1/2)
        g = gpu(c, dev)
        for s in (2.0**29, -(2.0**29), 2.0**30 - 1001, -(2.0**30) + 1001):
            assert np.array_equal(host(hz.scalar_add(g, s)), ref.scalar_add(c, s)), s
            assert np.array_equal(host(hz.scalar_sub(g, s)), ref.scalar_sub(c, s)), s
        for s in (2.0**30, -(2.0**30) - 5, 2.0**31, 1e30):
            for fn, rf in ((hz.scalar_add, ref.scalar_add), (hz.scalar_sub, ref.scalar_sub)):
                with pytest.raises(ref.RefError) as e:
                    rf(c, s)
                assert err_of(fn, g, s) == e.value.code == hz.ERR_RANGE, s
        # bins at the edge of the range with narrow widths (fast path says no)
        top = np.full(3 * L + 7, BIN_MAX - 5, np.int32)
        top[::5] = BIN_MAX - 40
        ct = ref.encode_bins(top, 0.5, L)
        gt = gpu(ct, dev)
        assert np.array_equal(host(hz.scalar_add(gt, 5.0)), ref.scalar_add(ct, 5.0))
        assert err_of(hz.scalar_add, gt, 6.0) == hz.ERR_RANGE
        assert np.array_equal(host(hz.scalar_sub(gt, 2.0**31 - 100)),
                              ref.scalar_sub(ct, 2.0**31 - 100))


def test_scalar_shift_arguments(dev):
    x = walk(5000, 3)
    xc = ref.compress(x, 0.01, 32)
    c = gpu(xc, dev)
    for s in (math.nan, math.inf, -math.inf):
        assert err_of(hz.scalar_add, c, s) == hz.ERR_ARG
        assert err_of(hz.scalar_sub, c, s) == hz.ERR_ARG
    small = torch.empty(xc.size - 16, dtype=torch.uint8, device=dev)
    assert err_of(hz.scalar_add, c, 1.0, out=small) == hz.ERR_CAPACITY
    buf = torch.zeros(2 * xc.size + 64, dtype=torch.uint8, device=dev)
    buf[:xc.size] = c
    assert err_of(hz.scalar_add, buf[:xc.size], 1.0, out=buf[16:16 + xc.size]) == hz.ERR_ARG
    assert err_of(hz.negate, buf[:xc.size], out=buf[16:16 + xc.size]) == hz.ERR_ARG
    bad = xc.copy()
    bad[0] = ord("X")
    assert err_of(hz.scalar_add, gpu(bad, dev), 1.0) == hz.ERR_FORMAT


@pytest.mark.parametrize("n,L", CASES)
def test_elementwise_sub(dev, n, L):
    print(f"case sub n={n} L={L}", flush=True)
    x = walk(n, 11 + n % 13)
    y = walk(n, 12 + n % 17, scale=0.5)
    y[: min(n, 3 * L)] = x[: min(n, 3 * L)]    # equal leading blocks: zero differences
    eb = synth.rel_eb(x, 1e-3)
    xc, yc = ref.compress(x, eb, L), ref.compress(y, eb, L)
    a, b = gpu(xc, dev), gpu(yc, dev)
    assert np.array_equal(host(hz.sub(a, b)), ref.sub(xc, yc))
    assert np.array_equal(host(hz.sub(b, a)), ref.sub(yc, xc))
    assert not ref.decode_bins(host(hz.sub(a, a))).any()
    # A - B = A + (-B), also on the GPU
    assert np.array_equal(host(hz.sub(a, b)), host(hz.add(a, hz.negate(b))))


def test_sub_errors(dev):
    x = walk(3000, 5)
    eb = 0.01
    a = gpu(ref.compress(x, eb, 32), dev)
    for other in (ref.compress(x[:2999], eb, 32), ref.compress(x, eb, 64),
                  ref.compress(x, eb * (1 + 2**-52), 32)):
        assert err_of(hz.sub, a, gpu(other, dev)) == hz.ERR_MISMATCH
    hic = ref.encode_bins(np.full(100, BIN_MAX, np.int32), 0.5, 32)
    m1c = ref.encode_bins(np.full(100, -1, np.int32), 0.5, 32)
    p1c = ref.encode_bins(np.full(100, 1, np.int32), 0.5, 32)
    hi, m1, p1 = gpu(hic, dev), gpu(m1c, dev), gpu(p1c, dev)
    assert err_of(hz.sub, hi, m1) == hz.ERR_RANGE      # 2^31 - 1 + 1
    assert err_of(hz.sub, m1, hi) == hz.ERR_RANGE      # -1 - (2^31 - 1) = -2^31
    assert np.array_equal(host(hz.sub(p1, hi)), ref.sub(p1c, hic))  # -(2^31 - 1) + 2
    cap = hz.compress_bound(3000, 32)
    buf = torch.zeros(cap + 4096, dtype=torch.uint8, device=dev)
    xc = ref.compress(x, eb, 32)
    buf[:xc.size] = gpu(xc, dev)
    assert err_of(hz.sub, buf[:xc.size], a, out=buf[:cap]) == hz.ERR_ARG


@pytest.mark.parametrize("L", BLOCKS)
def test_std(dev, L):
    for n, seed in ((1, 1), (777, 2), (300001, 3)):
        x = walk(n, seed)
        eb = synth.rel_eb(x, 1e-4)
        xc = ref.compress(x, eb, L)
        want = ref.std(xc)
        got = hz.std(gpu(xc, dev))
        assert got == want or abs(got - want) <= 1e-12 * abs(want), (got, want)


# ------------------------------------------------ Hadamard and covariance

PAIR_CASES = [(1, 32), (33, 64), (5000, 32), (70001, 128), (300007, 256), (1500001, 32)]


@pytest.mark.parametrize("n,L", PAIR_CASES)
def test_hadamard(dev, n, L):
    print(f"case hadamard n={n} L={L}", flush=True)
    x = walk(n, 21 + n % 7, scale=2.0)
    y = walk(n, 22 + n % 5, scale=2.0)
    x[n // 2:n // 2 + 3 * L] = 0.0                     # zero products, constant blocks
    for rel in (1e-2, 1e-3):
        eb = synth.rel_eb(x, rel)
        xc, yc = ref.compress(x, eb, L), ref.compress(y, eb, L)
        a, b = gpu(xc, dev), gpu(yc, dev)
        want = ref.hadamard(xc, yc)
        assert np.array_equal(host(hz.hadamard(a, b)), want), rel
        assert np.array_equal(host(hz.hadamard(b, a)), want), rel


def test_hadamard_exact_cases(dev):
    """eps = 1/2 (decoded values are the bins: the product is exact), eps =
    1/4 (every odd product is a tie, rounded up), eps = 2^-1074-ish tiny and
    large products (range), mismatched operands."""
    rng = np.random.default_rng(6)
    qa = rng.integers(-40000, 40001, 90001).astype(np.int32)
    qb = rng.integers(-40000, 40001, 90001).astype(np.int32)
    for eb, L in ((0.5, 32), (0.25, 64), (0.375, 128), (1e-3, 256)):
        ac, bc = ref.encode_bins(qa, eb, L), ref.encode_bins(qb, eb, L)
        assert np.array_equal(host(hz.hadamard(gpu(ac, dev), gpu(bc, dev))), ref.hadamard(ac, bc)), eb
    ac = ref.encode_bins(np.full(100, 70000, np.int32), 0.5, 32)
    assert err_of(hz.hadamard, gpu(ac, dev), gpu(ac, dev)) == hz.ERR_RANGE
    tiny = ref.encode_bins(qa[:5000], 2.0**-1060, 32)
    assert np.array_equal(host(hz.hadamard(gpu(tiny, dev), gpu(tiny, dev))), ref.hadamard(tiny, tiny))
    x = walk(3000, 5)
    a = gpu(ref.compress(x, 0.01, 32), dev)
    for other in (ref.compress(x[:2999], 0.01, 32), ref.compress(x, 0.01, 64),
                  ref.compress(x, 0.01 * (1 + 2**-52), 32)):
        assert err_of(hz.hadamard, a, gpu(other, dev)) == hz.ERR_MISMATCH


def test_hadamard_wide_products(dev):
    """Products q_A q_B of 2^53 and more with in-range bins (eps = 2^-30:
    bins up to 2^27, products up to 2^54), exact ties 2 eps P = odd / 2 among
    them, and eps whose 2 eps is not a power of two: every segment must match
    the oracle, whichever binary64 or 128-bit path the kernel takes."""
    rng = np.random.default_rng(16)
    n = 70001
    for eb in (2.0**-30, 3 * 2.0**-33):
        qa = rng.integers(-(1 << 27), (1 << 27) + 1, n).astype(np.int32)
        qb = rng.integers(-(1 << 27), (1 << 27) + 1, n).astype(np.int32)
        qa[:3000] = rng.integers(-(1 << 13), (1 << 13) + 1, 3000)      # small products
        qb[:3000] = rng.integers(-(1 << 13), (1 << 13) + 1, 3000)
        qa[5000:6000] = 1 << 14                                         # P = 2^28 * odd: ties
        qb[5000:6000] = ((rng.integers(0, 1 << 12, 1000) * 2 + 1) << 14) * rng.choice([-1, 1], 1000)
        for L in (32, 128):
            ac, bc = ref.encode_bins(qa, eb, L), ref.encode_bins(qb, eb, L)
            print(f"case hadamard wide eb={eb} L={L}", flush=True)
            want = ref.hadamard(ac, bc)
            assert np.array_equal(host(hz.hadamard(gpu(ac, dev), gpu(bc, dev))), want), (eb, L)


@pytest.mark.parametrize("n,L", PAIR_CASES)
def test_covariance(dev, n, L):
    print(f"case covariance n={n} L={L}", flush=True)
    x = walk(n, 31 + n % 7)
    y = (0.5 * x + walk(n, 32 + n % 3)).astype(np.float32)
    ea, eb = synth.rel_eb(x, 1e-3), synth.rel_eb(y, 1e-4)   # different bounds are allowed
    xc, yc = ref.compress(x, ea, L), ref.compress(y, eb, L)
    a, b = gpu(xc, dev), gpu(yc, dev)
    for u, v, uc, vc in ((a, b, xc, yc), (b, a, yc, xc), (a, a, xc, xc)):
        want = ref.covariance(uc, vc)
        got = hz.covariance(u, v)
        assert got == want or abs(got - want) <= 1e-12 * abs(want), (got, want)
    assert hz.covariance(a, a) == ref.variance(xc) or \
        abs(hz.covariance(a, a) - ref.variance(xc)) <= 1e-12 * ref.variance(xc)


def test_covariance_extreme_bins(dev):
    """Bins near +-2^31 make q_A q_B ~ 2^62 and the 128-bit sums carry."""
    rng = np.random.default_rng(9)
    qa = rng.integers(-BIN_MAX, BIN_MAX + 1, 200003).astype(np.int32)
    qb = rng.integers(-BIN_MAX, BIN_MAX + 1, 200003).astype(np.int32)
    qb[::3] = qa[::3]
    for L in BLOCKS:
        ac, bc = ref.encode_bins(qa, 0.5, L), ref.encode_bins(qb, 0.25, L)
        want = ref.covariance(ac, bc)
        got = hz.covariance(gpu(ac, dev), gpu(bc, dev))
        assert got == want or abs(got - want) <= 1e-12 * abs(want), (L, got, want)
    x = walk(1000, 2)
    a = gpu(ref.compress(x, 0.01, 32), dev)
    for other in (ref.compress(x[:999], 0.01, 32), ref.compress(x, 0.01, 64)):
        assert err_of(hz.covariance, a, gpu(other, dev)) == hz.ERR_MISMATCH


# ------------------------------------------------------ block-wise means

@pytest.mark.parametrize("n,L", [(1, 32), (100, 64), (70001, 32), (300007, 128), (1048576, 256),
                                 (2000003, 32)])
def test_block_means(dev, n, L):
    print(f"case block means n={n} L={L}", flush=True)
    x = walk(n, 41 + n % 11)
    x[n // 4:n // 4 + 7 * L] = -2.5                 # constant blocks
    x[n // 2:n // 2 + 2 * L] = 0.0
    eb = synth.rel_eb(x, 1e-2)
    xc = ref.compress(x, eb, L)
    want, want_const = ref.block_means(xc)
    got, got_const = hz.block_means(gpu(xc, dev))
    assert got_const == want_const
    assert np.array_equal(host(got), want)
    res = hz.new_result(dev)
    out = torch.empty(want.size, dtype=torch.float64, device=dev)
    ctx = hz.context(0)
    assert hz._lib().hoszp_block_means_async(ctx.handle, hz._ptr(gpu(xc, dev)), xc.size,
                                             hz._ptr(out), out.numel(), hz._ptr(res),
                                             hz._stream(None)) == 0
    r = hz.read_result(res)
    assert r["code"] == 0 and r["count"] == want_const and r["value"] == ref.mean(xc)
    small = torch.empty(max(want.size - 1, 0), dtype=torch.float64, device=dev)
    if want.size > 1:
        with pytest.raises(hz.HoszpError) as e:
            hz.block_means(gpu(xc, dev), out=small)
        assert e.value.code == hz.ERR_CAPACITY
