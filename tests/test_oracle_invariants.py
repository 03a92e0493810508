"""Oracle pinned to closed forms, invariants and textbook special cases."""
import numpy as np
import pytest

from oracle import ref
import synth

BLOCKS = [32, 64, 128, 256]


def seeded(n, seed, scale=10.0):
    return np.random.default_rng(seed).normal(0.0, scale, size=n).astype(np.float32)


@pytest.mark.parametrize("L", BLOCKS)
def test_ramp_closed_form(L):
    """x_i = 2 eps i: bins i, every delta 1, so every block has width 1, no
    sign bit set, and payload bits 0 then 1 1 1 ... (slot 0 is 0).  Mean and
    variance of 0..N-1 are (N-1)/2 and (N^2-1)/12 (times 2 eps, (2 eps)^2)."""
    eb = 0.5                       # 2 eps = 1: x_i = i exactly
    n = 4 * L
    x = np.arange(n, dtype=np.float32)
    c = ref.compress(x, eb, L)
    info = ref.info(c)
    nb = n // L
    assert info["payload_bytes"] == nb * L // 8
    off_w = 64
    assert c[off_w:off_w + nb].tolist() == [1] * nb
    pay = c[info["total_bytes"] - info["payload_bytes"]:]
    per_block = [0x7F] + [0xFF] * (L // 8 - 1)
    assert pay.tolist() == per_block * nb
    assert ref.mean(c) == (n - 1) / 2.0
    assert ref.variance(c) == (n * n - 1) / 12.0


@pytest.mark.parametrize("L", BLOCKS)
@pytest.mark.parametrize("n", [1, 5, 31, 32, 33, 63, 64, 65, 127, 128, 129, 1000])
def test_error_bound_power_of_two(n, L):
    """|x - decompress(x)| <= eps exactly when eps is a power of two and the
    bins stay below 2^24 (every operation is then exact)."""
    x = seeded(n, 100 + n)
    eb = 2.0 ** -6
    y = ref.decompress(ref.compress(x, eb, L))
    assert np.all(np.abs(x.astype(np.float64) - y.astype(np.float64)) <= eb)


@pytest.mark.parametrize("rel", [1e-2, 1e-3, 1e-4])
def test_error_bound_general(rel):
    x = synth.sinusoid_1d(1 << 14, seed=1)
    eb = synth.rel_eb(x, rel)
    y = ref.decompress(ref.compress(x, eb, 32)).astype(np.float64)
    xd = x.astype(np.float64)
    slack = eb + 2.0 ** -24 * np.abs(y) + 2.0 ** -45 * np.abs(xd)
    assert np.all(np.abs(xd - y) <= slack)


@pytest.mark.parametrize("L", BLOCKS)
def test_negate_is_an_involution(L):
    c = ref.compress(seeded(1000, 3), 0.01, L)
    n1 = ref.negate(c)
    assert not np.array_equal(n1, c)
    assert np.array_equal(ref.negate(n1), c)


@pytest.mark.parametrize("L", BLOCKS)
def test_add_commutes_and_cancels(L):
    a = ref.compress(seeded(777, 4), 0.01, L)
    b = ref.compress(seeded(777, 5), 0.01, L)
    assert np.array_equal(ref.add(a, b), ref.add(b, a))
    z = ref.add(a, ref.negate(a))
    info = ref.info(z)
    nb = (777 + L - 1) // L
    assert info["payload_bytes"] == 0
    assert z[64:64 + nb].tolist() == [0] * nb
    assert np.all(ref.decode_bins(z) == 0)


@pytest.mark.parametrize("L", BLOCKS)
def test_sum_is_additive(L):
    a = ref.compress(seeded(999, 6), 0.05, L)
    b = ref.compress(seeded(999, 7), 0.05, L)
    sa, qa = ref.sums(a)
    sb, qb = ref.sums(b)
    sz, _ = ref.sums(ref.add(a, b))
    assert sz == sa + sb


@pytest.mark.parametrize("L", BLOCKS)
def test_mul_identities(L):
    c = ref.compress(seeded(555, 8), 0.01, L)
    assert np.array_equal(ref.mul(c, 1.0), c)
    z = ref.mul(c, 0.0)
    assert np.all(ref.decode_bins(z) == 0)
    assert ref.info(z)["payload_bytes"] == 0
    assert np.array_equal(ref.decode_bins(ref.mul(c, -1.0)), -ref.decode_bins(c))
    assert np.array_equal(ref.decode_bins(ref.mul(c, 2.0)), 2 * ref.decode_bins(c))


@pytest.mark.parametrize("L", BLOCKS)
def test_constant_field(L):
    x = np.full(300, 3.0, dtype=np.float32)
    eb = 0.25                                 # bins floor(3.25 / 0.5) = 6
    c = ref.compress(x, eb, L)
    assert ref.info(c)["payload_bytes"] == 0
    assert ref.mean(c) == 3.0
    assert ref.variance(c) == 0.0


@pytest.mark.parametrize("L", BLOCKS)
def test_mean_variance_match_numpy(L):
    """Textbook special case: numpy's mean and var (ddof=0) of the decoded
    values 2 eps q computed in float64."""
    x = synth.sinusoid_1d(20000, seed=2)
    eb = synth.rel_eb(x, 1e-3)
    c = ref.compress(x, eb, L)
    vals = ref.decode_bins(c).astype(np.float64) * (2.0 * eb)
    assert abs(ref.mean(c) - vals.mean()) <= 1e-12 * max(1.0, abs(vals.mean()))
    assert abs(ref.variance(c) - vals.var()) <= 1e-12 * vals.var()


def test_traditional_workflow_equivalence():
    """Theorem 1 against the decompress-operate-recompress workflow: negate,
    add and mul on the compressed stream equal re-compressing the operated
    decompressed field (bins far below 2^24, no ties)."""
    a = synth.sinusoid_1d(4096, seed=1)
    b = synth.sinusoid_1d(4096, seed=2)
    eb = synth.rel_eb(a, 1e-3)
    ca = ref.compress(a, eb, 32)
    cb = ref.compress(b, eb, 32)
    da = ref.decompress(ca)
    db = ref.decompress(cb)
    assert np.array_equal(ref.decode_bins(ref.negate(ca)), ref.decode_bins(ref.compress(-da, eb, 32)))
    assert np.array_equal(ref.add(ca, cb), ref.compress(da + db, eb, 32))
    # mul: the float32 intermediate of the traditional workflow can only
    # disagree where s q sits within float32 rounding of a half-integer tie
    s = 3.0 ** 0.5  # irrational-like: no exact half-integer ties
    trad = ref.decode_bins(ref.compress((da.astype(np.float64) * s).astype(np.float32), eb, 32))
    homo = ref.decode_bins(ref.mul(ca, s))
    q = ref.decode_bins(ca).astype(np.float64)
    frac = np.abs((q * s) - np.floor(q * s) - 0.5)
    differ = trad != homo
    assert np.all(frac[differ] < 1e-5 * np.maximum(1.0, np.abs(q[differ] * s)))
    assert np.all(np.abs(trad.astype(np.int64) - homo)[differ] == 1)
    assert differ.mean() < 0.01


@pytest.mark.parametrize("n", [1, 31, 32, 33])
def test_short_fields(n):
    x = seeded(n, 11)
    for L in BLOCKS:
        c = ref.compress(x, 0.1, L)
        assert ref.info(c)["n"] == n
        assert np.array_equal(ref.decode_bins(c), ref.quantize(x, 0.1))
