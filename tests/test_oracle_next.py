"""Pins of the oracle's remaining Table II operations against what the paper
and the mathematics fix (no GPU):

- scalar addition / subtraction (Sec. V-A, workflow 1): the scalar's bin by
  Eq. 3 added to (subtracted from) every outlier, everything else unchanged;
  the worked example; exact rational arithmetic;
- element-wise subtraction (Sec. V-C): bins q_A - q_B; A - B = A + (-B);
- standard deviation (Sec. V-B): the square root of the variance;
- Hadamard product (Sec. V-C): floor(2 eps q_A q_B + 1/2) exactly;
- covariance (Sec. V-D): exact population covariance of the decoded fields;
- block-wise means and constant blocks (Sec. V-B, Table VI).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import spec_fraction as spec
from oracle import ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")
BIN_MAX = 2**31 - 1


def golden():
    vals = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = (s.strip() for s in line.split("=", 1))
            vals[k] = v
    return vals


def stream(seed, n, L, rel=1e-3, scale=1.0):
    rng = np.random.default_rng(seed)
    x = np.cumsum(rng.normal(0.0, scale, n)).astype(np.float32)
    eb = rel * float(x.max() - x.min())
    return x, eb, ref.compress(x, eb, L)


def sections(c):
    i = ref.info(c)
    n, L = i["n"], i["block"]
    nb = (n + L - 1) // L
    r16 = lambda v: (v + 15) // 16 * 16  # noqa: E731
    ow = 64
    oo = r16(ow + nb)
    os_ = r16(oo + 4 * nb)
    op = r16(os_ + nb * L // 8)
    return nb, ow, oo, os_, op


def outliers(c):
    nb, ow, oo, os_, op = sections(c)
    return c[oo:oo + 4 * nb].view(np.int32)


def exact_scalar_bin(s, eb):
    return math.floor((Fraction(s) + Fraction(eb)) / (2 * Fraction(eb)))


# ------------------------------------------------------ scalar add / sub

def test_scalar_add_worked_example():
    """The 2x2 block of Sec. IV-A (bins -1 -1 -3 -3, eps 0.01) plus 0.67.
    Eq. 3 gives the scalar bin floor((0.67 + 0.01) / 0.02) = 34 in exact
    arithmetic; the paper prints 33 (and outlier 32), one less: a slip in the
    example, since its own proof adds s / (2 eps) = 33.5 unrounded.  Signs
    and magnitudes are unchanged (workflow 1 touches only the outliers)."""
    g = golden()
    eps = float(g["eps"])
    x = np.array([float(v) for v in g["values"].split()], dtype=np.float32)
    s = float(g["scalar_add_scalar"])
    assert exact_scalar_bin(s, eps) == int(g["scalar_add_bin_printed"]) + 1 == 34
    for L in (32, 64, 128, 256):
        c = ref.compress(x, eps, L)
        z = ref.scalar_add(c, s)
        assert ref.decode_bins(z).tolist() == [b + 34 for b in (-1, -1, -3, -3)]
        assert int(outliers(z)[0]) == int(g["scalar_add_outlier_printed"]) + 1 == 33
        diff = np.nonzero(z != c)[0]
        nb, ow, oo, os_, op = sections(c)
        assert diff.size > 0 and diff.min() >= oo and diff.max() < oo + 4 * nb


@pytest.mark.parametrize("L", [32, 64, 128, 256])
def test_scalar_add_sub_exact(L):
    rng = np.random.default_rng(L)
    for seed in range(6):
        x, eb, c = stream(seed, 3001 + 97 * seed, L)
        q = ref.decode_bins(c).astype(np.int64)
        for s in rng.uniform(-50, 50, 4).tolist() + [0.0, -0.0, eb, -eb, 1e-300]:
            if spec.near_tie(s, eb):
                continue
            qs = exact_scalar_bin(s, eb)
            za, zs = ref.scalar_add(c, s), ref.scalar_sub(c, s)
            assert np.array_equal(ref.decode_bins(za), q + qs), (seed, s)
            assert np.array_equal(ref.decode_bins(zs), q - qs), (seed, s)
            assert np.array_equal(ref.scalar_sub(za, s), c)
            assert np.array_equal(ref.scalar_add(zs, s), c)
            # only the outliers change
            nb, ow, oo, os_, op = sections(c)
            keep = np.ones(c.size, bool)
            keep[oo:oo + 4 * nb] = False
            assert np.array_equal(za[keep], c[keep]) and np.array_equal(zs[keep], c[keep])


def test_scalar_add_keeps_negated_sign_bits():
    """On a negated stream (sign bits of zero deltas flipped, not canonical)
    scalar addition still changes nothing but the outliers."""
    x, eb, c = stream(3, 5000, 64)
    n = ref.negate(c)
    z = ref.scalar_add(n, 2.5)
    nb, ow, oo, os_, op = sections(c)
    keep = np.ones(c.size, bool)
    keep[oo:oo + 4 * nb] = False
    assert np.array_equal(z[keep], n[keep])
    assert np.array_equal(ref.decode_bins(z), ref.decode_bins(n) + exact_scalar_bin(2.5, eb))


def test_scalar_add_range():
    big = np.full(300, BIN_MAX - 5, np.int32)
    big[::3] = BIN_MAX - 50
    c = ref.encode_bins(big, 0.5, 32)          # eps 1/2: the scalar's bin is floor(s + 1/2)
    assert np.array_equal(ref.decode_bins(ref.scalar_add(c, 5.0)), big.astype(np.int64) + 5)
    for s in (6.0, 1e12):
        with pytest.raises(ref.RefError) as e:
            ref.scalar_add(c, s)
        assert e.value.code == ref.ERR_RANGE
    # a wide block far from the limit: the crude bound |O| + 31 (2^31 - 1) fails,
    # the exact bins fit
    wide = np.zeros(64, np.int32)
    wide[1::2] = 1 << 30
    wide[2::4] = -(1 << 30)
    cw = ref.encode_bins(wide, 0.5, 32)
    assert ref.info(cw)["payload_bytes"] > 0
    assert np.array_equal(ref.decode_bins(ref.scalar_add(cw, 2.0**29)),
                          wide.astype(np.int64) + 2**29)
    with pytest.raises(ref.RefError) as e:
        ref.scalar_add(cw, 2.0**30)
    assert e.value.code == ref.ERR_RANGE
    with pytest.raises(ref.RefError) as e:
        ref.scalar_sub(cw, 2.0**30)
    assert e.value.code == ref.ERR_RANGE
    for s in (math.nan, math.inf):
        with pytest.raises(ref.RefError) as e:
            ref.scalar_add(cw, s)
        assert e.value.code == ref.ERR_ARG


# --------------------------------------------------- element-wise subtraction

@pytest.mark.parametrize("L", [32, 64, 128, 256])
def test_sub_exact_and_relations(L):
    for seed in range(4):
        n = 2500 + 311 * seed
        x, eb, a = stream(seed, n, L)
        y = np.cumsum(np.random.default_rng(seed + 50).normal(0, 1, n)).astype(np.float32)
        b = ref.compress(y, eb, L)
        qa = ref.decode_bins(a).astype(np.int64)
        qb = ref.decode_bins(b).astype(np.int64)
        d = ref.sub(a, b)
        assert np.array_equal(ref.decode_bins(d), qa - qb)
        assert np.array_equal(d, ref.encode_bins((qa - qb).astype(np.int32), eb, L))
        assert np.array_equal(d, ref.add(a, ref.negate(b)))          # A - B = A + (-B)
        assert np.array_equal(ref.decode_bins(ref.sub(b, a)), qb - qa)  # not commutative
        assert not ref.decode_bins(ref.sub(a, a)).any()


def test_sub_errors():
    x, eb, a = stream(1, 1000, 32)
    for other in (ref.compress(x[:999], eb, 32), ref.compress(x, eb, 64),
                  ref.compress(x, eb * (1 + 2**-52), 32)):
        with pytest.raises(ref.RefError) as e:
            ref.sub(a, other)
        assert e.value.code == ref.ERR_MISMATCH
    hi = ref.encode_bins(np.full(50, BIN_MAX, np.int32), 0.5, 32)
    lo = ref.encode_bins(np.full(50, -1, np.int32), 0.5, 32)
    with pytest.raises(ref.RefError) as e:
        ref.sub(hi, lo)
    assert e.value.code == ref.ERR_RANGE


# ------------------------------------------------------ standard deviation

def test_std_is_sqrt_of_variance():
    g = golden()
    x = np.array([float(v) for v in g["values"].split()], dtype=np.float32)
    c = ref.compress(x, float(g["eps"]), 32)
    assert abs(ref.std(c) - math.sqrt(float(g["variance_derived"]))) <= 1e-15
    for seed, L in ((0, 32), (1, 64), (2, 128)):
        x, eb, c = stream(seed, 20000, L)
        q = ref.decode_bins(c).astype(np.int64).tolist()
        exact = math.sqrt(spec.var_exact(q, eb))
        assert abs(ref.std(c) - exact) <= 1e-13 * exact
        vals = np.asarray(q, dtype=np.float64) * (2.0 * eb)
        assert abs(ref.std(c) - np.std(vals)) <= 1e-12 * exact


# -------------------------------------------------------- Hadamard product

def hadamard_exact(qa, qb, eb):
    two = 2 * Fraction(eb)
    return [math.floor(two * a * b + Fraction(1, 2)) for a, b in zip(qa, qb)]


@pytest.mark.parametrize("L", [32, 128])
def test_hadamard_exact(L):
    for seed in range(4):
        n = 1500 + 97 * seed
        x, eb, a = stream(seed, n, L, rel=1e-2, scale=3.0)
        y = np.cumsum(np.random.default_rng(seed + 9).normal(0, 3.0, n)).astype(np.float32)
        b = ref.compress(y, eb, L)
        qa = ref.decode_bins(a).tolist()
        qb = ref.decode_bins(b).tolist()
        h = ref.hadamard(a, b)
        assert ref.decode_bins(h).tolist() == hadamard_exact(qa, qb, eb)
        assert np.array_equal(h, ref.hadamard(b, a))  # commutative


def test_hadamard_special_cases():
    rng = np.random.default_rng(4)
    qa = rng.integers(-3000, 3001, 777).astype(np.int32)
    qb = rng.integers(-3000, 3001, 777).astype(np.int32)
    # eps = 1/2: decoded values are the bins, so the product is exact
    a, b = ref.encode_bins(qa, 0.5, 32), ref.encode_bins(qb, 0.5, 32)
    assert np.array_equal(ref.decode_bins(ref.hadamard(a, b)), qa.astype(np.int64) * qb)
    # eps = 1/4: floor(q_A q_B / 2 + 1/2), ties (odd products) round up
    a, b = ref.encode_bins(qa, 0.25, 64), ref.encode_bins(qb, 0.25, 64)
    p = qa.astype(np.int64) * qb
    assert np.array_equal(ref.decode_bins(ref.hadamard(a, b)), (p + 1) // 2)
    assert (p % 2 != 0).any()
    # a product outside the bin range
    big = ref.encode_bins(np.full(40, 70000, np.int32), 0.5, 32)
    with pytest.raises(ref.RefError) as e:
        ref.hadamard(big, big)
    assert e.value.code == ref.ERR_RANGE


# --------------------------------------------------------------- covariance

def cov_exact(qa, qb, ea, eb):
    n = len(qa)
    ma = Fraction(sum(qa), n)
    mb = Fraction(sum(qb), n)
    s = sum((a - ma) * (b - mb) for a, b in zip(qa, qb)) / n
    return s * (2 * Fraction(ea)) * (2 * Fraction(eb))


@pytest.mark.parametrize("L", [32, 64, 256])
def test_covariance_exact(L):
    for seed in range(4):
        n = 3000 + 123 * seed
        x, ea, a = stream(seed, n, L)
        y = (0.3 * x + np.random.default_rng(seed + 3).normal(0, 1, n)).astype(np.float32)
        eb = 1e-3 * float(y.max() - y.min())    # a different error bound is allowed
        b = ref.compress(y, eb, L)
        qa = ref.decode_bins(a).astype(np.int64).tolist()
        qb = ref.decode_bins(b).astype(np.int64).tolist()
        want = cov_exact(qa, qb, ea, eb)
        got = ref.covariance(a, b)
        assert abs(Fraction(got) - want) <= Fraction(1e-14) * abs(want)
        va = np.asarray(qa, np.float64) * (2 * ea)
        vb = np.asarray(qb, np.float64) * (2 * eb)
        npc = np.cov(va, vb, bias=True)[0, 1]
        assert abs(got - npc) <= 1e-10 * abs(npc)
        assert ref.covariance(a, a) == ref.variance(a)   # same exact integers, same formula
        assert abs(ref.covariance(b, a) - got) <= 1e-15 * abs(got)


def test_covariance_mismatch():
    x, eb, a = stream(1, 1000, 32)
    for other in (ref.compress(x[:999], eb, 32), ref.compress(x, eb, 64)):
        with pytest.raises(ref.RefError) as e:
            ref.covariance(a, other)
        assert e.value.code == ref.ERR_MISMATCH


# ------------------------------------------------------ block-wise means

@pytest.mark.parametrize("L", [32, 64, 128, 256])
def test_block_means_exact(L):
    rng = np.random.default_rng(L + 1)
    n = 40 * L + 13                      # a ragged last block
    x = np.cumsum(rng.normal(0, 1, n)).astype(np.float32)
    x[5 * L:9 * L] = 7.25                # four constant blocks
    x[20 * L:20 * L + L] = 0.0           # and a fifth
    eb = 1e-3 * float(x.max() - x.min())
    c = ref.compress(x, eb, L)
    q = ref.decode_bins(c).astype(np.int64)
    means, const = ref.block_means(c)
    nb = (n + L - 1) // L
    assert means.size == nb
    two = 2 * Fraction(eb)
    n_const = 0
    for b in range(nb):
        blk = q[b * L:(b + 1) * L]
        exact = Fraction(int(blk.sum()), blk.size) * two
        assert abs(Fraction(means[b]) - exact) <= Fraction(2.0**-51) * abs(exact)
        n_const += int((blk == blk[0]).all())
    assert const == n_const >= 5
    # the mean of the block means weighted by block length is the mean
    w = np.array([min(L, n - b * L) for b in range(nb)], np.float64)
    assert abs(float((means * w).sum() / n) - ref.mean(c)) <= 1e-12 * abs(ref.mean(c)) + 1e-15


def test_constant_blocks_are_width_zero_blocks():
    """A block is constant exactly when all its bins are equal: blocks whose
    bins differ by one (width 1) are not counted."""
    rng = np.random.default_rng(8)
    for L in (32, 64):
        q = np.cumsum(rng.integers(-3, 4, 30 * L)).astype(np.int32)
        q[3 * L:4 * L] = 17                              # constant
        q[4 * L:5 * L] = 17 + (np.arange(L) % 2)          # width 1
        q[7 * L:8 * L] = -5                               # constant
        q[9 * L:10 * L] = 100 + (np.arange(L) >= L // 2)  # width 1, one step
        c = ref.encode_bins(q, 0.5, L)
        means, const = ref.block_means(c)
        blocks = q.reshape(-1, L)
        assert const == int((blocks == blocks[:, :1]).all(axis=1).sum()) == 2
        assert np.array_equal(means, blocks.mean(axis=1))   # eps 1/2: 2 eps = 1


def test_block_means_worked_example():
    g = golden()
    x = np.array([float(v) for v in g["values"].split()], dtype=np.float32)
    means, const = ref.block_means(ref.compress(x, float(g["eps"]), 32))
    assert means.tolist() == [float(g["mean"])] and const == 0
