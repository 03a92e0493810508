"""Oracle pinned to exact rational arithmetic on tiny inputs (brute force).

Each property here fails for a plausible slip in the oracle: a wrong rounding
in Eq. 3, a dropped or doubled delta, a sign or bit-order error in the
packing, a missing term of the variance, an off-by-one in the mul rounding.
"""
from fractions import Fraction
import math

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import spec_fraction as spec
from oracle import ref

BLOCKS = [32, 64, 128, 256]

small_floats = st.floats(min_value=-1000.0, max_value=1000.0, allow_nan=False,
                         allow_infinity=False, width=32)
ebs = st.one_of(st.sampled_from([2.0 ** -k for k in range(1, 12)]),
                st.floats(min_value=1e-4, max_value=10.0, allow_nan=False, allow_infinity=False))


def field(draw_list):
    return np.array(draw_list, dtype=np.float32)


settings.register_profile("oracle", max_examples=150, deadline=None,
                          suppress_health_check=[HealthCheck.too_slow])
settings.load_profile("oracle")


@given(st.lists(small_floats, min_size=1, max_size=300), ebs)
def test_quantize_is_exact_floor(xs, eb):
    x = field(xs)
    q = ref.quantize(x, eb)
    for v, got in zip(x.tolist(), q.tolist()):
        want = spec.exact_bin(v, eb)
        if got != want:
            assert spec.near_tie(v, eb), (v, eb, got, want)
            assert abs(got - want) == 1


@given(st.integers(min_value=-50, max_value=50), st.sampled_from([2.0 ** -k for k in range(1, 20)]))
def test_bin_edges_power_of_two(k, eb):
    """Exactly on the edge (2k-1) eps of bin k, Eq. 3 gives bin k (floor of an
    integer); just below it gives k-1.  With eps a power of two the binary64
    evaluation is exact, so no tie slack is needed."""
    edge = np.float32((2 * k - 1) * eb)
    if float(edge) != (2 * k - 1) * eb:
        return
    below = np.nextafter(edge, np.float32(-np.inf))
    q = ref.quantize(np.array([edge, below], dtype=np.float32), eb)
    assert q[0] == k
    assert q[1] == k - 1


@given(st.lists(small_floats, min_size=1, max_size=300), ebs, st.sampled_from(BLOCKS))
def test_stream_bytes_match_bit_list_encoder(xs, eb, L):
    x = field(xs)
    q = ref.quantize(x, eb)
    c = ref.compress(x, eb, L)
    assert bytes(c) == spec.encode(q.tolist(), eb, L)


@given(st.lists(small_floats, min_size=1, max_size=300), ebs, st.sampled_from(BLOCKS))
def test_decode_inverts_encode(xs, eb, L):
    x = field(xs)
    q = ref.quantize(x, eb)
    c = ref.compress(x, eb, L)
    assert np.array_equal(ref.decode_bins(c), q)
    y = ref.decompress(c)
    assert np.array_equal(y, (q.astype(np.float64) * (2.0 * eb)).astype(np.float32))


@given(st.lists(small_floats, min_size=1, max_size=300), ebs, st.sampled_from(BLOCKS))
def test_mean_variance_exact(xs, eb, L):
    x = field(xs)
    c = ref.compress(x, eb, L)
    q = ref.decode_bins(c).tolist()
    m_exact = spec.mean_exact(q, eb)
    v_exact = spec.var_exact(q, eb)
    m = ref.mean(c)
    v = ref.variance(c)
    assert abs(Fraction(m) - m_exact) <= Fraction(1, 10 ** 15) * abs(m_exact) + Fraction(0)
    assert abs(Fraction(v) - v_exact) <= Fraction(1, 10 ** 15) * abs(v_exact)
    s, qq = ref.sums(c)
    assert s == sum(q)
    assert qq == sum(b * b for b in q)


@given(st.lists(small_floats, min_size=1, max_size=200), ebs, st.sampled_from(BLOCKS),
       st.floats(min_value=-8.0, max_value=8.0, allow_nan=False, allow_infinity=False))
def test_mul_exact_half_up(xs, eb, L, s):
    x = field(xs)
    c = ref.compress(x, eb, L)
    q = ref.decode_bins(c).tolist()
    want = [spec.mul_bin_exact(s, b) for b in q]
    m = ref.mul(c, s)
    assert ref.decode_bins(m).tolist() == want
    assert bytes(m) == spec.encode(want, eb, L)


@given(st.lists(small_floats, min_size=1, max_size=200),
       st.lists(small_floats, min_size=1, max_size=200), ebs, st.sampled_from(BLOCKS))
def test_add_and_negate_on_bins(xa, xb, eb, L):
    n = min(len(xa), len(xb))
    a = field(xa[:n])
    b = field(xb[:n])
    ca = ref.compress(a, eb, L)
    cb = ref.compress(b, eb, L)
    qa = ref.decode_bins(ca)
    qb = ref.decode_bins(cb)
    z = ref.add(ca, cb)
    # Theorem 1 at the integer level: the sum's stream is the canonical
    # stream of the summed bins
    assert bytes(z) == spec.encode((qa.astype(np.int64) + qb).tolist(), eb, L)
    neg = ref.negate(ca)
    assert np.array_equal(ref.decode_bins(neg), -qa)


def test_mul_rounding_ties_go_up():
    """q = 1, s = 0.5: s q = 0.5 exactly, floor(1.0) = 1; s = -0.5 gives 0."""
    eb = 0.5
    x = np.array([1.0, 1.0], dtype=np.float32)   # bins floor((1+0.5)/1) = 1
    c = ref.compress(x, eb, 32)
    assert ref.decode_bins(c).tolist() == [1, 1]
    assert ref.decode_bins(ref.mul(c, 0.5)).tolist() == [1, 1]
    assert ref.decode_bins(ref.mul(c, -0.5)).tolist() == [0, 0]
    assert ref.decode_bins(ref.mul(c, 2.5)).tolist() == [3, 3]


def test_mul_needs_more_than_binary64():
    """floor(s q + 1/2) where s q lies within one binary64 ulp of a half
    integer: a double product would round onto the tie."""
    q = (1 << 30) + 1
    s = 0.5 + 2.0 ** -53          # s q = 2^29 + 0.5 + (2^30+1) 2^-53
    assert spec.mul_bin_exact(s, q) == (1 << 29) + 1
    eb = 0.5
    c = ref.encode_bins(np.array([q], dtype=np.int32), eb, 32)
    assert ref.decode_bins(ref.mul(c, s)).tolist() == [(1 << 29) + 1]
    s2 = 0.5 - 2.0 ** -53         # just below the tie: rounds down
    assert ref.decode_bins(ref.mul(c, s2)).tolist() == [spec.mul_bin_exact(s2, q)]
    assert spec.mul_bin_exact(s2, q) == (1 << 29)


def test_variance_large_bins_exact():
    """Bins near 2^31 make S^2 and N Q exceed 2^64; the exact difference is
    still reproduced."""
    q = np.array([2**31 - 1, 2**31 - 2, -(2**31 - 1), 5, 2**31 - 1], dtype=np.int32)
    eb = 0.25
    c = ref.encode_bins(q, eb, 32)
    v = ref.variance(c)
    ve = spec.var_exact(q.tolist(), eb)
    assert abs(Fraction(v) - ve) <= Fraction(1, 10 ** 15) * ve
    m = ref.mean(c)
    me = spec.mean_exact(q.tolist(), eb)
    assert abs(Fraction(m) - me) <= Fraction(1, 10 ** 15) * abs(me)
    assert math.isfinite(v)
