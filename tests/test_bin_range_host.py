"""The float input interval of compress (hoszp_bin_range) pinned to its
definition on the host: the bin of Eq. 3, floor(((double)x + eb) * (1/(2 eb)))
in binary64 (Python floats are binary64 and apply no contraction), must be in
[-(2^31-1), 2^31-1] at both ends of the interval and outside it at the next
float beyond each end.  The kernels' range test relies on this interval."""
import math

import numpy as np
import pytest

import paper_2408_11971_amd as hz

K = 2.0**31 - 1
FLT_MAX = float(np.finfo(np.float32).max)


@pytest.fixture(scope="module", autouse=True)
def lib():
    import os
    if not os.path.exists(hz.LIB_PATH):
        from paper_2408_11971_amd import build
        build.build()
    return hz._lib()


def bin_of(x, eb):
    return math.floor((float(x) + eb) * (1.0 / (2.0 * eb)))


def step(x, direction):
    return float(np.nextafter(np.float32(x), np.float32(direction)))


def check(eb):
    lo, hi = hz.bin_range(eb)
    assert np.float32(lo) == lo and np.float32(hi) == hi
    assert -FLT_MAX <= lo <= 0.0 <= hi <= FLT_MAX
    assert bin_of(hi, eb) <= K and bin_of(lo, eb) >= -K
    if hi < FLT_MAX:
        assert bin_of(step(hi, math.inf), eb) > K
    if lo > -FLT_MAX:
        assert bin_of(step(lo, -math.inf), eb) < -K


def test_interval_ends_are_exact():
    for eb in (1e-3, 0.5, 0.25, 1.0, 1e-8, 3e-39, 1e-45, 1e30, 1e38, 2.0**-20, 0.01,
               0.030644772338867188):
        check(eb)
    rng = np.random.default_rng(8)
    for e in rng.uniform(-40, 38, 300):
        check(float(10.0**e))


def test_rejects_bad_bounds():
    for eb in (0.0, -1.0, math.inf, math.nan):
        with pytest.raises(hz.HoszpError) as e:
            hz.bin_range(eb)
        assert e.value.code == hz.ERR_ARG
