"""The rounding rule of scalar multiplication (Sec. V-A: q' = floor(s q + 1/2),
the unquantized scalar, half up) checked on the host, without a device:

- the library's own rounding function (``hoszp_mul_bins``, the same source the
  kernel compiles) against exact rational arithmetic on every near-tie class
  and on random scalars;
- the oracle's scalar multiplication (through a stream of the same bins)
  against the same exact results, so both sides are pinned to mathematics,
  not to each other.
"""
import numpy as np
import pytest

import paper_2408_11971_amd as hz
from mul_cases import BIN_MAX, exact_mul_bins, tie_cases
from oracle import ref


@pytest.fixture(scope="module", autouse=True)
def lib():
    import os
    if not os.path.exists(hz.LIB_PATH):
        from paper_2408_11971_amd import build
        build.build()
    return hz._lib()


def check_library(s, q):
    want = exact_mul_bins(s, q)
    rc, got = hz.mul_bins(s, q)
    in_range = np.array([w is not None for w in want])
    assert (rc == hz.ERR_RANGE) == (not in_range.all()), (s, rc)
    exp = np.array([w if w is not None else 0 for w in want], dtype=np.int64)
    bad = np.nonzero(got.astype(np.int64) != exp)[0]
    assert bad.size == 0, f"s={s!r} q={q[bad[:4]]} got={got[bad[:4]]} want={exp[bad[:4]]}"


def test_reported_cases():
    """Scalars for which a binary64 evaluation of y + 1/2 rounds across an
    integer: y = fl(s q) = 1/2 - 2^-54 (tie to even at 1.0) and
    y = 2^k - 1/2 + ulp(y) (tie to even at 2^k)."""
    for s, q, want in ((1.1, 465, 512), (0.55, 930, 512), (1e-5, 150000, 2),
                       (float(np.nextafter(0.5, 0)), 1, 0), (0.24999999999999997, 2, 0),
                       (-0.49999999999999994, -1, 0)):
        assert exact_mul_bins(s, [q])[0] == want
        rc, got = hz.mul_bins(s, np.array([q], dtype=np.int32))
        assert rc == hz.OK and int(got[0]) == want, (s, q, got)


def test_tie_classes():
    cases = tie_cases()
    assert len(cases) > 1000
    for s, q in cases:
        check_library(s, q)


def test_random_scalars():
    rng = np.random.default_rng(5)
    q = rng.integers(-BIN_MAX, BIN_MAX + 1, 3000).astype(np.int32)
    q[:200] = rng.integers(-1000, 1001, 200)
    for e in range(-50, 34, 3):
        for s in rng.uniform(-2.0, 2.0, 3) * 2.0**e:
            check_library(float(s), q)


def test_tiny_and_huge_scalars():
    q = np.array([0, 1, -1, 2, 1000, -BIN_MAX, BIN_MAX], dtype=np.int32)
    for s in (2.0**-47, 2.0**-48, 2.0**-49, 1e-300, 5e-324, -5e-324, 2.0**31, 2.0**52,
              1e300, -1e300, 0.0, -0.0):
        check_library(s, q)


def test_non_finite_scalar_is_an_argument_error():
    q = np.array([1, 2], dtype=np.int32)
    for s in (float("nan"), float("inf"), -float("inf")):
        assert hz.mul_bins(s, q)[0] == hz.ERR_ARG


def test_oracle_scalar_multiplication_is_exact():
    """ref.mul on a stream of these bins (eb = 1/2, so bins are the values)
    decodes to the exact results, or reports RANGE exactly when one leaves
    the bin range."""
    for s, q in tie_cases(seed=29, random_ties=100)[::3]:
        want = exact_mul_bins(s, q)
        c = ref.encode_bins(q, 0.5, 32)
        if any(w is None for w in want):
            with pytest.raises(ref.RefError) as e:
                ref.mul(c, s)
            assert e.value.code == ref.ERR_RANGE
            continue
        got = ref.decode_bins(ref.mul(c, s))
        assert np.array_equal(got.astype(np.int64), np.array(want, dtype=np.int64)), s
