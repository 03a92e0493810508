"""Scalars and bins that put s*q on, or within a few ulps of, a half-integer:
the places where floor(s q + 1/2) is decided by the last bits of the exact
product (scalar multiplication, Sec. V-A).  Pure numpy; shared by the CPU
test of the rounding function and the GPU parity test of the kernel.

Each case is (s, q) with q an int32 numpy array; the exact result comes from
``exact_mul_bins`` (Python integers, no floating point).
"""
from fractions import Fraction

import numpy as np

BIN_MAX = 2**31 - 1


def exact_mul_bins(s: float, q) -> np.ndarray:
    """floor(s q + 1/2) in exact rational arithmetic (Python ints); values
    outside the int32 bin range come back as None in an object array."""
    f = Fraction(s)
    num, den = f.numerator, f.denominator
    out = np.empty(len(q), dtype=object)
    for i, v in enumerate(np.asarray(q, dtype=np.int64).tolist()):
        r = (2 * num * v + den) // (2 * den)
        out[i] = r if -BIN_MAX <= r <= BIN_MAX else None
    return out


def _nb(x, k):
    """x moved k ulps (k may be negative)."""
    d = np.inf if k > 0 else -np.inf
    for _ in range(abs(k)):
        x = float(np.nextafter(x, d))
    return x


def _powers():
    p = [1 << j for j in range(31)]
    return np.array(p + [-v for v in p] + [BIN_MAX, -BIN_MAX, 3, -3, 5, -5, 7, -7],
                    dtype=np.int64)


def tie_cases(seed: int = 23, random_ties: int = 400):
    """List of (s, q) pairs covering the classes where a binary64 evaluation
    of s q + 1/2 can round across an integer:
      - s at and one ulp beside 1/2^(k+1) with q = +-2^k (s q next to 1/2);
      - s q = 2^k - 1/2 plus or minus a few ulps (y + 1/2 crossing a binade);
      - reported scalars: 1.1 * 465, 0.55 * 930, 1e-5 * 150000;
      - random half-integer targets t + 1/2 with s = (t + 1/2)/q and its
        neighbours;
      - dyadic scalars (exact products, frequent exact ties)."""
    rng = np.random.default_rng(seed)
    pw = _powers()
    cases = []
    for k in range(31):
        base = 0.5 / float(1 << k)
        for d in (-2, -1, 0, 1, 2):
            s = _nb(base, d)
            cases.append((s, pw))
            cases.append((-s, pw))
    for k in range(1, 31):
        target = float(1 << k) - 0.5
        for q in rng.integers(1, BIN_MAX, 3).tolist() + [1, 3, (1 << 20) + 1]:
            s0 = target / q
            for d in (-2, -1, 0, 1, 2):
                s = _nb(s0, d)
                cases.append((s, np.array([q, -q, q - 1, q + 1, 1, -1], dtype=np.int64)))
    for s, q in ((1.1, 465), (0.55, 930), (1e-5, 150000), (float(np.nextafter(0.5, 0)), 1),
                 (0.49999999999999994, 1), (0.24999999999999997, 2), (-0.49999999999999994, -1)):
        qs = np.array([q, -q, q - 1, q + 1, 2 * q, 3 * q], dtype=np.int64)
        cases.append((s, qs))
        cases.append((-s, qs))
    for _ in range(random_ties):
        q = int(rng.integers(1, BIN_MAX))
        if rng.random() < 0.5:
            q = -q
        t = int(rng.integers(-(1 << 30), 1 << 30)) + 0.5
        s0 = t / q
        d = int(rng.integers(-2, 3))
        cases.append((_nb(s0, d), np.array([q, -q], dtype=np.int64)))
    dy = rng.integers(-(1 << 20), 1 << 20, 512)
    for s in (0.5, -0.5, 0.25, 1.5, -2.5, 0.75, 1.0, -1.0, 0.0, 2.0**-30, 3 * 2.0**-20):
        cases.append((s, dy))
    return [(float(s), np.asarray(q, dtype=np.int64).clip(-BIN_MAX, BIN_MAX).astype(np.int32))
            for s, q in cases]
