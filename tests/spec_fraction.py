"""Exact-arithmetic brute force for tiny inputs (pins the oracle).

Everything here works on Python integers and ``fractions.Fraction`` built from
the exact binary values of the float32 inputs and the float64 bound, so there
is no rounding anywhere.  It is deliberately written differently from the C
oracle (whole-array integer manipulations, a bit list for the stream) so that
a mistake in one is unlikely to be repeated in the other.
"""
from fractions import Fraction
import math
import struct


def exact_t(x: float, eb: float) -> Fraction:
    """(x + eps) / (2 eps) with no rounding (Eq. 3 before the floor)."""
    return (Fraction(x) + Fraction(eb)) / (2 * Fraction(eb))


def exact_bin(x: float, eb: float) -> int:
    return math.floor(exact_t(x, eb))


def near_tie(x: float, eb: float, rel: float = 2.0 ** -40) -> bool:
    """True when the exact quotient is so close to an integer that the
    binary64 evaluation of Eq. 3 may legitimately land in either bin."""
    t = exact_t(x, eb)
    dist = abs(t - round(t))
    return dist <= Fraction(rel) * max(1, abs(t))


def bins_exact(xs, eb):
    return [exact_bin(float(v), eb) for v in xs]


def deltas(bins, L):
    """Per block: (outlier, [delta_0 = 0, q1-q0, ...] padded with zeros)."""
    out = []
    for start in range(0, len(bins), L):
        blk = bins[start:start + L]
        d = [0] + [blk[k] - blk[k - 1] for k in range(1, len(blk))]
        d += [0] * (L - len(d))
        out.append((blk[0], d))
    return out


def width_of(d):
    return max(abs(v) for v in d).bit_length()


def _pad16(buf):
    while len(buf) % 16:
        buf.append(0)


def encode(bins, eb, L):
    """Stream bytes for the given bins, built from bit lists."""
    blocks = deltas(bins, L)
    nb = len(blocks)
    widths = [width_of(d) for _, d in blocks]
    sign_bits = []
    pay_bits = []
    for (_, d), w in zip(blocks, widths):
        sign_bits += [1 if v < 0 else 0 for v in d]
        for v in d:
            m = abs(v)
            pay_bits += [(m >> (w - 1 - j)) & 1 for j in range(w)]

    def bits_to_bytes(bits):
        out = []
        for i in range(0, len(bits), 8):
            byte = 0
            for j, bit in enumerate(bits[i:i + 8]):
                byte |= bit << (7 - j)
            out.append(byte)
        return out

    body = bytearray(64)
    body += bytes(widths)
    _pad16(body)
    for o, _ in blocks:
        body += struct.pack("<i", o)
    _pad16(body)
    body += bytes(bits_to_bytes(sign_bits))
    _pad16(body)
    payload = bytes(bits_to_bytes(pay_bits))
    body += payload
    header = struct.pack("<4sHHII", b"HOSZ", 1, 0, L, 0)
    header += struct.pack("<QdQQQQ", len(bins), eb, nb, len(payload), len(body), 0)
    body[0:64] = header
    return bytes(body)


def mean_exact(bins, eb) -> Fraction:
    return Fraction(sum(bins), len(bins)) * 2 * Fraction(eb)


def var_exact(bins, eb) -> Fraction:
    n = len(bins)
    mu = Fraction(sum(bins), n)
    return sum((Fraction(b) - mu) ** 2 for b in bins) / n * (2 * Fraction(eb)) ** 2


def mul_bin_exact(s: float, q: int) -> int:
    """floor(s q + 1/2) in exact arithmetic."""
    return math.floor(Fraction(s) * q + Fraction(1, 2))
