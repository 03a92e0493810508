"""Oracle pinned to the values the paper prints for its worked example
(Sec. IV-A LZ/BF example, Sec. V-A-4 scalar multiplication, Sec. V-B-1 mean).
"""
import os

import numpy as np
import pytest

from oracle import ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")


def load_golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = (s.strip() for s in line.split("=", 1))
            vals[k] = v
    return vals


G = load_golden()
EPS = float(G["eps"])
X = np.array([float(v) for v in G["values"].split()], dtype=np.float32)


def ints(key):
    return [int(v) for v in G[key].split()]


def sections(c, L):
    """Split a one-block stream into (W, O, S bytes, P bytes) using the
    section placement rule: 64-byte header, then sections at 16-byte
    boundaries (W: 1 byte, O: 4 bytes, S: L/8 bytes for one block)."""
    off_w = 64
    off_o = 80
    off_s = 96
    off_p = 96 + ((L // 8 + 15) // 16) * 16
    w = int(c[off_w])
    o = int(c[off_o:off_o + 4].view(np.int32)[0])
    return w, o, c[off_s:off_s + L // 8], c[off_p:]


def sign_list(sbytes, n):
    return [(int(sbytes[k // 8]) >> (7 - k % 8)) & 1 for k in range(n)]


@pytest.mark.parametrize("L", [32, 64, 128, 256])
def test_compress_matches_paper_example(L):
    q = ref.quantize(X, EPS)
    assert q.tolist() == ints("bins")
    c = ref.compress(X, EPS, L)
    w, o, s, p = sections(c, L)
    assert o == int(G["outlier"])
    assert w == int(G["width"])
    assert sign_list(s, 4) == ints("signs")
    assert all(b == 0 for b in s.tolist()[1:])
    # the block's 4 magnitudes {0,0,2,0} at width 2 form the byte 0x08
    assert int(p[0]) == int(G["packed_first_byte"], 16)
    assert all(b == 0 for b in p.tolist()[1:])
    assert p.size == L * w // 8


def test_decompress_and_mean_match_paper():
    c = ref.compress(X, EPS, 32)
    y = ref.decompress(c)
    expect = np.array([float(v) for v in G["decompressed"].split()], dtype=np.float32)
    assert np.array_equal(y, expect)
    assert ref.mean(c) == float(G["mean"])
    assert abs(ref.variance(c) - float(G["variance_derived"])) <= 1e-18


def test_scalar_multiplication_matches_paper():
    c = ref.compress(X, EPS, 32)
    m = ref.mul(c, float(G["mul_scalar"]))
    assert ref.decode_bins(m).tolist() == ints("mul_bins")
    w, o, s, p = sections(m, 32)
    assert o == int(G["mul_outlier"])
    assert sign_list(s, 4) == ints("mul_signs")
    # magnitudes {0,0,6,0} at width 3: 000 000 110 000 -> 0x03 0x00
    mags = [(int.from_bytes(bytes(p[:2]), "big") >> (16 - 3 * (k + 1))) & 7 for k in range(4)]
    assert mags == ints("mul_magnitudes")
    assert w == 3


def test_deltas_of_example():
    """Eq. 4 on the example: deltas {0,0,-2,0}, i.e. magnitudes and signs."""
    c = ref.compress(X, EPS, 32)
    bins = ref.decode_bins(c).tolist()
    d = [0] + [bins[k] - bins[k - 1] for k in range(1, 4)]
    assert d == ints("deltas")
    assert [abs(v) for v in d] == ints("magnitudes")
