"""Pins for the FP16 / BF16 storage codec: bit patterns against brute-force rounding
with exact rational arithmetic, and the closed-form decode error bounds."""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import codec, hierarchy as Hh


def _fp16_value(bits):
    s = -1 if bits >> 15 else 1
    e = (bits >> 10) & 0x1F
    m = bits & 0x3FF
    if e == 0:
        return s * Fraction(m, 1 << 24)
    if e == 31:
        return None
    return s * Fraction(1024 + m, 1024) * Fraction(2) ** (e - 15)


def _bf16_value(bits):
    s = -1 if bits >> 15 else 1
    e = (bits >> 7) & 0xFF
    m = bits & 0x7F
    if e == 0 or e == 255:
        return None
    return s * Fraction(128 + m, 128) * Fraction(2) ** (e - 127)


def _brute_round(x, table):
    """Nearest representable value, ties to the even code."""
    fx = Fraction(float(x))
    best = None
    for bits, v in table:
        d = abs(v - fx)
        key = (d, bits & 1)
        if best is None or key < best[0]:
            best = (key, bits)
    return best[1]


def _tables():
    t16 = [(b, _fp16_value(b)) for b in range(1 << 16)]
    t16 = [(b, v) for b, v in t16 if v is not None and not (v == 0 and b == 0x8000)]
    tb = [(b, _bf16_value(b)) for b in range(1 << 16)]
    tb = [(b, v) for b, v in tb if v is not None and abs(v) <= 2]
    return t16, tb


def test_codes_match_brute_force_rounding():
    t16, tb = _tables()
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.uniform(-1, 1, 300), rng.uniform(-1, 1, 100) * 1e-3,
                         [1.0, -1.0, 0.5, 1 - 2 ** -12, 1 + 2 ** -11, 2 ** -13 * 3]])
    # restrict the tables to the neighbourhood of each sample to keep the search small
    v16 = np.array([float(v) for _, v in t16])
    vb = np.array([float(v) for _, v in tb])
    for x in xs:
        near16 = [t16[i] for i in np.argsort(np.abs(v16 - x))[:4]]
        nearb = [tb[i] for i in np.argsort(np.abs(vb - x))[:4]]
        got16 = int(np.array([x]).astype(np.float16).view(np.uint16)[0])
        assert _fp16_value(got16) == _fp16_value(_brute_round(x, near16))
        gotb = int(codec.to_bf16_bits(np.array([x]))[0])
        assert _bf16_value(gotb) == _bf16_value(_brute_round(x, nearb)), x


@pytest.mark.parametrize("fmt,rel", [("fp16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_decode_error_bounds(fmt, rel):
    h = Hh.build(W.c2_td(band_rounds=2, uniform_rounds=1))
    A = h.finest.A
    e, q = codec.encode(A, fmt)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    s = np.ldexp(1.0, e[rows])
    # row scale: s/2 < max |a| <= s
    mx = np.zeros(A.shape[0])
    np.maximum.at(mx, rows, np.abs(A.data))
    assert np.all((mx <= np.ldexp(1.0, e)) & ((mx > np.ldexp(1.0, e - 1)) | (mx == 0)))
    dec = codec.decode_f32(A, e, q, fmt).astype(np.float64)
    a = A.data
    err = np.abs(dec - a)
    normal = np.abs(a) >= (2.0 ** -14) * s if fmt == "fp16" else np.abs(a) >= 2.0 ** -120
    assert np.all(err[normal] <= rel * np.abs(a[normal]))
    assert np.all(err[~normal] <= 2.0 ** -25 * s[~normal])
