"""The 16-bit population format of LBM_STORE_C16 (include/lbmcg.h), checked on the CPU.

The format: sign, 4-bit exponent e with bias 7, 11-bit fraction f; value 2^(e-7) (1 + f/2^11)
for e >= 1 and 2^-6 f/2^11 for e = 0.  The device decodes it with FP32 bit operations (the
exponent-and-fraction bits shifted into an FP32 word, then one multiplication) and stores it
with stochastic rounding.  Here numpy models of those bit operations are compared with the
format's definition evaluated in exact rational arithmetic, so that an off-by-one shift, a wrong
rounding bias or a lost subnormal in the bit trick fails a test.  Round-to-nearest (ties to
even) is the format's nominal rounding, the one the host applies to the initial state; its
bit model below is the reference the stochastic store is checked against.
"""
from fractions import Fraction

import numpy as np
import pytest

MAXV = Fraction(2) ** 9 - Fraction(2) ** -3  # 2^8 (1 + 2047/2048)


def exact_value(bits):
    s = -1 if bits & 0x8000 else 1
    e, f = (bits >> 11) & 0xF, bits & 0x7FF
    if e == 0:
        return s * Fraction(2) ** -6 * Fraction(f, 2048)
    return s * Fraction(2) ** (e - 7) * (1 + Fraction(f, 2048))


def exact_encode(x):
    """Nearest representable value, ties to the even fraction; saturating."""
    x = Fraction(x)
    sign = 0x8000 if x < 0 else 0
    a = abs(x)
    if a >= MAXV:
        return sign | 0x7FFF
    best = None
    # candidates: every code is monotone in its 15 low bits, so bisect on them
    lo, hi = 0, 0x7FFF
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if exact_value(mid) <= a:
            lo = mid
        else:
            hi = mid
    dl, dh = a - exact_value(lo), exact_value(hi) - a
    if dl < dh or (dl == dh and lo % 2 == 0):
        best = lo
    else:
        best = hi
    return sign | best


def device_decode(bits, scale_exp):
    """numpy model of the device decode: bits << 12 into an FP32 word, times 2^(127-7-k)."""
    bits = np.asarray(bits, dtype=np.uint32)
    w = ((bits & 0x7FFF) << 12) | ((bits & 0x8000) << 16)
    f = w.view(np.float32)
    return f * np.float32(2.0 ** (120 - scale_exp))


def device_encode(v, scale_exp):
    """Round-to-nearest-even to the format by FP32 bit operations (FP32 multiply, integer
    increment of the magnitude); checked against the exact definition below."""
    t = (np.asarray(v, dtype=np.float32) * np.float32(2.0 ** (scale_exp - 120))).view(np.uint32)
    mag = t & np.uint32(0x7FFFFFFF)
    r = np.minimum((mag + np.uint32(0x7FF) + ((mag >> 12) & 1)) >> 12, 0x7FFF)
    return (r | ((t >> 16) & 0x8000)).astype(np.uint16)


def device_encode_sr(v, scale_exp, r):
    """numpy model of the step kernels' stochastic-rounding store: the scaled FP32 value clamped
    to +-0x07FFF000 (as bits) by a median of three, a random 12-bit offset r (0 .. 4095) added to
    the 12 dropped bits of the signed word, the sign moved to bit 15; the lower 16 bits are
    stored."""
    x = np.asarray(v, dtype=np.float32) * np.float32(2.0 ** (scale_exp - 120))
    top = np.uint32(0x07FFF000).view(np.float32)
    x = np.clip(x, -top, top)
    t = x.view(np.uint32) + (np.asarray(r, dtype=np.uint32) & np.uint32(0xFFF))
    return ((t >> 12) | ((t >> 16) & np.uint32(0x8000))).astype(np.uint16)


def _sr_inputs(scale_exp, n=20000, seed=2024):
    rng = np.random.default_rng(seed)
    S = 2.0 ** scale_exp
    mags = 10.0 ** rng.uniform(-12, 1.0, n) / S * 2.0 ** 8
    exact = [float(exact_value(c) / Fraction(2) ** scale_exp) for c in (1, 5, 2047, 2048, 12345, 0x7FFE)]
    vals = np.concatenate([mags, exact, [0.0, 1e-38, 1e30]]).astype(np.float32)
    return np.concatenate([vals, -vals])


@pytest.mark.parametrize("scale_exp", [9, 11, 13])
def test_stochastic_store_rounds_to_a_neighbouring_code(scale_exp):
    """For every random offset the stored code is one of the two codes next to the value: the
    round-to-nearest code or its neighbour on the value's other side (so the error is below one
    unit); exact codes stay exact, and values beyond the range saturate."""
    vals = _sr_inputs(scale_exp)
    rne = device_encode(vals, scale_exp).astype(np.int64)
    dec_rne = device_decode(rne.astype(np.uint32), scale_exp).astype(np.float64)
    above = np.abs(vals.astype(np.float64)) > np.abs(dec_rne)
    for r in (0, 1, 127, 2047, 2048, 3000, 4094, 4095):
        got = device_encode_sr(vals, scale_exp, np.full(vals.shape, r)).astype(np.int64)
        # same sign bit, magnitude code within one of the nearest one, on the value's side
        assert np.array_equal(got & 0x8000, rne & 0x8000)
        step = (got & 0x7FFF) - (rne & 0x7FFF)
        assert np.all(np.abs(step) <= 1)
        assert np.all((step >= 0) | ~above) and np.all((step <= 0) | above)
        assert np.all(step[np.abs(vals.astype(np.float64)) == np.abs(dec_rne)] == 0)
    big = np.array([1e6, -1e6], dtype=np.float32) / np.float32(2.0 ** scale_exp)
    assert list(device_encode_sr(big, scale_exp, [4095, 4095])) == [0x7FFF, 0xFFFF]


@pytest.mark.parametrize("scale_exp", [9, 11, 13])
def test_stochastic_store_is_unbiased(scale_exp):
    """Averaged over all 4096 equally likely offsets the decoded value equals the input (below
    the smallest normal code the scaled FP32 product is itself rounded on a grid 2^12 finer,
    which leaves up to 2^-13 of a unit), where round-to-nearest is off by up to half a unit:
    rounding errors carry no systematic part."""
    vals = _sr_inputs(scale_exp, n=300, seed=7)
    offsets = np.arange(4096, dtype=np.uint32)
    codes = device_encode_sr(vals[None, :], scale_exp, offsets[:, None])
    mean = device_decode(codes.astype(np.uint32), scale_exp).astype(np.float64).mean(axis=0)
    rne = device_encode(vals, scale_exp).astype(np.uint32)
    nxt = device_decode((rne & 0x8000) | np.minimum((rne & 0x7FFF) + 1, 0x7FFF), scale_exp).astype(np.float64)
    unit = np.abs(nxt - device_decode(rne, scale_exp).astype(np.float64))
    inrange = (rne & 0x7FFF) < 0x7FFE
    v = vals.astype(np.float64)
    assert np.all(np.abs(mean - v)[inrange] <= unit[inrange] * 2.0 ** -13 * (1 + 1e-6) + 1e-300)
    near = device_decode(rne, scale_exp).astype(np.float64)
    assert (np.abs(near - v)[inrange] / unit[inrange]).max() > 0.4


@pytest.mark.parametrize("scale_exp", [9, 11, 13])
def test_decode_matches_definition_for_every_code(scale_exp):
    codes = np.arange(0x10000, dtype=np.uint32)
    got = device_decode(codes, scale_exp).astype(np.float64)
    for c in list(range(0, 0x10000, 97)) + [0, 1, 2047, 2048, 2049, 0x7FFF, 0x8001, 0xFFFF]:
        want = exact_value(c) / Fraction(2) ** scale_exp
        assert Fraction(float(got[c])) == want, hex(c)


@pytest.mark.parametrize("scale_exp", [9, 11, 13])
def test_encode_is_round_to_nearest_even(scale_exp):
    rng = np.random.default_rng(1707)
    S = 2.0 ** scale_exp
    # deviations spanning subnormals, normals and saturation, both signs, plus exact ties
    mags = 10.0 ** rng.uniform(-9, 0.5, 4000) / S * 2.0 ** 8
    vals = np.concatenate([mags, -mags, [0.0, 1e-30]]).astype(np.float32)
    ties = [(exact_value(c) + exact_value(c + 1)) / 2 / Fraction(2) ** scale_exp
            for c in (5, 6, 2047, 2048, 4095, 12345, 0x7FFE)]
    vals = np.concatenate([vals, np.array([float(t) for t in ties], dtype=np.float32)])
    got = device_encode(vals, scale_exp)
    for v, g in zip(vals, got):
        want = exact_encode(Fraction(float(v)) * Fraction(2) ** scale_exp)
        assert int(g) == want, (float(v), hex(int(g)), hex(want))


def test_relative_error_bound_and_saturation():
    rng = np.random.default_rng(7)
    for k in (9, 11, 13):
        S = 2.0 ** k
        sign = rng.choice([-1.0, 1.0], 20000)
        # normal range: relative error at most half an ulp, 2^-12
        v = (sign * 2.0 ** rng.uniform(-6, 8.99, 20000) / S).astype(np.float32)
        back = device_decode(device_encode(v, k), k).astype(np.float64)
        rel = np.abs(back - v.astype(np.float64)) / np.abs(v.astype(np.float64))
        assert rel.max() <= 2.0 ** -12 * (1 + 1e-9)
        # subnormal range: absolute error at most half the subnormal step 2^-17 / S, plus the
        # FP32 subnormal rounding of the scaling product (a grid 2^12 times finer) that the
        # device codec rounds first: 2^-29 / S
        v = (sign * 2.0 ** rng.uniform(-30, -6, 20000) / S).astype(np.float32)
        back = device_decode(device_encode(v, k), k).astype(np.float64)
        assert np.abs(back - v.astype(np.float64)).max() <= (2.0 ** -18 + 2.0 ** -29) / S
        big = np.array([1e6 / S, -1e6 / S], dtype=np.float32)
        assert np.allclose(device_decode(device_encode(big, k), k), [float(MAXV) / S, -float(MAXV) / S])
