"""The stochastic rounding of the binary16 store (LBM_STORE_F16, include/lbmcg.h), checked on the CPU.

The step kernels add a random 13-bit offset to the 13 bits of the scaled FP32 value that binary16
drops, then convert with truncation.  Here a numpy model of those bit operations is compared with
binary16 as numpy defines it (round to nearest): every offset must give the round-to-nearest half
or its neighbour on the value's other side, and the mean over all 8192 offsets must equal the
value wherever binary16 is normal.
"""
import numpy as np
import pytest


def truncate_to_half(x):
    """FP32 -> binary16 with truncation, for values in binary16's normal range (bit model of the
    conversion instruction the kernels use there)."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32)
    sign = (b >> 16) & np.uint32(0x8000)
    e = ((b >> 23) & np.uint32(0xFF)).astype(np.int64) - 127 + 15
    assert np.all((e >= 1) & (e <= 30))
    m = (b >> 13) & np.uint32(0x3FF)
    return (sign | (e.astype(np.uint32) << np.uint32(10)) | m).astype(np.uint16).view(np.float16)


def device_encode_sr(v, scale, r):
    b = (np.asarray(v, dtype=np.float32) * np.float32(scale)).view(np.uint32)
    b = b + (np.asarray(r, dtype=np.uint32) & np.uint32(0x1FFF))
    return truncate_to_half(b.view(np.float32))


def _inputs(scale, n=20000, seed=11):
    rng = np.random.default_rng(seed)
    mags = 10.0 ** rng.uniform(-4.0, 4.2, n) / scale     # scaled values 1e-4 .. 1.6e4: normal halves
    v = np.concatenate([mags, -mags]).astype(np.float32)
    exact = (np.array([1.0, 1.5, 3.0009765625, 1000.5, -7.25], dtype=np.float16).astype(np.float32)
             / np.float32(scale))
    return np.concatenate([v, exact]).astype(np.float32)


@pytest.mark.parametrize("scale", [512.0, 2048.0, 8192.0])
def test_binary16_stochastic_store_rounds_to_a_neighbouring_half(scale):
    v = _inputs(scale)
    x = (v * np.float32(scale)).astype(np.float64)
    near = (v * np.float32(scale)).astype(np.float16).astype(np.float64)
    for r in (0, 1, 255, 4095, 4096, 6000, 8190, 8191):
        got = device_encode_sr(v, scale, np.full(v.shape, r)).astype(np.float64)
        assert np.all(np.sign(got) == np.sign(near))
        # the nearest half, or the next one beyond it on the value's side
        lo = np.minimum(np.abs(near), np.abs(x))
        hi = np.maximum(np.abs(near), np.abs(x))
        ulp = np.abs(np.spacing(np.abs(near).astype(np.float16)).astype(np.float64))
        assert np.all((np.abs(got) >= lo - ulp * (1 + 1e-9)) & (np.abs(got) <= hi + ulp * (1 + 1e-9)))
        exact = x == near
        assert np.all(got[exact] == near[exact])


@pytest.mark.parametrize("scale", [512.0, 2048.0, 8192.0])
def test_binary16_stochastic_store_is_unbiased(scale):
    v = _inputs(scale, n=200, seed=3)
    x = (v * np.float32(scale)).astype(np.float64)
    offsets = np.arange(8192, dtype=np.uint32)
    draws = device_encode_sr(v[None, :], scale, offsets[:, None]).astype(np.float64)
    mean = draws.mean(axis=0)
    # exact in the normal range: the offsets are uniform over the dropped unit
    assert np.allclose(mean, x, rtol=0, atol=0) or np.abs(mean - x).max() <= np.abs(x).max() * 2.0 ** -40
    near = (v * np.float32(scale)).astype(np.float16).astype(np.float64)
    unit = np.spacing(np.abs(near).astype(np.float16)).astype(np.float64)
    assert (np.abs(near - x) / unit).max() > 0.4   # round-to-nearest: up to half a unit
