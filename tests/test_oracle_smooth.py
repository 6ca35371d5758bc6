"""Pins for the oracle's 13-tap smoothing (the smoothing step of the pipeline
workload, Sec. 5).  Expected values come from closed forms that binomial taps
make exact in float32, and from an independent float64 convolution."""
import numpy as np
import pytest
from math import comb

scipy_ndimage = pytest.importorskip("scipy.ndimage")

BINOMIAL = np.array([comb(12, k) for k in range(13)], dtype=np.float64) / 4096.0   # exact in float32


def test_impulse_response_is_the_outer_product(oracle_mod):
    img = np.zeros((31, 40), dtype=np.float32)
    img[15, 20] = 1.0
    out = oracle_mod.smooth13(img, BINOMIAL)
    want = np.zeros_like(img, dtype=np.float64)
    want[9:22, 14:27] = np.outer(BINOMIAL, BINOMIAL)
    assert np.array_equal(out.astype(np.float64), want)


def test_constant_image_is_unchanged(oracle_mod):
    img = np.full((7, 9), 3.0, dtype=np.float32)
    assert np.array_equal(oracle_mod.smooth13(img, BINOMIAL), img)


def test_border_pixels_repeat(oracle_mod):
    # a single row: columns add nothing (every row index clamps to row 0)
    row = np.zeros((1, 20), dtype=np.float32)
    row[0, 0] = 1.0
    out = oracle_mod.smooth13(row, BINOMIAL)[0]
    # out[x] = sum of the taps whose neighbour clamps onto column 0: x + k - 6 <= 0
    want = np.array([BINOMIAL[: max(0, 7 - x)].sum() for x in range(20)])
    assert np.array_equal(out.astype(np.float64), want)


def test_matches_a_float64_convolution(oracle_mod):
    rng = np.random.default_rng(7)
    img = rng.standard_normal((50, 61)).astype(np.float32)
    taps = np.exp(-0.5 * (np.arange(13) - 6.0) ** 2 / 4.0)
    taps = (taps / taps.sum()).astype(np.float32)
    out = oracle_mod.smooth13(img, taps)
    w = taps.astype(np.float64)[::-1]   # correlate = convolve with the reversed kernel
    ref = scipy_ndimage.convolve1d(img.astype(np.float64), w, axis=1, mode="nearest")
    ref = scipy_ndimage.convolve1d(ref, w, axis=0, mode="nearest")
    assert np.allclose(out, ref, rtol=0, atol=2e-6)


def test_asymmetric_taps_select_the_right_neighbours(oracle_mod):
    # one tap at k = 12 picks the neighbour 6 to the right (rows) and 6 below (columns)
    taps = np.zeros(13, dtype=np.float32)
    taps[12] = 1.0
    rng = np.random.default_rng(8)
    img = rng.standard_normal((20, 25)).astype(np.float32)
    out = oracle_mod.smooth13(img, taps)
    ys = np.minimum(np.arange(20) + 6, 19)
    xs = np.minimum(np.arange(25) + 6, 24)
    assert np.array_equal(out, img[np.ix_(ys, xs)])
