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


def test_taps_are_summed_in_order_with_one_rounding_each(oracle_mod):
    """Each output starts at 0, adds tap k times its neighbour for k = 0..12 in that
    order, and rounds every sum to float32.  Taps (1, 2^-25 x 12) on a constant
    image of ones: after the first term the running sum is 1.0, and each further
    term 2^-25 is below half an ulp of 1.0 (2^-24), so it rounds away; the output
    is exactly 1.0 in both passes.  Adding the small taps first (any other order)
    gives 12 * 2^-25 + 1 = 1 + 3 * 2^-23 instead."""
    taps = np.array([1.0] + [2.0 ** -25] * 12, dtype=np.float32)
    img = np.ones((9, 14), dtype=np.float32)
    out = oracle_mod.smooth13(img, taps)
    assert np.array_equal(out, img)


def test_products_are_rounded_before_they_are_added(oracle_mod):
    """Tap 1 is w = 2^-24 (1 + 2^-12) and the pixel it meets is
    b = 1 - 2^-12 + 2^-24, so w * b = 2^-24 (1 + 2^-36) exactly, which rounds to
    2^-24 in float32.  Added to the running sum 1.0 that is an exact tie between
    1.0 and 1 + 2^-23, which rounds to the even 1.0.  A fused multiply-add keeps
    the 2^-60 and rounds up to 1 + 2^-23.

    Image: columns alternate 1.0 (even) and b (odd); odd rows are zero.  For an
    even row y >= 6 the column pass reads tmp[y-6] (tap 0) and a zero row (tap 1),
    so out[y] = tmp[y-6]; for even x >= 6 the row pass gives 1 * 1.0 + w * b -> 1.0,
    and for odd x >= 6 it gives 1 * b + w * 1.0 = b + 2^-24 + 2^-36 -> b + 2^-24."""
    w1 = np.float32(2.0 ** -24 * (1.0 + 2.0 ** -12))
    b = np.float32(1.0 - 2.0 ** -12 + 2.0 ** -24)
    assert float(w1) == 2.0 ** -24 * (1.0 + 2.0 ** -12) and float(b) == 1.0 - 2.0 ** -12 + 2.0 ** -24
    taps = np.zeros(13, dtype=np.float32)
    taps[0], taps[1] = 1.0, w1
    n1, n2 = 20, 24
    img = np.zeros((n1, n2), dtype=np.float32)
    img[0::2, 0::2] = 1.0
    img[0::2, 1::2] = b
    out = oracle_mod.smooth13(img, taps)
    inner = out[6::2, 6:]
    assert np.all(inner[:, 0::2] == np.float32(1.0))
    assert np.all(inner[:, 1::2] == np.float32(float(b) + 2.0 ** -24))
