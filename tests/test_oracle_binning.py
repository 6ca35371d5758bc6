"""Pins for the oracle's binning (value -> bin), the library's reading of how the
paper's gray-level histogram index (Sec. 4, Algorithm 2: 0..255 levels) extends
to 16-bit and float data.

Expected bins are written out by hand from the stated rules:
  integer data, range [lo, hi]:  ((clamp(v, lo, hi) - lo) * nbins) // (hi - lo + 1)
  float data, range [lo, hi]:    NaN -> nbins-1; hi == lo -> (x > hi ? nbins-1 : 0);
                                 else clamp(floor((x - lo) * nbins / (hi - lo)), 0, nbins-1)
"""
import numpy as np
import pytest


def _bins(oracle_mod, values, dtype, nbins, rng=None):
    a = np.array(values, dtype=dtype)
    b, used = oracle_mod.bins(a, nbins, rng)
    return b.tolist(), used


def test_u8_default_is_identity(oracle_mod):
    v = list(range(256))
    b, used = _bins(oracle_mod, v, np.uint8, 256)
    assert b == v and used == (0.0, 255.0)


def test_u8_coarse_bins(oracle_mod):
    # 4 bins over [0, 255]: 64 gray levels each
    b, _ = _bins(oracle_mod, [0, 63, 64, 127, 128, 191, 192, 255], np.uint8, 4)
    assert b == [0, 0, 1, 1, 2, 2, 3, 3]


def test_u16_explicit_range_and_clamp(oracle_mod):
    # [10, 19] is 10 levels onto 5 bins: two levels per bin; outside values clamp
    b, _ = _bins(oracle_mod, [0, 9, 10, 11, 12, 17, 18, 19, 20, 65535], np.uint16, 5, (10, 19))
    assert b == [0, 0, 0, 0, 1, 3, 4, 4, 4, 4]


def test_u16_more_bins_than_levels(oracle_mod):
    # 3 levels onto 7 bins: level a goes to floor(a * 7 / 3)
    b, _ = _bins(oracle_mod, [100, 101, 102], np.uint16, 7, (100, 102))
    assert b == [0, 2, 4]


def test_u16_auto_range(oracle_mod):
    b, used = _bins(oracle_mod, [300, 301, 302, 303], np.uint16, 4, "auto")
    assert used == (300.0, 303.0) and b == [0, 1, 2, 3]
    b, used = _bins(oracle_mod, [7, 7, 7], np.uint16, 16, "auto")
    assert used == (7.0, 7.0) and b == [0, 0, 0]


def test_f32_explicit(oracle_mod):
    nan, inf = float("nan"), float("inf")
    vals = [0.0, 0.2499, 0.25, 0.5, 0.75, 0.99, 1.0, 1.5, -0.1, nan, inf, -inf, -0.0]
    b, _ = _bins(oracle_mod, vals, np.float32, 4, (0.0, 1.0))
    assert b == [0, 0, 1, 2, 3, 3, 3, 3, 0, 3, 3, 0, 0]


def test_f32_auto_ignores_non_finite(oracle_mod):
    nan, inf = float("nan"), float("inf")
    b, used = _bins(oracle_mod, [2.0, 4.0, 3.0, nan, inf, -inf], np.float32, 2, "auto")
    assert used == (2.0, 4.0)
    assert b == [0, 1, 1, 1, 1, 0]
    b, used = _bins(oracle_mod, [nan, nan], np.float32, 8, "auto")
    assert used == (0.0, 0.0) and b == [7, 7]


def test_f32_flat_range(oracle_mod):
    b, _ = _bins(oracle_mod, [1.0, 0.5, 1.5, float("inf"), float("-inf")], np.float32, 8, (1.0, 1.0))
    assert b == [0, 0, 7, 7, 0]


def test_f32_binning_is_monotone(oracle_mod):
    rng = np.random.default_rng(3)
    x = np.sort(np.concatenate([rng.standard_normal(5000), rng.uniform(-3, 3, 5000)]).astype(np.float32))
    b, _ = oracle_mod.bins(x, 97, (-2.5, 2.5))
    assert np.all(np.diff(b) >= 0) and b.min() == 0 and b.max() == 96


def test_bins_commute_with_cell_values(oracle_mod):
    """Binning is monotone, so the ECC of a float image equals the ECC of its bin
    image, and a cell's bin is the max (vertex) / min (top) of its voxels' bins."""
    rng = np.random.default_rng(4)
    img = rng.standard_normal((9, 11, 7)).astype(np.float32)
    for cons in ("vertex", "top"):
        direct = oracle_mod.ecc(img, 33, cons, (-1.0, 1.2))
        b, _ = oracle_mod.bins(img, 33, (-1.0, 1.2))
        via = oracle_mod.prefix(oracle_mod.vcec_from_bins(b, 33, cons))
        assert np.array_equal(direct, via)


@pytest.mark.parametrize("args", [
    dict(nbins=0), dict(nbins=65536), dict(dtype=np.uint8, rng=(0, 256)),
    dict(dtype=np.uint8, rng=(3.5, 10)), dict(dtype=np.uint16, rng=(5, 4)),
    dict(dtype=np.float32, rng=(0.0, float("inf"))), dict(dtype=np.float32, rng=(2.0, 1.0)),
])
def test_bad_arguments_are_rejected(oracle_mod, args):
    a = np.zeros(4, dtype=args.get("dtype", np.uint8))
    with pytest.raises(ValueError):
        oracle_mod.bins(a, args.get("nbins", 8), args.get("rng"))


# ---------------------------------------------------------------------------
# Float binning near bin boundaries, against exact rational arithmetic.
#
# The reading of the gray-level histogram index for float data (Sec. 4 and
# Algorithm 2 use 0..255 levels) is t = ((double)x - lo) * (nbins / (hi - lo))
# with every operation rounded once in IEEE double, bin = clamp(floor(t)).  Those
# three roundings move t by at most about 4 * 2^-53 * t <= 3e-11 for nbins <= 65535,
# so wherever the exact rational value of (x - lo) * nbins / (hi - lo) lies at least
# 1e-9 away from an integer, the bin is the exact floor.  The cases below take
# float32 values adjacent to exact bin boundaries, where the exact value lies within
# about one float32 ulp of an integer: a computation carried out in float32 (or with
# a coarser scale) lands on the wrong side of the boundary for many of them.
from fractions import Fraction  # noqa: E402


def _boundary_cases(seed, groups=40, per_group=48):
    """(x float32 array, lo, hi, nbins, expected bins) groups whose expected bins
    come from fractions.Fraction alone."""
    rng = np.random.default_rng(seed)
    out = []
    for g in range(groups):
        nbins = int(rng.choice([7, 97, 256, 1000, 4096, 4095, 65535]))
        if g % 3 == 0:
            # float32 range ends, as an AUTO range over float32 data produces them
            lo = float(np.float32(rng.uniform(-500.0, 500.0)))
            hi = float(np.float32(lo + 10.0 ** rng.uniform(-2, 4)))
        else:
            # arbitrary double range ends (an explicit range)
            lo = float(rng.uniform(-50.0, 50.0))
            hi = lo + float(10.0 ** rng.uniform(-1, 3))
        if not hi > lo:
            continue
        flo, fhi = Fraction(lo), Fraction(hi)
        xs, want = [], []
        for j in rng.integers(1, nbins, size=per_group):
            edge = flo + (fhi - flo) * int(j) / nbins          # exact boundary of bin j
            x0 = np.float32(float(edge))
            for x in (np.nextafter(x0, np.float32(-np.inf)), x0, np.nextafter(x0, np.float32(np.inf))):
                t = (Fraction(float(x)) - flo) * nbins / (fhi - flo)
                dist = abs(t - round(t))
                if dist < Fraction(1, 10 ** 9) or dist > Fraction(1, 10 ** 3):
                    continue
                b = t.numerator // t.denominator                # floor of the exact value
                xs.append(x)
                want.append(min(max(b, 0), nbins - 1))
        if xs:
            out.append((np.array(xs, dtype=np.float32), lo, hi, nbins, np.array(want)))
    return out


def test_f32_bins_near_boundaries_are_the_exact_floor(oracle_mod):
    total = 0
    for xs, lo, hi, nbins, want in _boundary_cases(11):
        got, used = oracle_mod.bins(xs, nbins, (lo, hi))
        assert used == (lo, hi)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (f"nbins={nbins} range=({lo!r}, {hi!r}): x={xs[bad[0]]!r} "
                               f"bin {got[bad[0]]} != exact {want[bad[0]]}")
        total += xs.size
    assert total > 3000


def test_boundary_cases_separate_double_from_float32_arithmetic():
    """The cases above have teeth: the same formula evaluated in float32
    (subtraction and product rounded to float32) misplaces some of them."""
    wrong = 0
    for xs, lo, hi, nbins, want in _boundary_cases(11):
        d = xs - np.float32(lo)
        t = d * np.float32(nbins / (hi - lo))
        b = np.clip(np.floor(t.astype(np.float64)), 0, nbins - 1).astype(np.int64)
        wrong += int(np.count_nonzero(b != want))
    assert wrong > 50
