"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws and shapes input images.  It holds none of the method's
arithmetic (no binning, no cells, no Euler characteristic), so the GPU library,
the oracle and the tests can all take their inputs from it without sharing any
of the computation they check.

The paper measures on uniform noise, Gaussian random fields, breast phantoms and
CMB projections (Sec. 5, "Datasets").  The last two are not available, so every
workload here is synthetic and seeded:

* ``uniform_u8``            - i.i.d. uniform gray levels (the paper's "uniform noise");
* ``smoothed_noise_u8``     - white Gaussian noise smoothed by an isotropic Gaussian,
                              min-max scaled and quantized to 256 levels;
* ``grf``                   - Gaussian random field with power spectrum k^-3 made by
                              filtering white noise in Fourier space (float32);
* ``quantize_u16``          - min-max quantization of a field to ``levels`` levels;
* ``batch_images``          - the uneven 2D/3D batch (sides log-uniform);
* ``serving_requests``      - a Poisson request stream of crops of GRF pools.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft
from scipy import ndimage


def uniform_u8(shape, seed: int) -> np.ndarray:
    """I.i.d. uniform integers in [0, 255]."""
    return np.random.default_rng(seed).integers(0, 256, size=tuple(shape), dtype=np.uint8)


def _minmax_levels(x: np.ndarray, levels: int, dtype) -> np.ndarray:
    lo, hi = float(x.min()), float(x.max())
    if hi <= lo:
        return np.zeros(x.shape, dtype=dtype)
    q = np.floor((x - lo) * (levels / (hi - lo)))
    return np.minimum(q, levels - 1).astype(dtype)


def smoothed_noise_u8(shape, sigma: float, seed: int) -> np.ndarray:
    """White Gaussian noise, isotropic Gaussian smoothing, min-max scaled to 256 levels."""
    x = np.random.default_rng(seed).standard_normal(tuple(shape))
    x = ndimage.gaussian_filter(x, sigma=sigma, mode="reflect", truncate=4.0)
    return _minmax_levels(x, 256, np.uint8)


def grf(shape, seed: int, exponent: float = 3.0) -> np.ndarray:
    """Gaussian random field with power spectrum |k|^-exponent (float32).

    White noise is filtered in Fourier space by |k|^(-exponent/2); the k = 0
    amplitude is set to zero (zero-mean field)."""
    shape = tuple(int(s) for s in shape)
    w = np.random.default_rng(seed).standard_normal(shape, dtype=np.float32)
    F = sfft.rfftn(w, workers=-1)
    del w
    ks = [sfft.fftfreq(n).astype(np.float32) for n in shape[:-1]] + [sfft.rfftfreq(shape[-1]).astype(np.float32)]
    k2 = np.zeros(F.shape, dtype=np.float32)
    for ax, k in enumerate(ks):
        view = [1] * len(shape)
        view[ax] = k.size
        k2 += (k * k).reshape(view)
    with np.errstate(divide="ignore"):
        amp = np.power(k2, np.float32(-exponent / 4.0))   # |k|^(-exponent/2)
    amp.flat[0] = 0.0
    F *= amp
    del amp, k2
    x = sfft.irfftn(F, s=shape, workers=-1)
    return np.ascontiguousarray(x, dtype=np.float32)


def quantize_u16(x: np.ndarray, levels: int) -> np.ndarray:
    """Min-max quantization to integer levels 0..levels-1 (uint16)."""
    return _minmax_levels(x.astype(np.float64, copy=False), levels, np.uint16)


def _log_uniform_side(rng, a: int, b: int) -> int:
    return int(round(math.exp(rng.uniform(math.log(a), math.log(b)))))


def batch_shapes(count: int = 512, frac_2d: float = 0.75, seed: int = 5,
                 side2d=(64, 2048), side3d=(32, 256)):
    """Shapes of the uneven batch: 2D squares and 3D cubes, sides log-uniform."""
    rng = np.random.default_rng(seed)
    n2 = int(round(count * frac_2d))
    kinds = np.array([2] * n2 + [3] * (count - n2))
    rng.shuffle(kinds)
    shapes = []
    for k in kinds:
        if k == 2:
            s = _log_uniform_side(rng, *side2d)
            shapes.append((s, s))
        else:
            s = _log_uniform_side(rng, *side3d)
            shapes.append((s, s, s))
    return shapes


def batch_images(count: int = 512, seed: int = 5, sigma: float = 1.5, **kw):
    """The uneven batch: smoothed-noise uint8 images of the shapes above."""
    shapes = batch_shapes(count=count, seed=seed, **kw)
    out = []
    for i, shp in enumerate(shapes):
        out.append(smoothed_noise_u8(shp, sigma, seed * 100003 + i))
    return out


def serving_requests(rate: float, n_requests: int, seed: int = 6, frac_2d: float = 0.75,
                     side2d=(128, 4096), side3d=(32, 384)):
    """Poisson arrivals (seconds) and request shapes/offsets into the GRF pools."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    reqs = []
    for i in range(n_requests):
        if rng.uniform() < frac_2d:
            s = _log_uniform_side(rng, *side2d)
            off = tuple(int(rng.integers(0, side2d[1] - s + 1)) for _ in range(2))
            reqs.append({"t": float(arrivals[i]), "shape": (s, s), "offset": off})
        else:
            s = _log_uniform_side(rng, *side3d)
            off = tuple(int(rng.integers(0, side3d[1] - s + 1)) for _ in range(3))
            reqs.append({"t": float(arrivals[i]), "shape": (s, s, s), "offset": off})
    return reqs
