"""Oracle: a plain CPU computation of the Euler characteristic curve (ECC).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code with
the GPU library (``paper_2203_09087_amd``) and neither imports the other.

The arithmetic lives in ``ecc_oracle.c`` (plain C, one cell at a time, every
cell of the cubical complex enumerated explicitly).  This module only loads the
compiled file and marshals numpy arrays.  The definitions followed are those of
Wang, Wagner and Chen (SoCG 2022): the cubical filtration of Sec. 2.1, the ECC
of Eq. (1), and the VCEC with its prefix sum of Sec. 2.3.  Two filtrations are
offered:

* ``"vertex"`` - voxels are vertices; a cell takes the maximum of its vertices;
* ``"top"``    - voxels are top cells (the paper's Sec. 2.1 construction); a
  cell takes the minimum over the voxels containing it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ecc_oracle.c")
_LIB = os.path.join(_HERE, "libecc_oracle.so")

DTYPES = {np.dtype(np.uint8): 0, np.dtype(np.uint16): 1, np.dtype(np.float32): 2}
CONSTRUCTIONS = {"vertex": 0, "top": 1}
RANGE_DEFAULT, RANGE_EXPLICIT, RANGE_AUTO = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compiles ecc_oracle.c into libecc_oracle.so with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
               "-ffp-contract=off", "-pthread", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        dblp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_bins.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int, ctypes.c_double, ctypes.c_double, i32p, dblp, dblp]
        lib.oracle_bins.restype = ctypes.c_int
        lib.oracle_vcec_from_bins.argtypes = [i32p, ctypes.c_int, i64p, ctypes.c_int32,
                                              ctypes.c_int, ctypes.c_int, i64p]
        lib.oracle_vcec_from_bins.restype = ctypes.c_int
        lib.oracle_prefix.argtypes = [i64p, ctypes.c_int32, i64p]
        lib.oracle_prefix.restype = None
        lib.oracle_ecc.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int32,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, i64p]
        lib.oracle_ecc.restype = ctypes.c_int
        fltp = ctypes.POINTER(ctypes.c_float)
        lib.oracle_smooth13.argtypes = [fltp, fltp, ctypes.c_int64, ctypes.c_int64, fltp]
        lib.oracle_smooth13.restype = ctypes.c_int
        _lib = lib
    return _lib


def _range_args(value_range):
    """None -> DEFAULT, "auto" -> AUTO, (lo, hi) -> EXPLICIT."""
    if value_range is None:
        return RANGE_DEFAULT, 0.0, 0.0
    if isinstance(value_range, str):
        if value_range != "auto":
            raise ValueError(f"unknown range {value_range!r}")
        return RANGE_AUTO, 0.0, 0.0
    lo, hi = value_range
    return RANGE_EXPLICIT, float(lo), float(hi)


def _as_image(image):
    a = np.ascontiguousarray(image)
    if a.dtype not in DTYPES:
        raise TypeError(f"unsupported dtype {a.dtype}")
    if a.ndim < 1 or a.ndim > 8 or a.size == 0:
        raise ValueError(f"unsupported shape {a.shape}")
    return a


def bins(image, nbins: int, value_range=None):
    """Bin of every voxel (int32 array of the image's shape) and the range used."""
    lib = _load()
    a = _as_image(image)
    mode, lo, hi = _range_args(value_range)
    out = np.empty(a.shape, dtype=np.int32)
    lo_used, hi_used = ctypes.c_double(), ctypes.c_double()
    rc = lib.oracle_bins(a.ctypes.data, DTYPES[a.dtype], a.size, int(nbins), mode, lo, hi,
                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                         ctypes.byref(lo_used), ctypes.byref(hi_used))
    if rc != 0:
        raise ValueError("oracle_bins rejected the arguments")
    return out, (lo_used.value, hi_used.value)


def vcec_from_bins(b, nbins: int, construction: str = "vertex", threads: int = 1):
    """VCEC (int64[nbins]) of an integer bin image, every cell enumerated once."""
    lib = _load()
    b = np.ascontiguousarray(b, dtype=np.int32)
    if b.size and (b.min() < 0 or b.max() >= nbins):
        raise ValueError("bins out of range")
    dims = np.array(b.shape, dtype=np.int64)
    out = np.zeros(int(nbins), dtype=np.int64)
    rc = lib.oracle_vcec_from_bins(b.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), b.ndim,
                                   dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(nbins),
                                   CONSTRUCTIONS[construction], int(threads),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError("oracle_vcec_from_bins rejected the arguments")
    return out


def prefix(vcec):
    """ECC_i = sum_{j<=i} VCEC_j."""
    lib = _load()
    v = np.ascontiguousarray(vcec, dtype=np.int64)
    out = np.empty_like(v)
    lib.oracle_prefix(v.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), v.size,
                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


def ecc(image, nbins: int, construction: str = "vertex", value_range=None, threads: int = 1):
    """ECC (int64[nbins]) of a u8/u16/f32 image of 1 to 8 dimensions."""
    lib = _load()
    a = _as_image(image)
    mode, lo, hi = _range_args(value_range)
    dims = np.array(a.shape, dtype=np.int64)
    out = np.zeros(int(nbins), dtype=np.int64)
    rc = lib.oracle_ecc(a.ctypes.data, DTYPES[a.dtype], a.ndim,
                        dims.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(nbins),
                        CONSTRUCTIONS[construction], mode, lo, hi, int(threads),
                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError("oracle_ecc rejected the arguments")
    return out


def vcec(image, nbins: int, construction: str = "vertex", value_range=None, threads: int = 1):
    """VCEC of an image: the bins, then every cell enumerated once."""
    b, _ = bins(image, nbins, value_range)
    return vcec_from_bins(b, nbins, construction, threads)


def smooth13(image, taps):
    """One separable 13-tap smoothing pass of a 2D float32 image (rows, then
    columns; border pixels repeated; float32 sums in tap order)."""
    lib = _load()
    a = np.ascontiguousarray(image, dtype=np.float32)
    w = np.ascontiguousarray(taps, dtype=np.float32)
    if a.ndim != 2 or w.shape != (13,):
        raise ValueError("smooth13 takes a 2D image and 13 taps")
    out = np.empty_like(a)
    fltp = ctypes.POINTER(ctypes.c_float)
    rc = lib.oracle_smooth13(a.ctypes.data_as(fltp), out.ctypes.data_as(fltp), a.shape[0], a.shape[1],
                             w.ctypes.data_as(fltp))
    if rc != 0:
        raise ValueError("oracle_smooth13 rejected the arguments")
    return out
