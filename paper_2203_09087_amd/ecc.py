"""Python binding of the C ABI in ``include/ecc.h`` (argument marshalling only).

Every step of the computation runs in the HIP library ``libecc_hip.so``; this
module only converts Python/torch arguments to the plain pointers and sizes of
the C entry points, which it exposes under the same names (``ecc_create``,
``ecc_compute``, ``ecc_compute_ex``, ``ecc_compute_batch``, ``ecc_destroy``,
``ecc_last_error``).  There is no fallback: if the library is missing, loading
fails with an error.

``Context`` is a convenience wrapper taking torch tensors that live on the GPU:
the image tensor's memory is passed as the device pointer, the output is an
int64 tensor of ``nbins`` values, and work is enqueued on the current torch
stream unless another is given.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libecc_hip.so")

ECC_OK, ECC_ERR_INVALID_ARG, ECC_ERR_UNSUPPORTED, ECC_ERR_OUT_OF_MEMORY, ECC_ERR_DEVICE = range(5)
ECC_U8, ECC_U16, ECC_F32 = 0, 1, 2
ECC_VERTEX, ECC_TOP = 0, 1
ECC_RANGE_DEFAULT, ECC_RANGE_EXPLICIT, ECC_RANGE_AUTO = 0, 1, 2
ECC_MAX_NDIM = 8   # most dimensions of an image

STATUS_NAMES = {0: "ECC_OK", 1: "ECC_ERR_INVALID_ARG", 2: "ECC_ERR_UNSUPPORTED",
                3: "ECC_ERR_OUT_OF_MEMORY", 4: "ECC_ERR_DEVICE"}
CONSTRUCTIONS = {"vertex": ECC_VERTEX, "top": ECC_TOP}

# Symbols declared in include/ecc.h.
EXPORTED = ("ecc_create", "ecc_destroy", "ecc_last_error", "ecc_compute", "ecc_compute_ex",
            "ecc_compute_batch", "ecc_set_kernel_timing", "ecc_kernel_time", "ecc_batch_plan_create",
            "ecc_batch_plan_launch", "ecc_batch_plan_destroy", "ecc_batch_plan_autotune", "ecc_autotune",
            "ecc_set_launch_shape", "ecc_compute_streamed",
            "ecc_smooth13", "ecc_batch_schedule", "ecc_compute_noalloc", "ecc_reserve")


class ecc_image(ctypes.Structure):
    """Mirror of ``ecc_image`` in include/ecc.h."""
    _fields_ = [
        ("data", ctypes.c_void_p),
        ("ndim", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("dims", ctypes.c_int64 * ECC_MAX_NDIM),
        ("range_mode", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("lo", ctypes.c_double),
        ("hi", ctypes.c_double),
        ("out", ctypes.c_void_p),
    ]


class ecc_batch_shape(ctypes.Structure):
    """Mirror of ``ecc_batch_shape`` in include/ecc.h."""
    _fields_ = [
        ("depth3", ctypes.c_int32),
        ("depth2", ctypes.c_int32),
        ("wgs_per_cu", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("ms", ctypes.c_double),
    ]


class ecc_launch_shape(ctypes.Structure):
    """Mirror of ``ecc_launch_shape`` in include/ecc.h."""
    _fields_ = [
        ("waves", ctypes.c_int32),
        ("wgs_per_cu", ctypes.c_int32),
        ("depth", ctypes.c_int64),
        ("ms", ctypes.c_double),
        ("window", ctypes.c_int32),
        ("copies", ctypes.c_int32),
    ]


class EccError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libecc_hip.so and declares the C signatures.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is not built; run __graft_entry__.build() (hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(path)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)
    lib.ecc_create.argtypes = [ctypes.POINTER(vp), i32, i32]
    lib.ecc_create.restype = ctypes.c_int
    lib.ecc_destroy.argtypes = [vp]
    lib.ecc_destroy.restype = ctypes.c_int
    lib.ecc_last_error.argtypes = [vp]
    lib.ecc_last_error.restype = ctypes.c_char_p
    lib.ecc_compute.argtypes = [vp, vp, i32, i64p, i32, i32, vp, vp]
    lib.ecc_compute.restype = ctypes.c_int
    lib.ecc_compute_ex.argtypes = [vp, ctypes.POINTER(ecc_image), i32, vp]
    lib.ecc_compute_ex.restype = ctypes.c_int
    lib.ecc_compute_noalloc.argtypes = [vp, ctypes.POINTER(ecc_image), i32, vp]
    lib.ecc_compute_noalloc.restype = ctypes.c_int
    lib.ecc_compute_batch.argtypes = [vp, ctypes.POINTER(ecc_image), i32, i32, vp]
    lib.ecc_compute_batch.restype = ctypes.c_int
    lib.ecc_reserve.argtypes = [vp, ctypes.c_size_t, ctypes.c_size_t]
    lib.ecc_reserve.restype = ctypes.c_int
    lib.ecc_set_kernel_timing.argtypes = [vp, i32]
    lib.ecc_set_kernel_timing.restype = ctypes.c_int
    lib.ecc_kernel_time.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i64p]
    lib.ecc_kernel_time.restype = ctypes.c_int
    lib.ecc_batch_plan_create.argtypes = [vp, ctypes.POINTER(ecc_image), i32, i32, ctypes.POINTER(vp)]
    lib.ecc_batch_plan_create.restype = ctypes.c_int
    lib.ecc_batch_plan_launch.argtypes = [vp, vp]
    lib.ecc_batch_plan_launch.restype = ctypes.c_int
    lib.ecc_batch_plan_destroy.argtypes = [vp]
    lib.ecc_batch_plan_autotune.argtypes = [vp, i32, vp, ctypes.POINTER(ecc_batch_shape)]
    lib.ecc_batch_plan_autotune.restype = ctypes.c_int
    lib.ecc_batch_plan_destroy.restype = ctypes.c_int
    lib.ecc_autotune.argtypes = [vp, ctypes.POINTER(ecc_image), i32, i32, vp, ctypes.POINTER(ecc_launch_shape)]
    lib.ecc_autotune.restype = ctypes.c_int
    lib.ecc_set_launch_shape.argtypes = [vp, ctypes.POINTER(ecc_image), i32, ctypes.POINTER(ecc_launch_shape)]
    lib.ecc_set_launch_shape.restype = ctypes.c_int
    lib.ecc_compute_streamed.argtypes = [vp, ctypes.POINTER(ecc_image), i32, ctypes.c_int64, vp]
    lib.ecc_compute_streamed.restype = ctypes.c_int
    fltp = ctypes.POINTER(ctypes.c_float)
    lib.ecc_smooth13.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_int64, fltp, vp]
    lib.ecc_smooth13.restype = ctypes.c_int
    lib.ecc_batch_schedule.argtypes = [ctypes.POINTER(ecc_image), i32, i32, i32, ctypes.POINTER(ecc_batch_shape), i32,
                                       ctypes.POINTER(i32), i64p, i64p, i64p]
    lib.ecc_batch_schedule.restype = ctypes.c_int
    _lib = lib
    return lib


# ----------------------------------------------------------- C entry points

def ecc_create(device: int = 0, construction: int = ECC_VERTEX) -> int:
    lib = load_library()
    h = ctypes.c_void_p()
    st = lib.ecc_create(ctypes.byref(h), int(device), int(construction))
    if st != ECC_OK:
        raise EccError(st, lib.ecc_last_error(None).decode())
    return h.value


def ecc_destroy(ctx: int) -> int:
    return load_library().ecc_destroy(ctx)


def ecc_last_error(ctx) -> str:
    return load_library().ecc_last_error(ctx).decode()


def ecc_compute(ctx: int, image_ptr: int, ndim: int, dims, dtype: int, nbins: int, out_ptr: int,
                stream: int = 0) -> int:
    dims_arr = (ctypes.c_int64 * max(1, len(dims)))(*[int(d) for d in dims])
    return load_library().ecc_compute(ctx, image_ptr, int(ndim), dims_arr, int(dtype), int(nbins),
                                      out_ptr, stream)


def ecc_compute_ex(ctx: int, img: ecc_image, nbins: int, stream: int = 0) -> int:
    return load_library().ecc_compute_ex(ctx, ctypes.byref(img), int(nbins), stream)


def ecc_compute_noalloc(ctx: int, img: ecc_image, nbins: int, stream: int = 0) -> int:
    return load_library().ecc_compute_noalloc(ctx, ctypes.byref(img), int(nbins), stream)


def ecc_compute_batch(ctx: int, imgs, nbins: int, stream: int = 0) -> int:
    """imgs: a list of ecc_image structures or a make_images() array."""
    ptr, keep, n = _descriptor_array(imgs)
    return load_library().ecc_compute_batch(ctx, ptr, n, int(nbins), stream)


def ecc_reserve(ctx: int, scratch_bytes: int, table_bytes: int) -> int:
    return load_library().ecc_reserve(ctx, int(scratch_bytes), int(table_bytes))


def batch_reserve_bytes(count: int, voxels: int, nbins: int, cu_count: int):
    """(scratch_bytes, table_bytes) that cover any ecc_compute_batch call of at most
    `count` images and `voxels` voxels in all (the header's bounds)."""
    w = min(int(nbins), 4096)
    segs = 2 * count + 6 * cu_count + voxels // (1 << 25) + 3
    tables = 2048 + 160 * count + 28 * segs + 24 * cu_count + 24 * (voxels // (1 << 20) + count)
    return 1024 + tables + 4 * w * segs, tables


def ecc_set_kernel_timing(ctx: int, enable: int) -> int:
    return load_library().ecc_set_kernel_timing(ctx, int(enable))


def ecc_kernel_time(ctx: int):
    """(status, total_ms, launches) of the histogram-kernel launches since the last read."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    st = load_library().ecc_kernel_time(ctx, ctypes.byref(ms), ctypes.byref(n))
    return st, ms.value, n.value


def ecc_batch_plan_create(ctx: int, imgs, nbins: int):
    """(status, plan handle or None)."""
    ptr, keep, n = _descriptor_array(imgs)
    h = ctypes.c_void_p()
    st = load_library().ecc_batch_plan_create(ctx, ptr, n, int(nbins), ctypes.byref(h))
    return st, h.value


def ecc_batch_plan_launch(plan: int, stream: int = 0) -> int:
    return load_library().ecc_batch_plan_launch(plan, stream)


def ecc_batch_plan_autotune(plan: int, reps: int, stream: int, shape: ecc_batch_shape) -> int:
    return load_library().ecc_batch_plan_autotune(plan, int(reps), stream, ctypes.byref(shape))


def ecc_batch_plan_destroy(plan: int) -> int:
    return load_library().ecc_batch_plan_destroy(plan)


def ecc_batch_schedule(imgs, nbins: int, shape=None, cu_count: int = 256, construction: int = ECC_VERTEX):
    """Host-only split of a batch (no device needed): (status, segments,
    max_segment_voxels, image_bricks list, covered_bricks list)."""
    ptr, keep, n = _descriptor_array(imgs)
    segs, mx = ctypes.c_int32(), ctypes.c_int64()
    ib, cb = (ctypes.c_int64 * max(1, n))(), (ctypes.c_int64 * max(1, n))()
    sh = ctypes.byref(shape) if shape is not None else None
    st = load_library().ecc_batch_schedule(ptr, n, int(nbins), int(construction), sh, int(cu_count),
                                           ctypes.byref(segs),
                                           ctypes.byref(mx), ib, cb)
    return st, segs.value, mx.value, list(ib)[:n], list(cb)[:n]


def ecc_autotune(ctx: int, img: ecc_image, nbins: int, reps: int, stream: int = 0):
    """(status, ecc_launch_shape)."""
    shape = ecc_launch_shape()
    st = load_library().ecc_autotune(ctx, ctypes.byref(img), int(nbins), int(reps), stream, ctypes.byref(shape))
    return st, shape


def ecc_set_launch_shape(ctx: int, img: ecc_image, nbins: int, waves: int, wgs_per_cu: int, depth: int,
                         window: int = 0, copies: int = 0) -> int:
    shape = ecc_launch_shape(int(waves), int(wgs_per_cu), int(depth), 0.0, int(window), int(copies))
    return load_library().ecc_set_launch_shape(ctx, ctypes.byref(img), int(nbins), ctypes.byref(shape))


def ecc_compute_streamed(ctx: int, img: ecc_image, nbins: int, slab_planes: int = 0, stream: int = 0) -> int:
    return load_library().ecc_compute_streamed(ctx, ctypes.byref(img), int(nbins), int(slab_planes), stream)


def ecc_smooth13(ctx: int, in_ptr: int, out_ptr: int, n1: int, n2: int, taps, stream: int = 0) -> int:
    w = (ctypes.c_float * 13)(*[float(t) for t in taps])
    return load_library().ecc_smooth13(ctx, in_ptr, out_ptr, int(n1), int(n2), w, stream)


# ------------------------------------------------------ torch convenience

def _dtype_code(t) -> int:
    import torch
    codes = {torch.uint8: ECC_U8, torch.uint16: ECC_U16, torch.int16: ECC_U16,
             torch.float32: ECC_F32}
    if t.dtype not in codes:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return codes[t.dtype]


def make_image(t, out, value_range=None) -> ecc_image:
    """Descriptor for a contiguous device tensor ``t`` and int64 output ``out``.

    t: uint8, uint16 (or int16 holding the bits of uint16 data) or float32.
    value_range: None (default range), "auto", or (lo, hi) (explicit)."""
    if not t.is_contiguous():
        raise ValueError("image tensor must be contiguous")
    im = ecc_image()
    im.data = t.data_ptr()
    im.ndim = t.dim()
    im.dtype = _dtype_code(t)
    for i, s in enumerate(t.shape[:ECC_MAX_NDIM]):
        im.dims[i] = int(s)
    im.range_mode, im.lo, im.hi = _range_fields(value_range)
    im.out = out.data_ptr()
    return im


def _range_fields(value_range):
    if value_range is None:
        return ECC_RANGE_DEFAULT, 0.0, 0.0
    if isinstance(value_range, str):
        if value_range != "auto":
            raise ValueError(f"unknown range {value_range!r}")
        return ECC_RANGE_AUTO, 0.0, 0.0
    return ECC_RANGE_EXPLICIT, float(value_range[0]), float(value_range[1])


_RECORD = []


def _image_record():
    """numpy record type with the byte layout of ``ecc_image`` (built once)."""
    if _RECORD:
        return _RECORD[0]
    import numpy as np
    f = {n: getattr(ecc_image, n) for n, _ in ecc_image._fields_}
    _RECORD.append(np.dtype({"names": [n for n, _ in ecc_image._fields_],
                     "formats": [np.uint64, np.int32, np.int32, (np.int64, ECC_MAX_NDIM), np.int32, np.int32, np.float64,
                                 np.float64, np.uint64],
                     "offsets": [f[n].offset for n, _ in ecc_image._fields_],
                     "itemsize": ctypes.sizeof(ecc_image)}))
    return _RECORD[0]


def make_images(tensors, outs, value_ranges=None):
    """Descriptors of many images at once (as make_image, one record each), as a
    numpy array with the layout of an ``ecc_image`` array; much cheaper than one
    ctypes structure per image for large batches."""
    import numpy as np
    import torch
    codes = {torch.uint8: ECC_U8, torch.uint16: ECC_U16, torch.int16: ECC_U16, torch.float32: ECC_F32}
    if value_ranges is None:
        value_ranges = [None] * len(tensors)
    rows = []
    for t, o, r in zip(tensors, outs, value_ranges):
        if not t.is_contiguous():
            raise ValueError("image tensor must be contiguous")
        code = codes.get(t.dtype)
        if code is None:
            raise TypeError(f"unsupported dtype {t.dtype}")
        sh = tuple(t.shape)[:ECC_MAX_NDIM]
        mode, lo, hi = (ECC_RANGE_DEFAULT, 0.0, 0.0) if r is None else _range_fields(r)
        rows.append((t.data_ptr(), len(t.shape), code, sh + (0,) * (ECC_MAX_NDIM - len(sh)), mode, 0, lo, hi,
                     o.data_ptr()))
    return np.array(rows, dtype=_image_record())


def _descriptor_array(imgs):
    """(pointer to ecc_image[], keep-alive object, count) for a list of
    ecc_image structures or a make_images array."""
    if hasattr(imgs, "ctypes") and hasattr(imgs, "dtype"):
        if imgs.dtype.itemsize != ctypes.sizeof(ecc_image) or not imgs.flags["C_CONTIGUOUS"]:
            raise ValueError("descriptor array must be a contiguous make_images() array")
        if len(imgs) == 0:
            keep = (ecc_image * 1)()
            return keep, keep, 0
        return imgs.ctypes.data_as(ctypes.POINTER(ecc_image)), imgs, len(imgs)
    arr = (ecc_image * max(1, len(imgs)))(*imgs)
    return arr, arr, len(imgs)


class Context:
    """Owns an ``ecc_ctx`` on one device for one filtration ("vertex" or "top")."""

    def __init__(self, device: int = 0, construction: str = "vertex"):
        self.device = int(device)
        self.construction = construction
        self.handle = ecc_create(self.device, CONSTRUCTIONS[construction])

    def close(self):
        if self.handle:
            ecc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self, stream):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)

    def _check(self, st):
        if st != ECC_OK:
            raise EccError(st, ecc_last_error(self.handle))

    def compute(self, image, nbins: int, value_range=None, out=None, stream=None):
        """ECC (int64 tensor of nbins) of a device tensor, enqueued on `stream`."""
        import torch
        if out is None:
            out = torch.empty(int(nbins), dtype=torch.int64, device=image.device)
        im = make_image(image, out, value_range)
        self._check(ecc_compute_ex(self.handle, im, nbins, self._stream(stream)))
        return out

    def compute_noalloc(self, image, nbins: int, out, value_range=None, stream=None):
        """As compute(), through the entry point that allocates nothing (its
        scratch is the library's fixed per-device array); `out` is required."""
        im = make_image(image, out, value_range)
        self._check(ecc_compute_noalloc(self.handle, im, nbins, self._stream(stream)))
        return out

    def compute_batch(self, images, nbins: int, value_ranges=None, outs=None, stream=None):
        """ECCs of a list of device tensors in one call; returns the list of outputs."""
        import torch
        if outs is None:
            outs = [torch.empty(int(nbins), dtype=torch.int64, device=t.device) for t in images]
        if value_ranges is None:
            value_ranges = [None] * len(images)
        self._check(ecc_compute_batch(self.handle, make_images(images, outs, value_ranges), nbins,
                                      self._stream(stream)))
        return outs

    def reserve(self, scratch_bytes: int, table_bytes: int = 0):
        """Grows the context's device scratch and pinned table buffers now, so that
        later calls that fit neither allocate nor wait for the device."""
        self._check(ecc_reserve(self.handle, scratch_bytes, table_bytes))

    def set_kernel_timing(self, enable: bool = True):
        """Records HIP events around every histogram-kernel launch of later calls."""
        self._check(ecc_set_kernel_timing(self.handle, 1 if enable else 0))

    def kernel_time(self):
        """(total_ms, launches) of the histogram kernel since the last read; waits for them."""
        st, ms, n = ecc_kernel_time(self.handle)
        self._check(st)
        return ms, n

    def compute_streamed(self, host_image, nbins: int, value_range=None, out=None, slab_planes: int = 0,
                         stream=None):
        """ECC of a CPU tensor (ideally pinned) streamed to the device in slabs of
        the first axis; `out` is a device tensor.  The host tensor must stay
        unchanged until the stream has finished."""
        import torch
        if host_image.is_cuda:
            raise ValueError("compute_streamed takes a host (CPU) tensor")
        if out is None:
            out = torch.empty(int(nbins), dtype=torch.int64, device=torch.device("cuda", self.device))
        im = make_image(host_image, out, value_range)
        self._check(ecc_compute_streamed(self.handle, im, nbins, slab_planes, self._stream(stream)))
        return out

    def smooth13(self, image, taps, out=None, stream=None):
        """One separable 13-tap smoothing pass of a 2D float32 device tensor
        (out may be image itself)."""
        import torch
        if image.dtype != torch.float32 or image.dim() != 2 or not image.is_contiguous():
            raise ValueError("smooth13 takes a contiguous 2D float32 tensor")
        if len(taps) != 13:
            raise ValueError("smooth13 takes 13 taps")
        if out is None:
            out = torch.empty_like(image)
        self._check(ecc_smooth13(self.handle, image.data_ptr(), out.data_ptr(), image.shape[0], image.shape[1],
                                 taps, self._stream(stream)))
        return out

    def autotune(self, image, nbins: int, value_range=None, reps: int = 5, stream=None):
        """Times launch shapes for images shaped like `image` and keeps the fastest
        for later calls on this context; returns the chosen shape as a dict."""
        import torch
        out = torch.empty(int(nbins), dtype=torch.int64, device=image.device)
        st, shape = ecc_autotune(self.handle, make_image(image, out, value_range), nbins, reps,
                                 self._stream(stream))
        self._check(st)
        return {"waves": shape.waves, "wgs_per_cu": shape.wgs_per_cu, "depth": shape.depth, "window": shape.window,
                "copies": shape.copies, "ms": shape.ms}

    def set_launch_shape(self, image, nbins: int, waves: int = 0, wgs_per_cu: int = 0, depth: int = 0,
                         window: int = 0, copies: int = 0, ms=None):
        """Uses the given launch shape (0: default for that field) for later calls
        on images shaped like `image` (a tuned shape from another run)."""
        import torch
        out = torch.empty(1, dtype=torch.int64, device=image.device)
        self._check(ecc_set_launch_shape(self.handle, make_image(image, out, None), nbins, waves, wgs_per_cu,
                                         depth, window, copies))

    def plan_batch(self, images, nbins: int, value_ranges=None, outs=None):
        """A BatchPlan over device tensors (kept alive by the plan object)."""
        return BatchPlan(self, images, nbins, value_ranges, outs)


class BatchPlan:
    """A planned batch on a Context: launch() enqueues kernels only, so it can be
    captured into a HIP graph.  Holds references to its images and outputs."""

    def __init__(self, ctx: Context, images, nbins: int, value_ranges=None, outs=None):
        import torch
        self.ctx = ctx
        self.images = list(images)
        self.outs = outs if outs is not None else [
            torch.empty(int(nbins), dtype=torch.int64, device=t.device) for t in self.images]
        if value_ranges is None:
            value_ranges = [None] * len(self.images)
        st, h = ecc_batch_plan_create(ctx.handle, make_images(self.images, self.outs, value_ranges), nbins)
        ctx._check(st)
        self.handle = h

    def launch(self, stream=None):
        self.ctx._check(ecc_batch_plan_launch(self.handle, self.ctx._stream(stream)))
        return self.outs

    def autotune(self, reps: int = 3, stream=None) -> dict:
        """Times the candidate launch shapes and keeps the fastest (blocking; the
        outputs hold the batch's ECCs afterwards)."""
        sh = ecc_batch_shape()
        self.ctx._check(ecc_batch_plan_autotune(self.handle, reps, self.ctx._stream(stream), sh))
        return {"depth3": sh.depth3, "depth2": sh.depth2, "wgs_per_cu": sh.wgs_per_cu, "ms": sh.ms}

    def close(self):
        if self.handle:
            ecc_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
