/*
 * ecc.h -- C ABI of the MI355X (gfx950) library that computes the Euler
 * characteristic curve (ECC) of 2D and 3D grayscale images.
 *
 * Method (Wang, Wagner, Chen, "GPU Computation of the Euler Characteristic Curve
 * for Imaging Data", SoCG 2022):
 *   - Sec. 2.1: the image is a d-dimensional array of values; thresholding at t
 *     keeps the part of a cubical complex with filtration value <= t.
 *   - Eq. (1):  ECC_i = chi(K_{<=t_i}) = sum_j (-1)^j c_j(K_{<=t_i}).
 *   - Sec. 2.3: VCEC_i = ECC_i - ECC_{i-1}; every cell is credited, with sign
 *     (-1)^dim, to the voxel that completes it (Algorithm 1), and the ECC is the
 *     prefix sum of the VCEC.
 * The curve is indexed by integer bins: out[i] = chi of the cells whose value
 * falls in bins 0..i (empty bins included, so out has exactly nbins entries).
 *
 * Two filtrations (ecc_construction):
 *   ECC_VERTEX (default) - voxels are the vertices of the complex; a cell (a block
 *                          of 2^k voxels) takes the maximum value of its vertices;
 *   ECC_TOP              - voxels are the top-dimensional cells, as in the paper's
 *                          Sec. 2.1; a lower cell takes the minimum value of the
 *                          voxels that contain it.
 *
 * Binning of values into [0, nbins):
 *   integer data (ECC_U8, ECC_U16), integer range [lo, hi]:
 *       bin = ((clamp(v, lo, hi) - lo) * nbins) / (hi - lo + 1)       (exact)
 *   float data (ECC_F32), range [lo, hi]:
 *       NaN -> nbins-1;  hi == lo -> (x > hi ? nbins-1 : 0);  otherwise
 *       bin = clamp(floor(((double)x - lo) * s), 0, nbins-1) with
 *       s = (double)nbins / (hi - lo); every operation is one IEEE double
 *       rounding, no fused multiply-add.
 *   Range modes: ECC_RANGE_DEFAULT = [0,255] for u8 and AUTO otherwise;
 *   ECC_RANGE_AUTO = [min, max] of the image, computed on the device (finite
 *   values only for f32; [0,0] when there are none); ECC_RANGE_EXPLICIT = [lo, hi]
 *   from the caller (integers inside the type's range for u8/u16, finite for f32).
 *
 * Conventions shared by every entry point:
 *   - Images are DEVICE pointers, contiguous, row-major, dims[0] slowest.  Any
 *     alignment is accepted.  ndim is 2 to ECC_MAX_NDIM (see ecc_compute for
 *     images of 4 or more dimensions); entry points that do not take a
 *     dimension return ECC_ERR_UNSUPPORTED for it: the batch calls, plans,
 *     ecc_compute_noalloc and ecc_compute_streamed take 2 to 4.  Every dim is
 *     >= 1.
 *   - `out` is a DEVICE pointer to nbins int64 values, overwritten (not
 *     accumulated) with the ECC.  1 <= nbins <= 65535.
 *   - Every call validates all of its arguments on the host before anything is
 *     enqueued; a call that returns an error has enqueued nothing.  Successful
 *     calls are asynchronous on `hip_stream` (a hipStream_t; NULL = the null
 *     stream); results are valid once that stream has completed the work.
 *   - The caller owns images and outputs and keeps them alive until the stream
 *     has finished.  The context owns its device scratch memory, which it grows
 *     with hipMalloc when a call needs more than it holds.
 *   - A context is used by one host thread at a time.  Calls on one context that
 *     are enqueued on different streams must not overlap in time (they share the
 *     context's scratch memory).
 *   - No C++ exception crosses this interface; ecc_last_error() gives the text of
 *     the last error of a context.
 */
#ifndef ECC_H
#define ECC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ecc_ctx ecc_ctx;

typedef enum {
    ECC_OK = 0,
    ECC_ERR_INVALID_ARG = 1,   /* a null pointer, a bad size, range or enum value */
    ECC_ERR_UNSUPPORTED = 2,   /* a valid request the library does not serve */
    ECC_ERR_OUT_OF_MEMORY = 3, /* device scratch memory could not be allocated */
    ECC_ERR_DEVICE = 4         /* a HIP runtime call failed */
} ecc_status;

typedef enum { ECC_U8 = 0, ECC_U16 = 1, ECC_F32 = 2 } ecc_dtype;

/* Most dimensions of an image (the cubical complex of Sec. 2.1 is defined in
 * every dimension). */
#define ECC_MAX_NDIM 8

typedef enum { ECC_VERTEX = 0, ECC_TOP = 1 } ecc_construction;

typedef enum {
    ECC_RANGE_DEFAULT = 0,
    ECC_RANGE_EXPLICIT = 1,
    ECC_RANGE_AUTO = 2
} ecc_range_mode;

/* One image of a call.  Enum-valued fields are int32_t for a fixed layout. */
typedef struct {
    const void* data;    /* device pointer to the voxels */
    int32_t ndim;        /* 2 .. ECC_MAX_NDIM, as the entry point takes them */
    int32_t dtype;       /* ecc_dtype */
    int64_t dims[ECC_MAX_NDIM]; /* dims[0] slowest; entries beyond ndim are ignored */
    int32_t range_mode;  /* ecc_range_mode */
    int32_t reserved;    /* must be 0 */
    double lo, hi;       /* used with ECC_RANGE_EXPLICIT only */
    int64_t* out;        /* device pointer, nbins int64, overwritten with the ECC */
} ecc_image;

/* Creates a context on HIP device `device` for filtration `construction`
 * (ecc_construction).  Sec. 2.1 defines the filtration; the vertex variant is the
 * library's default reading.  On success *ctx owns no device memory yet.
 * Errors: ECC_ERR_INVALID_ARG (ctx null, bad enum), ECC_ERR_DEVICE (no such
 * device), ECC_ERR_OUT_OF_MEMORY (host allocation failed). */
ecc_status ecc_create(ecc_ctx** ctx, int32_t device, int32_t construction);

/* Releases the context and its device memory.  Waits for nothing: the caller
 * must have synchronized every stream the context enqueued work on.  A null
 * ctx is accepted and ignored. */
ecc_status ecc_destroy(ecc_ctx* ctx);

/* Grows the context's device scratch to at least scratch_bytes and each of its
 * pinned table buffers (host memory the batch descriptors are staged in before
 * their copy to the device) to at least table_bytes, now, so that later calls
 * whose needs fit neither allocate nor wait: growing the scratch inside a call
 * waits for the whole device (the old buffer may still be in use on any
 * stream), which a serving loop with several streams cannot afford.  This call
 * itself may wait for the device.  Generous bounds for a batch
 * (ecc_compute_batch) of n images of V voxels in all, with W = min(nbins, 4096)
 * and C compute units: at most S = 2 n + 6 C + V / 2^25 + 3 workgroup segments;
 * tables <= 2 KiB + 160 n + 28 S + 24 C + 24 (V / 2^20 + n) bytes; scratch <=
 * 1 KiB + tables + 4 W S bytes.  A single image needs less scratch than a
 * batch of it.
 * Calls that need more still work, growing the buffers as before.
 * Errors: ECC_ERR_INVALID_ARG (ctx null, scratch_bytes > 2^40 or table_bytes >
 * 2^30), ECC_ERR_OUT_OF_MEMORY, ECC_ERR_DEVICE. */
ecc_status ecc_reserve(ecc_ctx* ctx, size_t scratch_bytes, size_t table_bytes);

/* Text of the last error recorded on `ctx` ("" if none); valid until the next
 * call on the same context.  A null ctx returns the last ecc_create error. */
const char* ecc_last_error(const ecc_ctx* ctx);

/* ECC of one image with the default range (Eq. (1), Sec. 2.3).
 * image: device pointer; ndim 2 .. ECC_MAX_NDIM; dims: HOST pointer to ndim
 * int64; dtype: ecc_dtype; out: device pointer to nbins int64 (overwritten).
 * A 4D image (the cubical complex of Sec. 2.1 in four dimensions) is computed as
 * signed 3D passes over its hyperplanes dims[0] and over the elementwise max
 * (vertex) or min (top) of adjacent hyperplanes.  An image of five or more
 * dimensions is reduced the same way one axis at a time down to 4D: each
 * hyperplane of axis 0 and the elementwise max (min) of each adjacent pair,
 * the latter written into the context's scratch (one hyperplane per reduced
 * axis), is a (d-1)-dimensional image counted with its sign; the 3D passes
 * number prod over the first d-3 axes of (2 dims[i] - 1).
 * Errors: ECC_ERR_INVALID_ARG for any bad argument (nothing enqueued),
 * ECC_ERR_OUT_OF_MEMORY, ECC_ERR_DEVICE. */
ecc_status ecc_compute(ecc_ctx* ctx, const void* image, int32_t ndim, const int64_t* dims,
                       int32_t dtype, int32_t nbins, int64_t* out, void* hip_stream);

/* ECC of one image described by `img` (HOST pointer to the descriptor; its data
 * and out fields are device pointers).  Same semantics and errors as ecc_compute
 * (ndim 2 .. ECC_MAX_NDIM), plus the range selection of the descriptor; an AUTO
 * range of an image of 4 or more dimensions is the min/max of all its voxels. */
ecc_status ecc_compute_ex(ecc_ctx* ctx, const ecc_image* img, int32_t nbins, void* hip_stream);

/* ecc_compute_ex for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, semantics, results and errors as ecc_compute_ex
 * (ndim 2 to 4; ECC_ERR_UNSUPPORTED for more), but the call allocates nothing (no hipMalloc/hipFree, no
 * allocating library routine): its scratch is a fixed array of 24 MiB
 * (kNoAllocBytes) that the library keeps on each device it runs on, set up by
 * the first ecc_create on that device and held until the process ends.  The
 * context's own scratch is not used.  All calls on one device share that
 * array, so calls that overlap in time on one device (any context, any
 * stream) race and give wrong results: the caller serialises them.  The
 * launch grid is narrowed to fit the array; an image that cannot fit (more than
 * about 2^38 voxels) is refused with ECC_ERR_UNSUPPORTED before anything is
 * enqueued.  Asynchronous on hip_stream like ecc_compute_ex. */
ecc_status ecc_compute_noalloc(ecc_ctx* ctx, const ecc_image* img, int32_t nbins, void* hip_stream);

/* ECC of `count` images in one persistent histogram launch per dtype present
 * (then one merge and one scan launch for all images).  imgs: HOST array of `count`
 * descriptors; images may differ in ndim, dtype, size and range mode but share
 * nbins and the context's filtration; each writes its own `out`.  A 4D image
 * enters as its signed 3D passes (hyperplanes and adjacent max/min pairs, as in
 * ecc_compute), each counted like a 3D image of the batch into rows of its own
 * image.  The result of every image is identical to what ecc_compute_ex returns
 * for it alone.  Images of more than 4 dimensions are refused
 * (ECC_ERR_UNSUPPORTED).
 * count == 0 is a no-op.  Errors as above; the index of the first bad descriptor
 * is named in ecc_last_error. */
ecc_status ecc_compute_batch(ecc_ctx* ctx, const ecc_image* imgs, int32_t count, int32_t nbins,
                             void* hip_stream);

/* ECC of an image that stays in HOST memory (Sec. 4.4's streaming of volumes
 * larger than device memory): slabs of `slab_planes` planes of the first axis
 * (0: about 256 MiB each), each with the one plane after it, are copied to the
 * device in turn on a copy stream of the context while the previous slab is
 * counted on hip_stream; the slab VCECs add up exactly, since every cell is
 * counted by the slab that owns its first-axis start.  img->data is a HOST
 * pointer (pinned memory copies fastest, pageable memory works), img->out a
 * device pointer.  A 2D image travels as one slab.  A 4D image streams in
 * slabs of hyperplanes (its first axis), each with the hyperplane after it,
 * a slab counting the signed 3D terms of its own hyperplanes (as ecc_compute).
 * An AUTO range reads the volume twice (min/max first).  Asynchronous: the host image must stay
 * unchanged until hip_stream has completed the call.  Two device slab buffers
 * are kept by the context.  Results are identical to ecc_compute_ex.
 * Errors: as ecc_compute_ex, plus ECC_ERR_INVALID_ARG for slab_planes < 0. */
ecc_status ecc_compute_streamed(ecc_ctx* ctx, const ecc_image* img, int32_t nbins, int64_t slab_planes,
                                void* hip_stream);

/* One separable 13-tap smoothing pass of a 2D float32 image: the smoothing step
 * of the smoothing + ECC pipeline (Sec. 5, a discrete Gaussian convolution of
 * width 13 applied along each axis).  Rows first, then columns; each output is
 * the sum over k = 0..12, in that order from 0, of taps[k] times the neighbour
 * at offset k - 6 (border pixels repeated), every product and sum rounded once
 * in float32.  in, out: device pointers to n1 * n2 floats (row-major), out may
 * equal in; taps: HOST array of 13 floats.  The context keeps an n1 * n2 float
 * intermediate buffer.  Asynchronous on hip_stream.
 * Errors: ECC_ERR_INVALID_ARG (null pointer, n1 or n2 outside [1, 2^31], more
 * than 2^40 pixels), ECC_ERR_OUT_OF_MEMORY, ECC_ERR_DEVICE. */
ecc_status ecc_smooth13(ecc_ctx* ctx, const float* in, float* out, int64_t n1, int64_t n2, const float* taps,
                        void* hip_stream);

/* Launch shape of the single-image kernel: waves per workgroup (a workgroup
 * covers waves * 63 consecutive position columns), rows (2D) or planes (3D) per
 * workgroup brick, resident workgroups per CU aimed for, `window`, the bins
 * one pass counts in LDS (Sec. 4.3's block-shared histogram; fewer than nbins
 * makes several passes over the image, each with less LDS; 0: all of nbins up to
 * 4096), and `copies`, the copies of that histogram the lanes of a wave spread
 * their adds over (2, 4 or 8; 0: 8 up to 256 bins, 4 up to 1024, else 2).  `ms`
 * is the mean time of one call measured by ecc_autotune. */
typedef struct {
    int32_t waves;
    int32_t wgs_per_cu;
    int64_t depth;
    double ms;
    int32_t window;
    int32_t copies;
} ecc_launch_shape;

/* Times a set of launch shapes for the image `img` on hip_stream (after about
 * 40 ms of calls at the default shape, which bring the device's clocks up: two
 * rounds over the shapes, `reps` calls per shape and round, the faster round
 * counting; the calls overwrite img->out) and makes `ctx` use the
 * fastest for every later call on an image with the same ndim, dims (for 4 or
 * more dimensions: the last three), dtype and filtration and nbins on the same
 * side of 4096.  Every shape gives the same
 * ECC; only the time differs.  An image of 4 or more dimensions is tuned for
 * the shape of its 3D passes (the launches of ecc_compute on it).  Blocks until the timing runs have
 * finished.
 * chosen (HOST pointer, may be null) receives the chosen shape.  Not for use
 * during graph capture.
 * Errors: as ecc_compute_ex, plus ECC_ERR_INVALID_ARG for reps outside
 * [1, 1000]. */
ecc_status ecc_autotune(ecc_ctx* ctx, const ecc_image* img, int32_t nbins, int32_t reps, void* hip_stream,
                        ecc_launch_shape* chosen);

/* Makes `ctx` use `shape` (HOST pointer) for every later call on an image with
 * the same key as ecc_autotune's (ndim, dims, dtype, filtration, nbins on the
 * same side of 4096), as if ecc_autotune had chosen it: for reusing a shape
 * tuned in another process, e.g. in a run under a profiler, whose timings the
 * profiler distorts.  A field <= 0 keeps the default for that field; `ms` is
 * ignored.  The result of a call does not depend on the shape.  Enqueues
 * nothing.  img->data and img->out are not read; img->ndim is 2 .. ECC_MAX_NDIM.
 * Errors: ECC_ERR_INVALID_ARG (null pointer, an invalid descriptor as for
 * ecc_compute_ex, waves above 9, wgs_per_cu above 16, depth above 4096, window
 * above 4096, copies other than 0, 2, 4 or 8). */
ecc_status ecc_set_launch_shape(ecc_ctx* ctx, const ecc_image* img, int32_t nbins, const ecc_launch_shape* shape);

/* A planned batch (Sec. 5's many-files workload, kept on the device): the
 * tables of ecc_compute_batch built once and copied to device memory owned by
 * the plan, so that each launch enqueues kernels only -- no allocation, no host
 * copy, no host synchronisation -- and may be captured into a HIP graph and
 * replayed.  The plan keeps the images' and outputs' device addresses, shapes,
 * dtypes and range modes; the image contents may change between launches (AUTO
 * ranges are recomputed on every launch).  The caller keeps every image and
 * output alive until the plan is destroyed.  Launches of one plan must not
 * overlap in time (they share the plan's scratch); plans of one context follow
 * the context's threading rule.  Results are identical to ecc_compute_batch.
 * ecc_batch_plan_create: imgs is a HOST array of `count` (>= 1) descriptors, as
 * for ecc_compute_batch; blocks until the tables are on the device.
 * Errors: ECC_ERR_INVALID_ARG (bad descriptor or argument; *plan stays null),
 * ECC_ERR_OUT_OF_MEMORY, ECC_ERR_DEVICE; messages via ecc_last_error(ctx). */
typedef struct ecc_batch_plan ecc_batch_plan;
ecc_status ecc_batch_plan_create(ecc_ctx* ctx, const ecc_image* imgs, int32_t count, int32_t nbins,
                                 ecc_batch_plan** plan);
/* Enqueues one run of the planned batch on hip_stream (asynchronous). */
ecc_status ecc_batch_plan_launch(ecc_batch_plan* plan, void* hip_stream);

/* Launch shape of a planned batch: bricks of depth3 planes (3D images) and
 * depth2 rows (2D images), at most wgs_per_cu workgroups per compute unit; ms is
 * the mean time of one run measured by ecc_batch_plan_autotune. */
typedef struct {
    int32_t depth3;
    int32_t depth2;
    int32_t wgs_per_cu;
    int32_t reserved;
    double ms;
} ecc_batch_shape;

/* Chooses the plan's launch shape by timing: runs the batch `reps` times (1..1000)
 * for each candidate shape on hip_stream, keeps the fastest in the plan (every
 * shape gives the same ECCs) and, if `chosen` is not null, writes it there.
 * Blocking: it waits for its runs, and it writes the images' outputs, which hold
 * the batch's ECCs when it returns.  The caller keeps the plan's images alive as
 * for ecc_batch_plan_launch.  Errors: ECC_ERR_INVALID_ARG (null plan, reps out of
 * range), ECC_ERR_OUT_OF_MEMORY, ECC_ERR_DEVICE; on error the plan keeps its
 * previous shape. */
ecc_status ecc_batch_plan_autotune(ecc_batch_plan* plan, int32_t reps, void* hip_stream, ecc_batch_shape* chosen);
/* Releases the plan's device memory; waits for nothing (the caller must have
 * synchronized its launches).  A null plan is accepted and ignored. */
ecc_status ecc_batch_plan_destroy(ecc_batch_plan* plan);

/* Diagnostics (host only: needs no device, touches no memory the descriptors
 * point to, enqueues nothing): how ecc_compute_batch on a context of filtration
 * `construction` (ecc_construction), or a plan with launch shape `shape` (HOST
 * pointer; null = the default shape), splits a batch over the workgroups of
 * `cu_count` compute units.  The bricks of every image are cut into segments,
 * one workgroup histogram each; a segment covers at most 2^27 voxels, so its
 * int32 counters cannot overflow (a voxel position adds at most 8 in absolute
 * value; Sec. 4.3's shared-memory counters hold the sums).  Outputs (HOST
 * pointers): *segments = the number of segments, *max_segment_voxels = the most
 * voxels one segment covers (whole bricks), and, if not null, image_bricks[i] =
 * the bricks of image i and covered_bricks[i] = the bricks of image i that
 * segments cover (equal for a valid schedule).  imgs: HOST array of `count`
 * (>= 1) descriptors, validated as for ecc_compute_batch (data and out must be
 * non-null but are not read).
 * Errors: ECC_ERR_INVALID_ARG, ECC_ERR_UNSUPPORTED; message via
 * ecc_last_error(NULL). */
ecc_status ecc_batch_schedule(const ecc_image* imgs, int32_t count, int32_t nbins, int32_t construction,
                              const ecc_batch_shape* shape,
                              int32_t cu_count, int32_t* segments, int64_t* max_segment_voxels,
                              int64_t* image_bricks, int64_t* covered_bricks);

/* Kernel timing, for measurement tools (the method itself does not need it).
 * With enable != 0, every later call on `ctx` gives each launch of the
 * histogram kernel (the voxel pass of Sec. 2.3 that reads the image; AUTO
 * min/max, merge and scan launches are not counted) a pair of HIP events that
 * take that kernel's own start and end (hipExtLaunchKernel).
 * enable == 0 stops recording and drops unread records.  Timing changes no result.
 * Errors: ECC_ERR_INVALID_ARG (ctx null), ECC_ERR_DEVICE. */
ecc_status ecc_set_kernel_timing(ecc_ctx* ctx, int32_t enable);

/* Waits for the recorded events, writes the summed duration in milliseconds of
 * the histogram-kernel launches recorded since the previous read to *total_ms and
 * their number to *launches (both HOST pointers), and clears the tally.  Blocks
 * until those launches have finished.  After 4096 unread launches a call folds
 * its records into the tally, waiting for them first.
 * Errors: ECC_ERR_INVALID_ARG (null pointer), ECC_ERR_DEVICE. */
ecc_status ecc_kernel_time(ecc_ctx* ctx, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* ECC_H */
