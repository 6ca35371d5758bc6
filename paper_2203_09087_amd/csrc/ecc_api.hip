// ecc_api.hip -- host runtime behind the C ABI of include/ecc.h.
//
// Validates every argument before anything is enqueued, resolves the binning
// parameters (on the host for explicit ranges, on the device for AUTO ranges),
// owns the context's scratch memory, and enqueues the kernel sequence
//     [minmax -> params]  ->  hist (per LDS bin window) -> reduce  ->  scan
// on the caller's stream.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>

#include "../../include/ecc.h"
#include "ecc_internal.h"

struct ecc_ctx {
    int device = 0;
    int construction = 0;
    int cu_count = 256;
    void* ws = nullptr;     // device scratch
    size_t ws_bytes = 0;
    std::string err;
};

namespace {

thread_local std::string g_create_err;

constexpr int kMinmaxBlocks = 1024;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

ecc_status fail(ecc_ctx* ctx, ecc_status st, const std::string& msg)
{
    ctx->err = msg;
    return st;
}

ecc_status hip_fail(ecc_ctx* ctx, hipError_t e, const char* what)
{
    ctx->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? ECC_ERR_OUT_OF_MEMORY : ECC_ERR_DEVICE;
}

ecc_status ensure_ws(ecc_ctx* ctx, size_t bytes)
{
    if (bytes <= ctx->ws_bytes) return ECC_OK;
    size_t want = std::max(bytes, ctx->ws_bytes * 2);
    if (ctx->ws) {
        // The old buffer may still be in use by enqueued work on any stream.
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    hipError_t e = hipMalloc(&ctx->ws, want);
    if (e != hipSuccess) {
        ctx->ws = nullptr;
        return hip_fail(ctx, e, "hipMalloc(scratch)");
    }
    ctx->ws_bytes = want;
    return ECC_OK;
}

// Validated form of one image.
struct Job {
    const void* data;
    int ndim, dtype, range_mode;
    ecc::Geom g;
    int64_t nvox;
    double lo, hi;
    int64_t* out;
};

ecc_status validate(ecc_ctx* ctx, const ecc_image& im, int32_t nbins, const char* where, Job* job)
{
    char buf[256];
    if (!im.data) { snprintf(buf, sizeof buf, "%s: null image pointer", where); return fail(ctx, ECC_ERR_INVALID_ARG, buf); }
    if (!im.out) { snprintf(buf, sizeof buf, "%s: null output pointer", where); return fail(ctx, ECC_ERR_INVALID_ARG, buf); }
    if (im.ndim != 2 && im.ndim != 3) {
        snprintf(buf, sizeof buf, "%s: ndim must be 2 or 3 (got %d)", where, im.ndim);
        return fail(ctx, ECC_ERR_INVALID_ARG, buf);
    }
    if (im.dtype != ECC_U8 && im.dtype != ECC_U16 && im.dtype != ECC_F32) {
        snprintf(buf, sizeof buf, "%s: unknown dtype %d", where, im.dtype);
        return fail(ctx, ECC_ERR_INVALID_ARG, buf);
    }
    if (im.range_mode != ECC_RANGE_DEFAULT && im.range_mode != ECC_RANGE_EXPLICIT &&
        im.range_mode != ECC_RANGE_AUTO) {
        snprintf(buf, sizeof buf, "%s: unknown range mode %d", where, im.range_mode);
        return fail(ctx, ECC_ERR_INVALID_ARG, buf);
    }
    if (im.reserved != 0) { snprintf(buf, sizeof buf, "%s: reserved field must be 0", where); return fail(ctx, ECC_ERR_INVALID_ARG, buf); }
    if (nbins < 1 || nbins > 65535) {
        snprintf(buf, sizeof buf, "%s: nbins must be in [1, 65535] (got %d)", where, nbins);
        return fail(ctx, ECC_ERR_INVALID_ARG, buf);
    }
    int64_t nvox = 1;
    for (int i = 0; i < im.ndim; ++i) {
        if (im.dims[i] < 1 || im.dims[i] > (int64_t(1) << 31)) {
            snprintf(buf, sizeof buf, "%s: dims[%d] = %lld out of [1, 2^31]", where, i, (long long)im.dims[i]);
            return fail(ctx, ECC_ERR_INVALID_ARG, buf);
        }
        if (nvox > (int64_t(1) << 46) / im.dims[i]) {
            snprintf(buf, sizeof buf, "%s: image has more than 2^46 voxels", where);
            return fail(ctx, ECC_ERR_INVALID_ARG, buf);
        }
        nvox *= im.dims[i];
    }
    if (im.range_mode == ECC_RANGE_EXPLICIT) {
        if (im.dtype == ECC_F32) {
            if (!std::isfinite(im.lo) || !std::isfinite(im.hi) || !(im.lo <= im.hi)) {
                snprintf(buf, sizeof buf, "%s: explicit f32 range must be finite with lo <= hi", where);
                return fail(ctx, ECC_ERR_INVALID_ARG, buf);
            }
        } else {
            const double maxv = im.dtype == ECC_U8 ? 255.0 : 65535.0;
            if (!(im.lo >= 0.0) || !(im.hi <= maxv) || !(im.lo <= im.hi) ||
                im.lo != (double)(int64_t)im.lo || im.hi != (double)(int64_t)im.hi) {
                snprintf(buf, sizeof buf, "%s: explicit integer range must be integers 0 <= lo <= hi <= %g",
                         where, maxv);
                return fail(ctx, ECC_ERR_INVALID_ARG, buf);
            }
        }
    }
    job->data = im.data;
    job->ndim = im.ndim;
    job->dtype = im.dtype;
    job->range_mode = im.range_mode;
    if (job->range_mode == ECC_RANGE_DEFAULT)
        job->range_mode = im.dtype == ECC_U8 ? ECC_RANGE_EXPLICIT : ECC_RANGE_AUTO;
    job->lo = im.range_mode == ECC_RANGE_DEFAULT ? 0.0 : im.lo;
    job->hi = im.range_mode == ECC_RANGE_DEFAULT ? 255.0 : im.hi;
    if (im.ndim == 2) job->g = {1, im.dims[0], im.dims[1]};
    else job->g = {im.dims[0], im.dims[1], im.dims[2]};
    job->nvox = nvox;
    job->out = im.out;
    return ECC_OK;
}

ecc::BinParams host_params(const Job& j, int32_t nbins)
{
    ecc::BinParams p = {};
    p.dtype = j.dtype;
    p.nbins = nbins;
    p.lo = j.lo;
    p.hi = j.hi;
    if (j.dtype == ECC_F32) {
        p.flat = (j.hi == j.lo) ? 1 : 0;
        p.scale = p.flat ? 0.0 : (double)nbins / (j.hi - j.lo);
    } else {
        const uint32_t ilo = (uint32_t)j.lo, ihi = (uint32_t)j.hi;
        const uint64_t D = (uint64_t)(ihi - ilo) + 1u;
        p.ilo = ilo;
        p.ihi = ihi;
        p.q0 = (uint32_t)((uint64_t)nbins / D);
        const uint64_t r = (uint64_t)nbins % D;
        p.magic = (uint32_t)(((r << 32) / D) + 1u);
    }
    return p;
}

struct Sizes {
    int grid;
    int32_t window;
    size_t off_params, off_mm, off_partials, total;
};

Sizes plan_sizes(const ecc_ctx* ctx, const Job& j, int32_t nbins)
{
    Sizes s;
    const int64_t tiles = ecc::hist_tiles(j.ndim, j.g);
    s.grid = (int)std::min<int64_t>(tiles, (int64_t)ctx->cu_count * 4);
    s.window = std::min<int32_t>(nbins, ecc::kMaxLdsBins);
    s.off_params = 0;
    s.off_mm = align_up(sizeof(ecc::BinParams));
    s.off_partials = s.off_mm + align_up((size_t)kMinmaxBlocks * 2 * sizeof(uint32_t));
    s.total = s.off_partials + align_up((size_t)s.grid * (size_t)s.window * sizeof(int32_t));
    return s;
}

ecc_status enqueue_one(ecc_ctx* ctx, const Job& j, int32_t nbins, hipStream_t stream)
{
    const Sizes sz = plan_sizes(ctx, j, nbins);
    ecc_status st = ensure_ws(ctx, sz.total);
    if (st != ECC_OK) return st;
    char* base = (char*)ctx->ws;
    ecc::BinParams* pdev = nullptr;
    hipError_t e;
    if (j.range_mode == ECC_RANGE_AUTO) {
        uint32_t* mm = (uint32_t*)(base + sz.off_mm);
        pdev = (ecc::BinParams*)(base + sz.off_params);
        const int blocks = (int)std::min<int64_t>(kMinmaxBlocks, (j.nvox + 255) / 256);
        if ((e = ecc::launch_minmax(j.data, j.dtype, j.nvox, mm, blocks, stream)) != hipSuccess)
            return hip_fail(ctx, e, "minmax launch");
        if ((e = ecc::launch_params_from_minmax(mm, blocks, j.dtype, nbins, pdev, stream)) != hipSuccess)
            return hip_fail(ctx, e, "params launch");
    }
    ecc::HistLaunch L;
    L.data = j.data;
    L.ndim = j.ndim;
    L.dtype = j.dtype;
    L.construction = ctx->construction;
    L.g = j.g;
    L.params_dev = pdev;
    L.params = host_params(j, nbins);
    L.partials = (int32_t*)(base + sz.off_partials);
    L.grid = sz.grid;
    for (int32_t b0 = 0; b0 < nbins; b0 += sz.window) {
        L.bin_lo = b0;
        L.width = std::min<int32_t>(sz.window, nbins - b0);
        if ((e = ecc::launch_hist(L, stream)) != hipSuccess) return hip_fail(ctx, e, "hist launch");
        if ((e = ecc::launch_reduce(L.partials, L.grid, L.width, j.out + b0, stream)) != hipSuccess)
            return hip_fail(ctx, e, "reduce launch");
    }
    if ((e = ecc::launch_scan(j.out, nbins, stream)) != hipSuccess) return hip_fail(ctx, e, "scan launch");
    return ECC_OK;
}

}  // namespace

extern "C" {

ecc_status ecc_create(ecc_ctx** ctx, int32_t device, int32_t construction)
{
    if (!ctx) { g_create_err = "ecc_create: null ctx"; return ECC_ERR_INVALID_ARG; }
    *ctx = nullptr;
    if (construction != ECC_VERTEX && construction != ECC_TOP) {
        g_create_err = "ecc_create: unknown construction";
        return ECC_ERR_INVALID_ARG;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        g_create_err = "ecc_create: no such HIP device";
        return ECC_ERR_DEVICE;
    }
    ecc_ctx* c = new (std::nothrow) ecc_ctx;
    if (!c) { g_create_err = "ecc_create: out of host memory"; return ECC_ERR_OUT_OF_MEMORY; }
    c->device = device;
    c->construction = construction;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->cu_count = prop.multiProcessorCount;
    g_create_err.clear();
    *ctx = c;
    return ECC_OK;
}

ecc_status ecc_destroy(ecc_ctx* ctx)
{
    if (!ctx) return ECC_OK;
    if (ctx->ws) {
        DeviceGuard g(ctx->device);
        (void)hipFree(ctx->ws);
    }
    delete ctx;
    return ECC_OK;
}

const char* ecc_last_error(const ecc_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

ecc_status ecc_compute_ex(ecc_ctx* ctx, const ecc_image* img, int32_t nbins, void* hip_stream)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!img) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_compute_ex: null descriptor");
    Job j;
    ecc_status st = validate(ctx, *img, nbins, "ecc_compute_ex", &j);
    if (st != ECC_OK) return st;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    return enqueue_one(ctx, j, nbins, (hipStream_t)hip_stream);
}

ecc_status ecc_compute(ecc_ctx* ctx, const void* image, int32_t ndim, const int64_t* dims,
                       int32_t dtype, int32_t nbins, int64_t* out, void* hip_stream)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!dims) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_compute: null dims");
    if (ndim != 2 && ndim != 3) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_compute: ndim must be 2 or 3");
    ecc_image im;
    memset(&im, 0, sizeof im);
    im.data = image;
    im.ndim = ndim;
    im.dtype = dtype;
    for (int i = 0; i < ndim; ++i) im.dims[i] = dims[i];
    im.range_mode = ECC_RANGE_DEFAULT;
    im.out = out;
    Job j;
    ecc_status st = validate(ctx, im, nbins, "ecc_compute", &j);
    if (st != ECC_OK) return st;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    return enqueue_one(ctx, j, nbins, (hipStream_t)hip_stream);
}

ecc_status ecc_compute_batch(ecc_ctx* ctx, const ecc_image* imgs, int32_t count, int32_t nbins,
                             void* hip_stream)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (count < 0) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_compute_batch: negative count");
    if (count == 0) return ECC_OK;
    if (!imgs) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_compute_batch: null descriptor array");
    Job* jobs = new (std::nothrow) Job[(size_t)count];
    if (!jobs) return fail(ctx, ECC_ERR_OUT_OF_MEMORY, "ecc_compute_batch: out of host memory");
    for (int32_t i = 0; i < count; ++i) {
        char where[64];
        snprintf(where, sizeof where, "ecc_compute_batch: image %d", i);
        ecc_status st = validate(ctx, imgs[i], nbins, where, &jobs[i]);
        if (st != ECC_OK) { delete[] jobs; return st; }
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) { delete[] jobs; return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed"); }
    size_t need = 0;
    for (int32_t i = 0; i < count; ++i) need = std::max(need, plan_sizes(ctx, jobs[i], nbins).total);
    ecc_status st = ensure_ws(ctx, need);
    for (int32_t i = 0; i < count && st == ECC_OK; ++i)
        st = enqueue_one(ctx, jobs[i], nbins, (hipStream_t)hip_stream);
    delete[] jobs;
    return st;
}

}  // extern "C"
