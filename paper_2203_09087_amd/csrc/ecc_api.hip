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
#include <cstddef>
#include <cmath>
#include <functional>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "../../include/ecc.h"
#include "ecc_internal.h"

struct ecc_batch_plan;

struct ecc_ctx {
    int device = 0;
    int construction = 0;
    int cu_count = 256;
    void* ws = nullptr;          // device scratch
    size_t ws_bytes = 0;
    // pinned host buffers for the batch tables, used in turn: a call waits for a
    // buffer's previous copy only when all of them are still being copied from
    struct Staging {
        void* ptr = nullptr;
        size_t bytes = 0;
        hipEvent_t done = nullptr;   // recorded after the last copy out of ptr
        bool pending = false;
    };
    static constexpr int kStagingSlots = 4;
    Staging staging[kStagingSlots];
    int staging_next = 0;
    // streaming (ecc_compute_streamed): two device slab buffers, a copy stream,
    // and events ordering copies and kernels on them
    void* slab_buf[2] = {nullptr, nullptr};
    size_t slab_cap = 0;
    hipStream_t copy_stream = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr}, consumed[2] = {nullptr, nullptr};
    // intermediate buffer of ecc_smooth13
    void* smooth_tmp = nullptr;
    size_t smooth_cap = 0;
    // launch shapes chosen by ecc_autotune, by image shape (see TuneKey)
    std::map<std::tuple<int, int, int, int, int64_t, int64_t, int64_t>, ecc_launch_shape> tuned;
    // kernel timing (ecc_set_kernel_timing): event pairs around histogram launches
    bool timing = false;
    std::vector<hipEvent_t> tev;   // 2 * kTimingPairs events, created on enable
    size_t tused = 0;              // pairs recorded since the last fold
    double tms = 0.0;              // folded milliseconds
    int64_t tcount = 0;            // folded launches
    std::string err;
};

namespace {

thread_local std::string g_create_err;

constexpr int kMinmaxBlocks = 1024;
// The first bytes of the scratch hold the counters of the single-image merge,
// which the kernels re-arm after every call; no other use may overwrite them.
constexpr size_t kCounterBytes = 1024;
static_assert(kCounterBytes >= ecc::kCounterWords * sizeof(uint32_t), "counter region too small");
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

constexpr size_t kTimingPairs = 4096;

// Adds the durations of the recorded pairs to the tally (waits for them).
ecc_status fold_timing(ecc_ctx* ctx)
{
    for (size_t i = 0; i < ctx->tused; ++i) {
        hipError_t e = hipEventSynchronize(ctx->tev[2 * i + 1]);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize(timing)");
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, ctx->tev[2 * i], ctx->tev[2 * i + 1])) != hipSuccess)
            return hip_fail(ctx, e, "hipEventElapsedTime");
        ctx->tms += ms;
        ctx->tcount += 1;
    }
    ctx->tused = 0;
    return ECC_OK;
}

// Runs `launch(start, stop)` (returning hipError_t), with a pair of timing
// events when the context records kernel timing, else with null events.  The
// events go to the launch itself (hipExtLaunchKernel), which gives them the
// kernel's own start and end: events recorded on the stream around it would
// also count the wait between the start marker and the dispatch (about 6 us on
// a 150 us kernel).
template <class F>
hipError_t timed_launch(ecc_ctx* ctx, F&& launch)
{
    if (!ctx->timing) return launch(nullptr, nullptr);
    if (ctx->tused == kTimingPairs && fold_timing(ctx) != ECC_OK) return hipErrorUnknown;
    const hipError_t e = launch(ctx->tev[2 * ctx->tused], ctx->tev[2 * ctx->tused + 1]);
    if (e == hipSuccess) ctx->tused += 1;
    return e;
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
    // The brick and merge counters live in the scratch and must start at zero;
    // the kernels re-arm them after every call.
    if ((e = hipMemset(ctx->ws, 0, want)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        return hip_fail(ctx, e, "hipMemset(scratch)");
    }
    ctx->ws_bytes = want;
    return ECC_OK;
}

// the descriptor layout the bindings mirror
static_assert(sizeof(ecc_image) == 112 && offsetof(ecc_image, dims) == 16 && offsetof(ecc_image, range_mode) == 80 &&
                  offsetof(ecc_image, lo) == 88 && offsetof(ecc_image, out) == 104,
              "ecc_image layout");

// Validated form of one image.

struct Job {
    const void* data;
    const void* data2;    // 4D pair passes: count the max (min) of data and data2
    int ndim, dtype, range_mode;
    ecc::Geom g;          // 2D/3D: the image; 4D and up: the last three axes
    int64_t nw;           // 4D and up: dims[ndim-4] (hyperplanes of a 4D part); else 1
    int64_t dims[ECC_MAX_NDIM];
    // 3D passes of a 4D part: npass volumes of this shape, pass_stride bytes
    // apart, counted by one launch (EccLaunch::npass)
    int32_t npass = 1;
    int64_t pass_stride = 0;
    int64_t nvox;
    double lo, hi;
    int64_t* out;
};

// max_ndim: the most dimensions the entry point takes (ECC_MAX_NDIM for the
// single-image calls, 4 for batches and the fixed-scratch call, 3 for
// streaming); a valid ndim above it is ECC_ERR_UNSUPPORTED.
ecc_status validate(ecc_ctx* ctx, const ecc_image& im, int32_t nbins, const char* where, Job* job,
                    int max_ndim)
{
    char buf[256];
    if (!im.data) { snprintf(buf, sizeof buf, "%s: null image pointer", where); return fail(ctx, ECC_ERR_INVALID_ARG, buf); }
    if (!im.out) { snprintf(buf, sizeof buf, "%s: null output pointer", where); return fail(ctx, ECC_ERR_INVALID_ARG, buf); }
    if (im.ndim < 2 || im.ndim > ECC_MAX_NDIM) {
        snprintf(buf, sizeof buf, "%s: ndim must be in [2, %d] (got %d)", where, ECC_MAX_NDIM, im.ndim);
        return fail(ctx, ECC_ERR_INVALID_ARG, buf);
    }
    if (im.ndim > max_ndim) {
        snprintf(buf, sizeof buf, "%s: images of more than %d dimensions are not taken here (got %d)", where,
                 max_ndim, im.ndim);
        return fail(ctx, ECC_ERR_UNSUPPORTED, buf);
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
        if (nvox > (int64_t(1) << 40) / im.dims[i]) {
            snprintf(buf, sizeof buf, "%s: image has more than 2^40 voxels", where);
            return fail(ctx, ECC_ERR_INVALID_ARG, buf);
        }
        nvox *= im.dims[i];
    }
    {
        // the kernels address a brick with 32-bit byte offsets from its first row
        const int64_t esize = im.dtype == ECC_U8 ? 1 : (im.dtype == ECC_U16 ? 2 : 4);
        if (im.dims[im.ndim - 1] * esize > (int64_t(1) << 27)) {
            snprintf(buf, sizeof buf, "%s: rows longer than 2^27 bytes are not supported", where);
            return fail(ctx, ECC_ERR_UNSUPPORTED, buf);
        }
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
    job->data2 = nullptr;
    job->ndim = im.ndim;
    job->dtype = im.dtype;
    job->range_mode = im.range_mode;
    if (job->range_mode == ECC_RANGE_DEFAULT)
        job->range_mode = im.dtype == ECC_U8 ? ECC_RANGE_EXPLICIT : ECC_RANGE_AUTO;
    job->lo = im.range_mode == ECC_RANGE_DEFAULT ? 0.0 : im.lo;
    job->hi = im.range_mode == ECC_RANGE_DEFAULT ? 255.0 : im.hi;
    job->nw = 1;
    for (int i = 0; i < ECC_MAX_NDIM; ++i) job->dims[i] = i < im.ndim ? im.dims[i] : 1;
    const int d = im.ndim;
    if (d == 2) job->g = {1, im.dims[0], im.dims[1]};
    else {
        job->g = {im.dims[d - 3], im.dims[d - 2], im.dims[d - 1]};
        if (d >= 4) job->nw = im.dims[d - 4];
    }
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
        // a flat range bins through scale = +inf (see key_of in the kernels)
        p.scale = p.flat ? HUGE_VAL : (double)nbins / (j.hi - j.lo);
        p.base = p.flat ? std::nextafter(j.lo, HUGE_VAL) : j.lo;
    } else {
        const uint32_t ilo = (uint32_t)j.lo, ihi = (uint32_t)j.hi;
        const uint32_t D = ihi - ilo + 1u;
        p.ilo = ilo;
        p.ihi = ihi;
        p.ident = ((uint32_t)nbins == D) ? 1 : 0;
        p.rcp = std::nextafter(1.0 / (double)D, HUGE_VAL);
    }
    return p;
}

struct Sizes {
    int grid;
    int waves;
    int64_t depth;
    int32_t window;
    uint32_t hist_stride, hist_copies, sentinel, lds_bytes;   // LDS layout of the histogram kernel
    size_t off_params, off_counters, off_mm, off_level2, off_partials, total;
};

// Launch shape of the main kernel for one image:
//  - waves: a workgroup's waves cover a contiguous x-chunk of 63 * waves position
//    columns, the whole row when it has at most 9 * 63 positions, else chunks of
//    8 * 63;
//  - depth: planes (3D) or rows (2D) per workgroup brick, chosen so that there are
//    about two bricks per CU;
//  - grid: at most two resident workgroups per CU (more concurrent bricks cost
//    DRAM locality), at least enough that no workgroup histogram can reach 2^31
//    (every voxel position adds at most 8 in absolute value: four type counts of
//    at most 1, and at a brick's last plane four more).
using TuneKey = std::tuple<int, int, int, int, int64_t, int64_t, int64_t>;

TuneKey tune_key(const ecc_ctx* ctx, const Job& j, int32_t nbins)
{
    return TuneKey{j.ndim, j.dtype, ctx->construction, nbins > ecc::kMaxLdsBins ? 1 : 0, j.g.n0, j.g.n1, j.g.n2};
}

// The default launch shape of an image (waves 0 / depth 0 / wgs 0 in a forced
// shape mean "default" for that field).
Sizes plan_sizes(const ecc_ctx* ctx, const Job& j, int32_t nbins, const ecc_launch_shape* force = nullptr)
{
    Sizes s;
    const ecc_launch_shape* tuned = force;
    if (!tuned) {
        auto it = ctx->tuned.find(tune_key(ctx, j, nbins));
        if (it != ctx->tuned.end()) tuned = &it->second;
    }
    const int cons = ctx->construction;
    const int64_t xpos = ecc::axis_positions(j.g.n2, cons);
    const int64_t cols = (xpos + ecc::kLaneCols - 1) / ecc::kLaneCols;
    const int64_t max_waves = j.ndim == 3 ? ECC_MAX_WAVES_3D : ecc::kMaxWaves;
    s.waves = (int)(cols <= max_waves ? cols : std::min<int64_t>(8, max_waves));
    // 3D: when the last wave of a row would own only a few columns, one wave
    // fewer and a packed tail (ecc::layout_3d) keep more lanes busy
    if (j.ndim == 3 && cols > 1 && cols <= max_waves && ecc::layout_3d(j.g, cons, (int)cols - 1).spw > 0)
        s.waves = (int)cols - 1;
    if (tuned && tuned->waves > 0) s.waves = (int)std::min<int64_t>(std::min<int64_t>(tuned->waves, ecc::kMaxWaves), cols);
    const int64_t chunk = ecc::kLaneCols * (int64_t)s.waves;
    const int64_t nxc = (xpos + chunk - 1) / chunk;
    const int64_t target = 2 * (int64_t)ctx->cu_count;
    if (j.ndim == 3) {
        int64_t d = (j.g.n0 * ecc::layout_3d(j.g, cons, s.waves).per_z + target - 1) / target;
        s.depth = std::min<int64_t>(std::max<int64_t>(d, 4), 32);
        if (tuned && tuned->depth > 0) s.depth = std::min<int64_t>(tuned->depth, 256);
    } else {
        int64_t d = (j.g.n1 * nxc + target - 1) / target;
        d = std::min<int64_t>(std::max<int64_t>(d, ecc::kChunk2), 512);
        if (tuned && tuned->depth > 0) d = std::min<int64_t>(tuned->depth, 4096);
        s.depth = (d + ecc::kChunk2 - 1) / ecc::kChunk2 * ecc::kChunk2;
    }
    const int64_t bricks = ecc::wg_bricks(j.ndim, cons, j.g, s.waves, s.depth);
    // bins per LDS pass: all of them up to kMaxLdsBins, or fewer when tuned so
    s.window = std::min<int32_t>(nbins, ecc::kMaxLdsBins);
    if (tuned && tuned->window > 0) s.window = std::min<int32_t>(s.window, tuned->window);
    const bool windowed = s.window < nbins;
    s.hist_stride = ecc::lds_stride(s.window);
    s.hist_copies = ecc::hist_copies(s.window);
    if (tuned && tuned->copies > 0) s.hist_copies = (uint32_t)tuned->copies;
    s.sentinel = ecc::lds_sentinel(nbins);
    s.lds_bytes = 4u * ecc::lds_words(s.window, windowed, s.sentinel, s.hist_copies);
    int want_per_cu = j.ndim == 3 ? ECC_MAX_WGS_PER_CU_3D : ECC_MAX_WGS_PER_CU_2D;
    if (tuned && tuned->wgs_per_cu > 0) want_per_cu = tuned->wgs_per_cu;
    const int per_cu = std::min(want_per_cu, ecc::resident_wgs_per_cu(j.ndim, j.dtype, ctx->construction, windowed,
                                                                      s.waves, s.lds_bytes));
    int64_t grid = std::min<int64_t>(bricks, (int64_t)ctx->cu_count * per_cu);
    grid = std::max<int64_t>(grid, std::min<int64_t>(bricks, (j.nvox >> 27) + 1));
    s.grid = (int)std::max<int64_t>(grid, 1);
    s.off_counters = 0;   // fixed place, shared with the batch layout (never overwritten)
    s.off_params = kCounterBytes;
    s.off_mm = s.off_params + align_up(sizeof(ecc::BinParams));
    s.off_level2 = s.off_mm + align_up((size_t)(kMinmaxBlocks + 1) * 2 * sizeof(uint32_t));
    s.off_partials = s.off_level2 + align_up(ecc::kLevel2Words * sizeof(int64_t));
    s.total = s.off_partials + align_up((size_t)s.grid * (size_t)s.window * sizeof(int32_t));
    return s;
}

// ------------------------------------------- fixed scratch (no allocation)
//
// ecc_compute_noalloc takes its scratch from this array instead of the
// context's buffer.  Each device the library runs on holds its own copy from
// the first context created there until the process ends.  Host code never
// passes the array's name to a kernel (on the host it only stands in for the
// symbol): it uses the device address that hipGetSymbolAddress returned for the
// current device, kept per device in g_noalloc_ptr.
constexpr size_t kNoAllocBytes = size_t(24) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kMaxDevices] = {};   // device address of `scratch` per device; null until set up

__global__ void k_zero_words(uint32_t* p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

// Sets up the fixed scratch of `device`, which must be current: finds its
// device address and clears the merge counters (which the merge re-arms after
// every use; the rest of the scratch is written before it is read).  Runs once
// per device; later calls return at once.
ecc_status noalloc_setup(int device, std::string& err)
{
    if (device < 0 || device >= kMaxDevices) {
        err = "fixed scratch: device index beyond the supported devices";
        return ECC_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return ECC_OK;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return ECC_ERR_DEVICE;
    }
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, (hipStream_t)0, (uint32_t*)ptr,
                       (int)(kCounterBytes / sizeof(uint32_t)));
    if ((e = hipGetLastError()) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
        err = std::string("fixed scratch set-up: ") + hipGetErrorString(e);
        return ECC_ERR_DEVICE;
    }
    g_noalloc_ptr[device] = (char*)ptr;
    return ECC_OK;
}

// Device scratch of one call, laid out as `sz`: the context's buffer (grown
// with hipMalloc when too small), or with no_alloc the device's fixed array.
// For the fixed array the grid is narrowed until the partial rows fit, but never
// below the workgroups that keep each int32 row from overflowing (a workgroup
// takes at most 2^27 voxels); an image that cannot fit is refused before
// anything is enqueued.
ecc_status call_scratch(ecc_ctx* ctx, const Job& j, bool no_alloc, Sizes& sz, char** base)
{
    if (!no_alloc) {
        const ecc_status st = ensure_ws(ctx, sz.total);
        if (st != ECC_OK) return st;
        *base = (char*)ctx->ws;
        return ECC_OK;
    }
    char* ptr = (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_noalloc_ptr[ctx->device] : nullptr;
    if (!ptr) return fail(ctx, ECC_ERR_DEVICE, "ecc_compute_noalloc: the fixed scratch of this device is not set up");
    if (sz.total > kNoAllocBytes) {
        const size_t row = (size_t)sz.window * sizeof(int32_t);
        const int64_t fit = sz.off_partials < kNoAllocBytes ? (int64_t)((kNoAllocBytes - sz.off_partials) / row) : 0;
        const int64_t need = (j.nvox >> 27) + 1;
        if (fit < need) {
            char buf[160];
            snprintf(buf, sizeof buf,
                     "ecc_compute_noalloc: the image needs at least %lld workgroup rows of %zu bytes; the fixed "
                     "scratch holds %lld",
                     (long long)need, row, (long long)fit);
            return fail(ctx, ECC_ERR_UNSUPPORTED, buf);
        }
        sz.grid = (int)std::min<int64_t>(sz.grid, fit);
        sz.total = sz.off_partials + align_up((size_t)sz.grid * row);
    }
    *base = ptr;
    return ECC_OK;
}

// The histogram launches (and merges) of one image or slab, with the scratch
// laid out as `sz` from `base`.  With pass_only
// (one LDS window only) just the histogram kernel runs, writing (or with
// pass_add adding) its workgroup histograms times `sign` into the partial rows,
// which a later merge sums.  pdev: binning
// parameters on the device (AUTO), else the host parameters of j.  Planes
// [0, z_own) of j's planes are counted; they are planes z_base.. of a volume
// of n0_global planes.  accumulate: add the VCEC to out instead of writing it;
// scan: prefix-sum out after the last window.
ecc_status enqueue_hist(ecc_ctx* ctx, char* base, const Job& j, int32_t nbins, hipStream_t stream, const Sizes& sz,
                        const ecc::BinParams* pdev, int64_t z_own, int64_t z_base, int64_t n0_global,
                        bool accumulate, bool scan, int sign = 1, bool pass_only = false, bool pass_add = false)
{
    uint32_t* counters = (uint32_t*)(base + sz.off_counters);
    ecc::EccLaunch L;
    L.data = j.data;
    L.data2 = j.data2;
    L.ndim = j.ndim;
    L.dtype = j.dtype;
    L.construction = ctx->construction;
    L.g = j.g;
    L.params_dev = pdev;
    L.params = host_params(j, nbins);
    L.windowed = sz.window < nbins ? 1 : 0;
    L.grid = sz.grid;
    L.waves = sz.waves;
    L.depth = sz.depth;
    L.z_own = z_own;
    L.z_base = z_base;
    L.n0_global = n0_global;
    L.npass = j.npass;
    L.pass_stride = j.pass_stride;
    L.partials = (int32_t*)(base + sz.off_partials);
    L.flush_add = pass_add ? 1 : 0;
    L.flush_sign = sign;
    L.out = j.out;
    L.counter = counters;
    L.fused = 0;
    L.hist_stride = sz.hist_stride;
    L.hist_copies = sz.hist_copies;
    L.sentinel = sz.sentinel;
    L.lds_bytes = sz.lds_bytes;
    auto launch_l = [&](hipEvent_t t0, hipEvent_t t1) { return ecc::launch_ecc(L, stream, t0, t1); };
    hipError_t e;
    if (pass_only) {
        // one window, histogram kernel only: its rows are merged by a later call
        L.bin_lo = 0;
        L.width = sz.window;
        if ((e = timed_launch(ctx, launch_l)) != hipSuccess)
            return hip_fail(ctx, e, "ecc launch");
        return ECC_OK;
    }
    L.flush_add = 0;
    L.flush_sign = 1;
    if (!accumulate && scan && sign > 0 && L.npass == 1 && sz.window >= nbins &&
        (int64_t)L.grid * nbins <= ecc::kFusedMergeWords) {
        // few rows: the histogram kernel's last workgroup merges and scans them
        L.bin_lo = 0;
        L.width = nbins;
        L.fused = 1;
        if ((e = timed_launch(ctx, launch_l)) != hipSuccess)
            return hip_fail(ctx, e, "ecc launch");
        return ECC_OK;
    }
    for (int32_t b0 = 0; b0 < nbins; b0 += sz.window) {
        L.bin_lo = b0;
        L.width = std::min<int32_t>(sz.window, nbins - b0);
        const bool last = b0 + L.width >= nbins;
        if ((e = timed_launch(ctx, launch_l)) != hipSuccess)
            return hip_fail(ctx, e, "ecc launch");
        if ((e = ecc::launch_merge(L.partials, L.grid * L.npass, L.width, L.bin_lo, (int64_t*)(base + sz.off_level2),
                                   j.out, nbins, counters, accumulate, scan && last, sign, stream)) != hipSuccess)
            return hip_fail(ctx, e, "merge launch");
    }
    return ECC_OK;
}

ecc_status enqueue_one(ecc_ctx* ctx, const Job& j, int32_t nbins, hipStream_t stream,
                       const ecc_launch_shape* force = nullptr, bool no_alloc = false)
{
    Sizes sz = plan_sizes(ctx, j, nbins, force);
    char* base = nullptr;
    ecc_status st = call_scratch(ctx, j, no_alloc, sz, &base);
    if (st != ECC_OK) return st;
    ecc::BinParams* pdev = nullptr;
    hipError_t e;
    if (j.range_mode == ECC_RANGE_AUTO) {
        uint32_t* mm = (uint32_t*)(base + sz.off_mm);
        pdev = (ecc::BinParams*)(base + sz.off_params);
        const int blocks = (int)std::min<int64_t>(kMinmaxBlocks, (j.nvox + 4095) / 4096);
        if ((e = ecc::launch_minmax(j.data, j.dtype, j.nvox, mm, blocks, stream)) != hipSuccess)
            return hip_fail(ctx, e, "minmax launch");
        if ((e = ecc::launch_params_from_minmax(mm, blocks, j.dtype, nbins, pdev, stream)) != hipSuccess)
            return hip_fail(ctx, e, "params launch");
    }
    return enqueue_hist(ctx, base, j, nbins, stream, sz, pdev, j.g.n0, 0, j.g.n0, false, true);
}

// An image of four or more dimensions as signed 3D passes.  The cells of a
// d-dimensional complex are (d-1)-dimensional cells times a vertex or an edge
// of the first axis (Sec. 2.1), so with H_w the hyperplanes of that axis:
//   vertex: VCEC = sum_w V(H_w) - sum_{w<n-1} V(max(H_w, H_{w+1}))
//   top:    VCEC = sum_w c_w T(H_w) + sum_{w<n-1} T(min(H_w, H_{w+1})),
//           c_w = -1 + [w == 0] + [w == n-1]
// (elementwise max and min).  Applied once, this takes a 4D image to 3D passes;
// a pair pass reads both hyperplanes and counts the max (min) of their keys.
// Above four dimensions it is applied one axis at a time, and the max (min) of
// two hyperplanes of a reduced axis is written into a buffer of that axis in
// the scratch, whose hyperplanes the next axis then reads.  Every pass adds
// into (or subtracts from) the caller's output, the last one scans it.  The
// binning parameters are the whole image's.

// The 3D passes of one 4D image or 4D part (at img4, nw hyperplanes of the
// shape of h), each times `outer`; the first part writes out, the others add
// to it, and the last one scans it.
ecc_status enqueue_4d_part(ecc_ctx* ctx, char* base, const Sizes& sz, Job h, const char* img4, int64_t nw,
                           const ecc::BinParams* pdev, int32_t nbins, hipStream_t stream, int outer, bool first,
                           bool last, int64_t w_first = 0, int64_t nw_all = -1, int64_t n_own = -1)
{
    // img4 holds hyperplanes w_first .. of a 4D image of nw_all hyperplanes (all
    // nw of them unless a streamed slab); the terms of its own n_own hyperplanes
    // are counted (a pair term (w, w+1) belongs to w; the hyperplane after the
    // own ones, when held, completes the last pair).
    if (nw_all < 0) nw_all = nw;
    if (n_own < 0) n_own = nw;
    const int64_t hv = h.nvox;
    const size_t esize = h.dtype == ECC_U8 ? 1 : (h.dtype == ECC_U16 ? 2 : 4);
    const bool vertex = ctx->construction == ECC_VERTEX;
    auto plane = [&](int64_t w) { return (const void*)(img4 + (size_t)w * (size_t)hv * esize); };
    // The terms in groups of one sign and kind, each a run of hyperplanes (or
    // of pairs (w, w+1)) one hyperplane apart, the largest group first:
    //   vertex: hyperplanes (+), pairs (-);
    //   top:    pairs (+), interior hyperplanes (-) (the end ones have
    //           c_w = 0), or the one hyperplane of a single-hyperplane image (+).
    struct Group {
        int64_t w0, count;   // w0: index in img4
        int sign;
        bool pair;
    } groups[2];
    int ng = 0;
    const int64_t npairs = std::max<int64_t>(0, std::min<int64_t>(n_own, nw_all - 1 - w_first));
    if (vertex) {
        groups[ng++] = {0, n_own, 1, false};
        if (npairs > 0) groups[ng++] = {0, npairs, -1, true};
    } else if (nw_all == 1) {
        groups[ng++] = {0, 1, 1, false};
    } else {
        if (npairs > 0) groups[ng++] = {0, npairs, 1, true};
        const int64_t a = std::max<int64_t>(w_first, 1), b = std::min<int64_t>(w_first + n_own, nw_all - 1);
        if (b > a) groups[ng++] = {a - w_first, b - a, -1, false};
    }
    if (ng == 2 && groups[1].count > groups[0].count) std::swap(groups[0], groups[1]);
    // A group runs as launches of c passes each (EccLaunch::npass), gx
    // workgroups per pass: the first launch's gx * c rows (at most the buffer's
    // sz.grid) cover the rows of every later launch, which add into them.
    int64_t rows = sz.grid;
    auto for_launches = [&](auto&& fn) -> ecc_status {
        int64_t cap = sz.grid;
        bool first_launch = true;
        for (int g = 0; g < ng; ++g) {
            for (int64_t done = 0; done < groups[g].count;) {
                const int64_t c = std::min<int64_t>(groups[g].count - done, cap);
                const int64_t gx = std::max<int64_t>(1, cap / c);
                if (first_launch) {
                    cap = rows = gx * c;
                    first_launch = false;
                }
                const ecc_status r = fn(groups[g].w0 + done, c, groups[g].sign, groups[g].pair, gx);
                if (r != ECC_OK) return r;
                done += c;
            }
        }
        return ECC_OK;
    };
    // With one LDS window every launch adds into the same workgroup rows and one
    // merge follows, when the int32 rows cannot overflow: a row's workgroup sees
    // at most ceil(bricks / gx) bricks of chunk x rows x depth voxels per
    // launch, and a voxel adds at most 8 in absolute value.
    const int64_t bricks = ecc::wg_bricks(3, ctx->construction, h.g, sz.waves, sz.depth);
    const int64_t brick_vox = ecc::kLaneCols * sz.waves * ecc::kRows3 * sz.depth;
    int64_t nlaunch = 0, per_row = 0;
    for_launches([&](int64_t, int64_t, int, bool, int64_t gx) {
        ++nlaunch;
        per_row += (bricks + gx - 1) / gx * brick_vox;
        return ECC_OK;
    });
    const bool one_merge = sz.window >= nbins && per_row < (int64_t(1) << 28);
    int64_t k = 0;
    ecc_status st = for_launches([&](int64_t w0, int64_t c, int sign, bool pair, int64_t gx) {
        Job p = h;
        p.data = plane(w0);
        p.data2 = pair ? plane(w0 + 1) : nullptr;
        p.npass = (int32_t)c;
        p.pass_stride = (int64_t)hv * (int64_t)esize;
        Sizes s = sz;
        s.grid = (int)gx;
        const ecc_status r = enqueue_hist(ctx, base, p, nbins, stream, s, pdev, h.g.n0, 0, h.g.n0, !first || k > 0,
                                          last && k + 1 == nlaunch, sign * outer, one_merge, k > 0);
        ++k;
        return r;
    });
    if (st != ECC_OK) return st;
    if (one_merge) {
        uint32_t* counters = (uint32_t*)(base + sz.off_counters);
        const hipError_t e = ecc::launch_merge((int32_t*)(base + sz.off_partials), (int)rows, nbins, 0,
                                               (int64_t*)(base + sz.off_level2), h.out, nbins, counters, !first,
                                               last, 1, stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "merge launch");
    }
    return ECC_OK;
}

ecc_status enqueue_nd(ecc_ctx* ctx, const Job& j, int32_t nbins, hipStream_t stream, bool no_alloc = false,
                      const ecc_launch_shape* force = nullptr)
{
    const int d = j.ndim;
    const size_t esize = j.dtype == ECC_U8 ? 1 : (j.dtype == ECC_U16 ? 2 : 4);
    Job h = j;   // one hyperplane of the last three axes, as a 3D image
    h.ndim = 3;
    h.nw = 1;
    h.nvox = j.g.n0 * j.g.n1 * j.g.n2;
    h.data2 = nullptr;
    // the passes' launch shape: forced, tuned for this image's shape, or the default
    if (!force) {
        auto it = ctx->tuned.find(tune_key(ctx, j, nbins));
        if (it != ctx->tuned.end()) force = &it->second;
    }
    Sizes sz = plan_sizes(ctx, h, nbins, force);
    // one buffer per reduced axis a < d-4, a hyperplane of it, after the rest
    size_t mat_off[ECC_MAX_NDIM] = {};
    int64_t plane_vox[ECC_MAX_NDIM] = {};
    int64_t left = j.nvox;
    for (int a = 0; a + 4 < d; ++a) {
        left /= j.dims[a];
        plane_vox[a] = left;
        mat_off[a] = sz.total;
        sz.total += align_up((size_t)left * esize);
    }
    if (d > 4 && no_alloc) return fail(ctx, ECC_ERR_UNSUPPORTED, "images of more than 4 dimensions need scratch");
    char* base = nullptr;
    ecc_status st = call_scratch(ctx, h, no_alloc, sz, &base);
    if (st != ECC_OK) return st;
    ecc::BinParams* pdev = nullptr;
    hipError_t e;
    if (j.range_mode == ECC_RANGE_AUTO) {
        uint32_t* mm = (uint32_t*)(base + sz.off_mm);
        pdev = (ecc::BinParams*)(base + sz.off_params);
        const int blocks = (int)std::min<int64_t>(kMinmaxBlocks, (j.nvox + 4095) / 4096);
        if ((e = ecc::launch_minmax(j.data, j.dtype, j.nvox, mm, blocks, stream)) != hipSuccess)
            return hip_fail(ctx, e, "minmax launch");
        if ((e = ecc::launch_params_from_minmax(mm, blocks, j.dtype, nbins, pdev, stream)) != hipSuccess)
            return hip_fail(ctx, e, "params launch");
    }
    const bool vertex = ctx->construction == ECC_VERTEX;
    auto single_sign = [&](int64_t w, int64_t n) { return vertex ? 1 : -1 + (w == 0) + (w == n - 1); };
    // 4D parts in all: per reduced axis, its hyperplanes of nonzero sign and its pairs
    int64_t parts = 1;
    for (int a = 0; a + 4 < d; ++a) {
        int64_t c = j.dims[a] - 1;
        for (int64_t w = 0; w < j.dims[a]; ++w) c += single_sign(w, j.dims[a]) != 0;
        parts *= c;
    }
    int64_t done = 0;
    // axis a of the (d-a)-dimensional volume at vol, counted with sign
    std::function<ecc_status(int, const char*, int)> visit = [&](int a, const char* vol, int sign) -> ecc_status {
        if (a + 4 == d) {
            const bool first = done == 0, last = done + 1 == parts;
            ++done;
            return enqueue_4d_part(ctx, base, sz, h, vol, j.dims[a], pdev, nbins, stream, sign, first, last);
        }
        const int64_t n = j.dims[a];
        const size_t pb = (size_t)plane_vox[a] * esize;
        char* m = base + mat_off[a];
        for (int64_t w = 0; w < n; ++w) {
            ecc_status r;
            const int c = single_sign(w, n);
            if (c != 0 && (r = visit(a + 1, vol + (size_t)w * pb, sign * c)) != ECC_OK) return r;
            if (w + 1 < n) {
                hipError_t ce = ecc::launch_combine(vol + (size_t)w * pb, vol + (size_t)(w + 1) * pb, m,
                                                    plane_vox[a], j.dtype, vertex, stream);
                if (ce != hipSuccess) return hip_fail(ctx, ce, "combine launch");
                if ((r = visit(a + 1, m, vertex ? -sign : sign)) != ECC_OK) return r;
            }
        }
        return ECC_OK;
    };
    return visit(0, (const char*)j.data, 1);
}

// ------------------------------------------------------------------ batches

// The next staging buffer, of at least `bytes`.  Only when its previous copy
// (kStagingSlots calls ago) is still in flight does the host wait for it; only
// a buffer that is too small is replaced.
ecc_status ensure_staging(ecc_ctx* ctx, size_t bytes, ecc_ctx::Staging** out)
{
    hipError_t e;
    ecc_ctx::Staging& sl = ctx->staging[ctx->staging_next];
    ctx->staging_next = (ctx->staging_next + 1) % ecc_ctx::kStagingSlots;
    if (!sl.done) {
        if ((e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(ctx, e, "hipEventCreate");
    }
    if (sl.pending) {
        if ((e = hipEventSynchronize(sl.done)) != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
        sl.pending = false;
    }
    *out = &sl;
    if (bytes <= sl.bytes) return ECC_OK;
    if (sl.ptr) (void)hipHostFree(sl.ptr);
    sl.ptr = nullptr;
    sl.bytes = 0;
    const size_t want = std::max(bytes, (size_t)64 << 10);
    if ((e = hipHostMalloc(&sl.ptr, want, hipHostMallocDefault)) != hipSuccess) {
        sl.ptr = nullptr;
        return hip_fail(ctx, e, "hipHostMalloc(staging)");
    }
    sl.bytes = want;
    return ECC_OK;
}

// Byte layout of the batch tables, relative to the start of the tables (the
// same in the pinned staging buffer and in device memory), followed by the
// partial histogram rows on the device.
struct BatchLayout {
    size_t images, segs, wg_seg, slot_off, slots, mm, pieces, tables_end, partials, total;
};

struct BatchGroup {
    int dtype;
    int grid;
    size_t wg_seg_first;
    bool pairs;   // the group counts pair volumes
};

// Host form of a batch: descriptor tables, workgroup segments and launch groups.
struct BatchTables {
    int count = 0;
    int32_t nbins = 0, window = 0;
    std::vector<ecc::BatchImage> images;
    std::vector<ecc::BatchSeg> segs;
    std::vector<int32_t> wg_seg, slot_off, slots;
    std::vector<uint32_t> mm;
    std::vector<ecc::BatchPiece> pieces;
    std::vector<BatchGroup> groups;
    std::vector<int64_t> owner_bricks;   // bricks of each image's volumes
    BatchLayout lay;
};

// The batch's launch shape unless a plan was tuned.
constexpr ecc_batch_shape kDefaultBatchShape = {8, 128, 2, 0, 0.0};

// Voxels one batch segment may cover (counted over whole bricks, so including
// brick parts outside the image).  Its workgroup histogram and its partial row
// are int32 and a voxel position adds at most 8 in absolute value (four type
// counts of at most 1 in 3D, two in 2D, and as many again at a brick's last
// plane or row), so 2^27 voxels keep every counter below 2^31.
constexpr int64_t kSegVoxels = int64_t(1) << 27;

void build_batch_tables(int cu_count, int construction, const std::vector<Job>& jobs, int32_t nbins, BatchTables& T,
                        const ecc_batch_shape& shape = kDefaultBatchShape)
{
    const int count = (int)jobs.size();
    const int waves = ecc::kBatchWaves;
    T.count = count;
    T.nbins = nbins;
    T.window = std::min<int32_t>(nbins, ecc::kMaxLdsBins);
    T.images.assign((size_t)count, ecc::BatchImage{});
    // the volumes that are counted, in image order: a 2D or 3D image itself; a
    // 4D image's signed 3D passes (as in enqueue_nd), appended after the images
    std::vector<int> vols;
    for (int i = 0; i < count; ++i) {
        const Job& j = jobs[(size_t)i];
        ecc::BatchImage& im = T.images[(size_t)i];
        memset(&im, 0, sizeof im);
        im.data = j.data;
        im.g = j.g;
        im.ndim = j.ndim;
        im.dtype = j.dtype;
        im.auto_range = j.range_mode == ECC_RANGE_AUTO ? 1 : 0;
        im.nvox = j.nvox;
        im.params = host_params(j, nbins);
        im.out = j.out;
        im.sign = 1;
        im.owner = i;
        if (j.ndim != 4) {
            vols.push_back(i);
            continue;
        }
        const int64_t nw = j.nw, hv = j.g.n0 * j.g.n1 * j.g.n2;
        const size_t esize = j.dtype == ECC_U8 ? 1 : (j.dtype == ECC_U16 ? 2 : 4);
        const bool vertex = construction == ECC_VERTEX;
        for (int64_t w = 0; w < nw; ++w) {
            for (int pair = 0; pair < 2; ++pair) {
                const int sign = pair ? (vertex ? -1 : 1) : (vertex ? 1 : -1 + (w == 0) + (w == nw - 1));
                if (sign == 0 || (pair && w + 1 >= nw)) continue;
                ecc::BatchImage v = T.images[(size_t)i];
                v.ndim = 3;
                v.nvox = hv;
                v.data = (const char*)j.data + (size_t)w * (size_t)hv * esize;
                v.data2 = pair ? (const char*)j.data + (size_t)(w + 1) * (size_t)hv * esize : nullptr;
                v.sign = sign;
                vols.push_back((int)T.images.size());
                T.images.push_back(v);
            }
        }
    }
    const size_t nrec = T.images.size();
    std::vector<int64_t> bricks(nrec, 0), max_take(nrec, 1);
    std::vector<double> brick_cost(nrec, 0.0);
    T.owner_bricks.assign((size_t)count, 0);
    for (int i : vols) {
        ecc::BatchImage& im = T.images[(size_t)i];
        bricks[(size_t)i] = ecc::batch_bricks(im, construction, waves, shape.depth3, shape.depth2);
        T.owner_bricks[(size_t)im.owner] += bricks[(size_t)i];
        // time of one brick: a team of wpb waves walks its rows (two 2D problems
        // per row in 3D, twice the loads for a pair volume); W / wpb teams of a
        // workgroup share one pass
        const double teams = (double)(waves / im.wpb);
        brick_cost[(size_t)i] = (im.ndim == 3 ? 2.0 * ecc::kRows3 : 1.0) * (double)im.depth / teams;
        // a segment's histogram is an int32 row: at most kSegVoxels voxels each
        max_take[(size_t)i] = std::max<int64_t>(1, kSegVoxels / ecc::batch_brick_voxels(im));
    }
    // One launch per dtype present; the bricks of its volumes, in order, are cut
    // into one contiguous run per workgroup with about equal work.
    for (int dt = 0; dt < 3; ++dt) {
        double total = 0;
        int64_t nbr = 0;
        bool pairs = false;
        for (int i : vols)
            if (T.images[(size_t)i].dtype == dt) {
                total += bricks[(size_t)i] * brick_cost[(size_t)i];
                nbr += bricks[(size_t)i];
                pairs = pairs || T.images[(size_t)i].data2 != nullptr;
            }
        if (nbr == 0) continue;
        const int G = (int)std::max<int64_t>(1, std::min<int64_t>(nbr, (int64_t)shape.wgs_per_cu * cu_count));
        BatchGroup gr{dt, G, T.wg_seg.size(), pairs};
        const double per = total / G;
        int wg = 0;
        double acc = 0;   // work assigned to workgroups 0..wg-1 plus the current one
        T.wg_seg.push_back((int32_t)T.segs.size());
        for (int i : vols) {
            if (T.images[(size_t)i].dtype != dt) continue;
            int64_t b = 0;
            while (b < bricks[(size_t)i]) {
                // bricks of volume i that still fit in workgroup wg's share
                const double room = per * (wg + 1) - acc;
                int64_t take = (int64_t)std::ceil(room / brick_cost[(size_t)i] - 1e-9);
                if (wg == G - 1) take = bricks[(size_t)i] - b;
                take = std::max<int64_t>(1, std::min<int64_t>(take, bricks[(size_t)i] - b));
                take = std::min<int64_t>(take, max_take[(size_t)i]);
                T.segs.push_back(ecc::BatchSeg{i, (int32_t)T.segs.size(), b, b + take});
                acc += take * brick_cost[(size_t)i];
                b += take;
                if (acc >= per * (wg + 1) - 1e-9 && wg < G - 1) {
                    ++wg;
                    T.wg_seg.push_back((int32_t)T.segs.size());
                }
            }
        }
        while ((int)(T.wg_seg.size() - gr.wg_seg_first) < G + 1) T.wg_seg.push_back((int32_t)T.segs.size());
        T.groups.push_back(gr);
    }
    const int nseg = (int)T.segs.size();
    // partial rows of every image (its volumes' segments)
    T.slot_off.assign((size_t)count + 1, 0);
    T.slots.assign((size_t)nseg, 0);
    for (const auto& sg : T.segs) T.slot_off[(size_t)T.images[(size_t)sg.image].owner + 1]++;
    for (int i = 0; i < count; ++i) T.slot_off[(size_t)i + 1] += T.slot_off[(size_t)i];
    {
        std::vector<int32_t> fill(T.slot_off.begin(), T.slot_off.end() - 1);
        for (const auto& sg : T.segs) T.slots[(size_t)fill[(size_t)T.images[(size_t)sg.image].owner]++] = sg.slot;
    }
    // pieces of the AUTO images for the min/max pass
    const int64_t piece = int64_t(1) << 20;
    for (int i = 0; i < count; ++i)
        if (T.images[(size_t)i].auto_range)
            for (int64_t b = 0; b < T.images[(size_t)i].nvox; b += piece)
                T.pieces.push_back(ecc::BatchPiece{i, 0, b, std::min(T.images[(size_t)i].nvox, b + piece)});
    T.mm.assign((size_t)count * 2, 0u);
    for (int i = 0; i < count; ++i) T.mm[2 * (size_t)i] = 0xFFFFFFFFu;

    BatchLayout& lay = T.lay;
    lay.images = 0;
    lay.segs = align_up(lay.images + T.images.size() * sizeof(ecc::BatchImage));
    lay.wg_seg = align_up(lay.segs + T.segs.size() * sizeof(ecc::BatchSeg));
    lay.slot_off = align_up(lay.wg_seg + T.wg_seg.size() * sizeof(int32_t));
    lay.slots = align_up(lay.slot_off + T.slot_off.size() * sizeof(int32_t));
    lay.mm = align_up(lay.slots + T.slots.size() * sizeof(int32_t));
    lay.pieces = align_up(lay.mm + T.mm.size() * sizeof(uint32_t));
    lay.tables_end = align_up(lay.pieces + T.pieces.size() * sizeof(ecc::BatchPiece));
    lay.partials = lay.tables_end;
    lay.total = lay.partials + align_up((size_t)nseg * (size_t)T.window * sizeof(int32_t));
}

// Copies the tables into host memory laid out as lay (bytes [0, tables_end)).
void pack_batch_tables(const BatchTables& T, char* h)
{
    const BatchLayout& lay = T.lay;
    memcpy(h + lay.images, T.images.data(), T.images.size() * sizeof(ecc::BatchImage));
    memcpy(h + lay.segs, T.segs.data(), T.segs.size() * sizeof(ecc::BatchSeg));
    memcpy(h + lay.wg_seg, T.wg_seg.data(), T.wg_seg.size() * sizeof(int32_t));
    memcpy(h + lay.slot_off, T.slot_off.data(), T.slot_off.size() * sizeof(int32_t));
    memcpy(h + lay.slots, T.slots.data(), T.slots.size() * sizeof(int32_t));
    memcpy(h + lay.mm, T.mm.data(), T.mm.size() * sizeof(uint32_t));
    if (!T.pieces.empty()) memcpy(h + lay.pieces, T.pieces.data(), T.pieces.size() * sizeof(ecc::BatchPiece));
}

// Enqueues the kernels of a batch whose tables are at device address d (layout
// T.lay).  reset_mm: re-initialise the AUTO min/max keys on the device first
// (plans; a per-call upload carries them already).
ecc_status launch_batch_kernels(ecc_ctx* ctx, const BatchTables& T, char* d, bool reset_mm, hipStream_t stream)
{
    const BatchLayout& lay = T.lay;
    ecc::BatchLaunch B;
    memset(&B, 0, sizeof B);
    B.images = (const ecc::BatchImage*)(d + lay.images);
    B.count = T.count;
    B.segs = (const ecc::BatchSeg*)(d + lay.segs);
    B.slot_off = (const int32_t*)(d + lay.slot_off);
    B.slots = (const int32_t*)(d + lay.slots);
    B.mm = (uint32_t*)(d + lay.mm);
    B.partials = (int32_t*)(d + lay.partials);
    B.nbins = T.nbins;
    B.waves = ecc::kBatchWaves;
    B.windowed = T.window < T.nbins ? 1 : 0;
    B.hist_stride = ecc::lds_stride(T.window);
    B.hist_copies = ecc::hist_copies(T.window);
    B.sentinel = ecc::lds_sentinel(T.nbins);
    B.lds_bytes = 4u * ecc::lds_words(T.window, B.windowed != 0, B.sentinel, B.hist_copies);
    hipError_t e;
    if (!T.pieces.empty()) {
        if (reset_mm && (e = ecc::launch_mm_init(B.mm, T.count, stream)) != hipSuccess)
            return hip_fail(ctx, e, "batch min/max init launch");
        if ((e = ecc::launch_minmax_batch(B.images, (const ecc::BatchPiece*)(d + lay.pieces), (int)T.pieces.size(),
                                          B.mm, stream)) != hipSuccess)
            return hip_fail(ctx, e, "batch minmax launch");
    }
    for (int32_t b0 = 0; b0 < T.nbins; b0 += T.window) {
        B.bin_lo = b0;
        B.width = std::min<int32_t>(T.window, T.nbins - b0);
        for (const BatchGroup& gr : T.groups) {
            B.dtype = gr.dtype;
            B.grid = gr.grid;
            B.wg_seg = (const int32_t*)(d + lay.wg_seg) + gr.wg_seg_first;
            B.pairs = gr.pairs ? 1 : 0;
            auto launch_b = [&](hipEvent_t t0, hipEvent_t t1) {
                return ecc::launch_ecc_batch(B, ctx->construction, stream, t0, t1);
            };
            if ((e = timed_launch(ctx, launch_b)) != hipSuccess) return hip_fail(ctx, e, "batch launch");
        }
        if ((e = ecc::launch_merge_batch(B, b0 + B.width >= T.nbins, stream)) != hipSuccess)
            return hip_fail(ctx, e, "batch merge launch");
    }
    return ECC_OK;
}

ecc_status enqueue_batch(ecc_ctx* ctx, const std::vector<Job>& jobs, int32_t nbins, hipStream_t stream)
{
    BatchTables T;
    build_batch_tables(ctx->cu_count, ctx->construction, jobs, nbins, T);
    // the tables follow the single-image counters in the scratch (never overwritten)
    const size_t base = kCounterBytes;
    ecc_status st = ensure_ws(ctx, base + T.lay.total);
    if (st != ECC_OK) return st;
    ecc_ctx::Staging* sl = nullptr;
    if ((st = ensure_staging(ctx, T.lay.tables_end, &sl)) != ECC_OK) return st;
    pack_batch_tables(T, (char*)sl->ptr);
    char* d = (char*)ctx->ws + base;
    hipError_t e;
    if ((e = hipMemcpyAsync(d, sl->ptr, T.lay.tables_end, hipMemcpyHostToDevice, stream)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemcpyAsync(batch tables)");
    if ((e = hipEventRecord(sl->done, stream)) != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
    sl->pending = true;
    return launch_batch_kernels(ctx, T, d, false, stream);
}

}  // namespace

// ------------------------------------------------------------- streaming

ecc_status ensure_streaming(ecc_ctx* ctx, size_t slab_bytes)
{
    hipError_t e;
    if (!ctx->copy_stream) {
        if ((e = hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking)) != hipSuccess) {
            ctx->copy_stream = nullptr;
            return hip_fail(ctx, e, "hipStreamCreate(copy)");
        }
        for (int b = 0; b < 2; ++b) {
            if ((e = hipEventCreateWithFlags(&ctx->copied[b], hipEventDisableTiming)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&ctx->consumed[b], hipEventDisableTiming)) != hipSuccess)
                return hip_fail(ctx, e, "hipEventCreate(streaming)");
        }
    }
    if (slab_bytes <= ctx->slab_cap) return ECC_OK;
    // the old buffers may still be read by enqueued work
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
    for (int b = 0; b < 2; ++b) {
        if (ctx->slab_buf[b]) (void)hipFree(ctx->slab_buf[b]);
        ctx->slab_buf[b] = nullptr;
    }
    ctx->slab_cap = 0;
    for (int b = 0; b < 2; ++b) {
        if ((e = hipMalloc(&ctx->slab_buf[b], slab_bytes)) != hipSuccess) {
            ctx->slab_buf[b] = nullptr;
            return hip_fail(ctx, e, "hipMalloc(slab)");
        }
    }
    ctx->slab_cap = slab_bytes;
    return ECC_OK;
}

// Copies planes [z0, z0 + n) of the host volume into slab buffer b on the copy
// stream, after the kernels that last read that buffer.
ecc_status stream_copy(ecc_ctx* ctx, const char* host, size_t plane_bytes, int64_t z0, int64_t n, int b)
{
    hipError_t e;
    if ((e = hipStreamWaitEvent(ctx->copy_stream, ctx->consumed[b], 0)) != hipSuccess)
        return hip_fail(ctx, e, "hipStreamWaitEvent(copy)");
    if ((e = hipMemcpyAsync(ctx->slab_buf[b], host + (size_t)z0 * plane_bytes, (size_t)n * plane_bytes,
                            hipMemcpyHostToDevice, ctx->copy_stream)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemcpyAsync(slab)");
    if ((e = hipEventRecord(ctx->copied[b], ctx->copy_stream)) != hipSuccess)
        return hip_fail(ctx, e, "hipEventRecord(copied)");
    return ECC_OK;
}

ecc_status enqueue_streamed(ecc_ctx* ctx, const Job& vol, int32_t nbins, int64_t slab_planes, hipStream_t stream)
{
    // A 4D image streams in slabs of hyperplanes (its first axis) the same way
    // a 3D one streams in slabs of planes; each slab counts the 3D terms of its
    // own hyperplanes (enqueue_4d_part), the hyperplane after them completing
    // the last pair.
    const bool four = vol.ndim == 4;
    const int64_t N = four ? vol.nw : vol.g.n0;
    const size_t esize = vol.dtype == ECC_U8 ? 1 : (vol.dtype == ECC_U16 ? 2 : 4);
    const int64_t plane_vox = four ? vol.g.n0 * vol.g.n1 * vol.g.n2 : vol.g.n1 * vol.g.n2;
    const size_t plane_bytes = (size_t)plane_vox * esize;
    int64_t S = slab_planes;
    if (S <= 0) S = std::max<int64_t>(1, (int64_t)((size_t)256 << 20) / (int64_t)plane_bytes);
    S = std::min<int64_t>(S, N);
    const int64_t nslabs = (N + S - 1) / S;
    ecc_status st = ensure_streaming(ctx, (size_t)(std::min<int64_t>(S + 1, N)) * plane_bytes);
    if (st != ECC_OK) return st;
    // one scratch size for every slab (the first is the largest; for a 4D
    // image, that of its hyperplanes' 3D terms), fixed before anything is
    // enqueued so that no slab reallocates it
    Job first = vol;
    if (four) {
        first.ndim = 3;
        first.nw = 1;
        first.nvox = plane_vox;
    } else {
        first.g.n0 = std::min<int64_t>(S + 1, N);
        first.nvox = first.g.n0 * vol.g.n1 * vol.g.n2;
    }
    const Sizes sz = plan_sizes(ctx, first, nbins);
    if ((st = ensure_ws(ctx, sz.total)) != ECC_OK) return st;
    hipError_t e;
    // the slab buffers are free once work already on `stream` is done
    for (int b = 0; b < 2; ++b)
        if ((e = hipEventRecord(ctx->consumed[b], stream)) != hipSuccess)
            return hip_fail(ctx, e, "hipEventRecord(consumed)");
    const char* host = (const char*)vol.data;
    char* base = (char*)ctx->ws;
    ecc::BinParams* pdev = nullptr;
    if (vol.range_mode == ECC_RANGE_AUTO) {
        // pass 1: min/max keys of every slab's own planes, folded on the device
        uint32_t* mm = (uint32_t*)(base + sz.off_mm);
        uint32_t* acc = mm + 2 * kMinmaxBlocks;
        pdev = (ecc::BinParams*)(base + sz.off_params);
        for (int64_t k = 0; k < nslabs; ++k) {
            const int b = (int)(k & 1);
            const int64_t z0 = k * S, n = std::min<int64_t>(S, N - z0);
            if ((st = stream_copy(ctx, host, plane_bytes, z0, n, b)) != ECC_OK) return st;
            if ((e = hipStreamWaitEvent(stream, ctx->copied[b], 0)) != hipSuccess)
                return hip_fail(ctx, e, "hipStreamWaitEvent(compute)");
            const int64_t nv = n * plane_vox;
            const int blocks = (int)std::min<int64_t>(kMinmaxBlocks, (nv + 4095) / 4096);
            if ((e = ecc::launch_minmax(ctx->slab_buf[b], vol.dtype, nv, mm, blocks, stream)) != hipSuccess ||
                (e = ecc::launch_mm_fold(mm, blocks, acc, k == 0, stream)) != hipSuccess)
                return hip_fail(ctx, e, "streamed minmax launch");
            if ((e = hipEventRecord(ctx->consumed[b], stream)) != hipSuccess)
                return hip_fail(ctx, e, "hipEventRecord(consumed)");
        }
        if ((e = ecc::launch_params_from_minmax(acc, 1, vol.dtype, nbins, pdev, stream)) != hipSuccess)
            return hip_fail(ctx, e, "params launch");
    }
    // pass 2: slab k counts its own planes [k*S, k*S + n) and reads one collar
    // plane beyond them (the plane its last plane pairs with).  A 4D slab may
    // own no term (the top filtration's last hyperplane has c_w = 0 and no
    // pair): it is skipped, and the first and last slabs with terms write and
    // scan the output.
    auto has_terms = [&](int64_t z0, int64_t n) {
        if (!four || ctx->construction == ECC_VERTEX || N == 1) return true;
        const int64_t pairs = std::min<int64_t>(n, N - 1 - z0);
        return pairs > 0 || std::min<int64_t>(z0 + n, N - 1) > std::max<int64_t>(z0, 1);
    };
    int64_t k_first = -1, k_last = -1;
    for (int64_t k = 0; k < nslabs; ++k)
        if (has_terms(k * S, std::min<int64_t>(S, N - k * S))) {
            if (k_first < 0) k_first = k;
            k_last = k;
        }
    for (int64_t k = 0; k < nslabs; ++k) {
        const int b = (int)(k & 1);
        const int64_t z0 = k * S, n = std::min<int64_t>(S, N - z0);
        const int64_t loaded = std::min<int64_t>(n + 1, N - z0);
        if (four && !has_terms(z0, n)) continue;
        if ((st = stream_copy(ctx, host, plane_bytes, z0, loaded, b)) != ECC_OK) return st;
        if ((e = hipStreamWaitEvent(stream, ctx->copied[b], 0)) != hipSuccess)
            return hip_fail(ctx, e, "hipStreamWaitEvent(compute)");
        if (four) {
            Job h = first;
            h.data = nullptr;
            if ((st = enqueue_4d_part(ctx, base, sz, h, (const char*)ctx->slab_buf[b], loaded, pdev, nbins, stream,
                                      1, k == k_first, k == k_last, z0, N, n)) != ECC_OK)
                return st;
            if ((e = hipEventRecord(ctx->consumed[b], stream)) != hipSuccess)
                return hip_fail(ctx, e, "hipEventRecord(consumed)");
            continue;
        }
        Job slab = vol;
        slab.data = ctx->slab_buf[b];
        slab.g.n0 = loaded;
        slab.nvox = loaded * vol.g.n1 * vol.g.n2;
        Sizes ssz = plan_sizes(ctx, slab, nbins);
        ssz.off_counters = sz.off_counters;   // the layout of the scratch sized above
        if (ssz.total > sz.total) ssz = sz;
        if ((st = enqueue_hist(ctx, base, slab, nbins, stream, ssz, pdev, n, z0, N, k > 0, k == nslabs - 1)) != ECC_OK)
            return st;
        if ((e = hipEventRecord(ctx->consumed[b], stream)) != hipSuccess)
            return hip_fail(ctx, e, "hipEventRecord(consumed)");
    }
    return ECC_OK;
}

// A planned batch: its tables and partial rows live in device memory owned by
// the plan, written once at creation.
struct ecc_batch_plan {
    ecc_ctx* ctx = nullptr;
    std::vector<Job> jobs;
    int32_t nbins = 0;
    ecc_batch_shape shape = kDefaultBatchShape;
    BatchTables tables;
    void* dbuf = nullptr;
    size_t dbuf_bytes = 0;
};

// Builds the plan's tables for `shape` and uploads them (synchronously: the
// plan's earlier runs must have finished), growing its device buffer if needed.
ecc_status plan_upload(ecc_batch_plan* p, const ecc_batch_shape& shape)
{
    ecc_ctx* ctx = p->ctx;
    BatchTables T;
    build_batch_tables(ctx->cu_count, ctx->construction, p->jobs, p->nbins, T, shape);
    const BatchLayout& lay = T.lay;
    std::vector<char> host(lay.tables_end);
    pack_batch_tables(T, host.data());
    hipError_t e;
    if (lay.total > p->dbuf_bytes) {
        void* nb = nullptr;
        if ((e = hipMalloc(&nb, lay.total)) != hipSuccess) return hip_fail(ctx, e, "hipMalloc(batch plan)");
        if (p->dbuf) (void)hipFree(p->dbuf);
        p->dbuf = nb;
        p->dbuf_bytes = lay.total;
    }
    if ((e = hipMemcpy(p->dbuf, host.data(), lay.tables_end, hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(ctx, e, "hipMemcpy(batch plan tables)");
    p->tables = std::move(T);
    p->shape = shape;
    return ECC_OK;
}

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
    {
        // the fixed scratch of ecc_compute_noalloc on this device (once per
        // device; a failure here is reported by that entry point, which retries)
        DeviceGuard g(device);
        std::string ignored;
        if (g.ok) (void)noalloc_setup(device, ignored);
    }
    g_create_err.clear();
    *ctx = c;
    return ECC_OK;
}

ecc_status ecc_destroy(ecc_ctx* ctx)
{
    if (!ctx) return ECC_OK;
    {
        DeviceGuard g(ctx->device);
        if (ctx->ws) (void)hipFree(ctx->ws);
        for (auto& sl : ctx->staging) {
            if (sl.done) (void)hipEventSynchronize(sl.done);
            if (sl.ptr) (void)hipHostFree(sl.ptr);
            if (sl.done) (void)hipEventDestroy(sl.done);
        }
        for (hipEvent_t ev : ctx->tev) (void)hipEventDestroy(ev);
        for (int b = 0; b < 2; ++b) {
            if (ctx->slab_buf[b]) (void)hipFree(ctx->slab_buf[b]);
            if (ctx->copied[b]) (void)hipEventDestroy(ctx->copied[b]);
            if (ctx->consumed[b]) (void)hipEventDestroy(ctx->consumed[b]);
        }
        if (ctx->copy_stream) (void)hipStreamDestroy(ctx->copy_stream);
        if (ctx->smooth_tmp) (void)hipFree(ctx->smooth_tmp);
    }
    delete ctx;
    return ECC_OK;
}

ecc_status ecc_reserve(ecc_ctx* ctx, size_t scratch_bytes, size_t table_bytes)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (scratch_bytes > ((size_t)1 << 40) || table_bytes > ((size_t)1 << 30)) {
        ctx->err = "ecc_reserve: sizes beyond 1 TiB of scratch or 1 GiB of tables";
        return ECC_ERR_INVALID_ARG;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return hip_fail(ctx, hipErrorInvalidDevice, "hipSetDevice");
    ecc_status st = ensure_ws(ctx, std::max(scratch_bytes, kCounterBytes));
    if (st != ECC_OK) return st;
    if (table_bytes == 0) return ECC_OK;
    for (int i = 0; i < ecc_ctx::kStagingSlots; ++i) {
        ecc_ctx::Staging* sl = nullptr;
        if ((st = ensure_staging(ctx, table_bytes, &sl)) != ECC_OK) return st;
    }
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
    ecc_status st = validate(ctx, *img, nbins, "ecc_compute_ex", &j, ECC_MAX_NDIM);
    if (st != ECC_OK) return st;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    if (j.ndim >= 4) return enqueue_nd(ctx, j, nbins, (hipStream_t)hip_stream);
    return enqueue_one(ctx, j, nbins, (hipStream_t)hip_stream);
}

ecc_status ecc_compute_noalloc(ecc_ctx* ctx, const ecc_image* img, int32_t nbins, void* hip_stream)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!img) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_compute_noalloc: null descriptor");
    Job j;
    ecc_status st = validate(ctx, *img, nbins, "ecc_compute_noalloc", &j, 4);
    if (st != ECC_OK) return st;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    if (ctx->device < 0 || ctx->device >= kMaxDevices || !g_noalloc_ptr[ctx->device]) {
        if ((st = noalloc_setup(ctx->device, ctx->err)) != ECC_OK) return st;
    }
    if (j.ndim >= 4) return enqueue_nd(ctx, j, nbins, (hipStream_t)hip_stream, true);
    return enqueue_one(ctx, j, nbins, (hipStream_t)hip_stream, nullptr, true);
}

ecc_status ecc_compute(ecc_ctx* ctx, const void* image, int32_t ndim, const int64_t* dims,
                       int32_t dtype, int32_t nbins, int64_t* out, void* hip_stream)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!dims) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_compute: null dims");
    if (ndim < 2 || ndim > ECC_MAX_NDIM) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_compute: ndim must be in [2, 8]");
    ecc_image im;
    memset(&im, 0, sizeof im);
    im.data = image;
    im.ndim = ndim;
    im.dtype = dtype;
    for (int i = 0; i < ndim; ++i) im.dims[i] = dims[i];
    im.range_mode = ECC_RANGE_DEFAULT;
    im.out = out;
    Job j;
    ecc_status st = validate(ctx, im, nbins, "ecc_compute", &j, ECC_MAX_NDIM);
    if (st != ECC_OK) return st;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    if (j.ndim >= 4) return enqueue_nd(ctx, j, nbins, (hipStream_t)hip_stream);
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
    std::vector<Job> jobs((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        char where[64];
        snprintf(where, sizeof where, "ecc_compute_batch: image %d", i);
        ecc_status st = validate(ctx, imgs[i], nbins, where, &jobs[i], 4);
        if (st != ECC_OK) return st;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    return enqueue_batch(ctx, jobs, nbins, (hipStream_t)hip_stream);
}

ecc_status ecc_batch_schedule(const ecc_image* imgs, int32_t count, int32_t nbins, int32_t construction,
                              const ecc_batch_shape* shape,
                              int32_t cu_count, int32_t* segments, int64_t* max_segment_voxels,
                              int64_t* image_bricks, int64_t* covered_bricks)
{
    g_create_err.clear();
    if (count < 1 || !imgs || cu_count < 1 || !segments || !max_segment_voxels) {
        g_create_err = "ecc_batch_schedule: bad argument";
        return ECC_ERR_INVALID_ARG;
    }
    if (construction != ECC_VERTEX && construction != ECC_TOP) {
        g_create_err = "ecc_batch_schedule: unknown construction";
        return ECC_ERR_INVALID_ARG;
    }
    ecc_batch_shape sh = shape ? *shape : kDefaultBatchShape;
    if (sh.depth3 < 1 || sh.depth2 < 1 || sh.wgs_per_cu < 1) {
        g_create_err = "ecc_batch_schedule: shape fields must be positive";
        return ECC_ERR_INVALID_ARG;
    }
    ecc_ctx probe;   // carries validation messages only; owns no device resource
    std::vector<Job> jobs((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        char where[64];
        snprintf(where, sizeof where, "ecc_batch_schedule: image %d", i);
        const ecc_status st = validate(&probe, imgs[i], nbins, where, &jobs[(size_t)i], 4);
        if (st != ECC_OK) {
            g_create_err = probe.err;
            return st;
        }
    }
    BatchTables T;
    build_batch_tables(cu_count, construction, jobs, nbins, T, sh);
    int64_t mx = 0;
    std::vector<int64_t> cov((size_t)count, 0);
    for (const auto& sg : T.segs) {
        const int64_t v = (sg.b1 - sg.b0) * ecc::batch_brick_voxels(T.images[(size_t)sg.image]);
        mx = std::max(mx, v);
        cov[(size_t)T.images[(size_t)sg.image].owner] += sg.b1 - sg.b0;
    }
    *segments = (int32_t)T.segs.size();
    *max_segment_voxels = mx;
    for (int32_t i = 0; i < count; ++i) {
        if (image_bricks) image_bricks[i] = T.owner_bricks[(size_t)i];
        if (covered_bricks) covered_bricks[i] = cov[(size_t)i];
    }
    return ECC_OK;
}

ecc_status ecc_set_kernel_timing(ecc_ctx* ctx, int32_t enable)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    if (!enable) {
        ctx->timing = false;
        ctx->tused = 0;
        ctx->tms = 0.0;
        ctx->tcount = 0;
        return ECC_OK;
    }
    if (ctx->tev.empty()) {
        std::vector<hipEvent_t> ev(2 * kTimingPairs, nullptr);
        for (size_t i = 0; i < ev.size(); ++i) {
            hipError_t e = hipEventCreate(&ev[i]);
            if (e != hipSuccess) {
                for (size_t k = 0; k < i; ++k) (void)hipEventDestroy(ev[k]);
                return hip_fail(ctx, e, "hipEventCreate(timing)");
            }
        }
        ctx->tev.swap(ev);
    }
    ctx->timing = true;
    return ECC_OK;
}

ecc_status ecc_kernel_time(ecc_ctx* ctx, double* total_ms, int64_t* launches)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!total_ms || !launches) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_kernel_time: null output pointer");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    ecc_status st = fold_timing(ctx);
    if (st != ECC_OK) return st;
    *total_ms = ctx->tms;
    *launches = ctx->tcount;
    ctx->tms = 0.0;
    ctx->tcount = 0;
    return ECC_OK;
}

ecc_status ecc_batch_plan_create(ecc_ctx* ctx, const ecc_image* imgs, int32_t count, int32_t nbins,
                                 ecc_batch_plan** plan)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!plan) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_batch_plan_create: null plan pointer");
    *plan = nullptr;
    if (count < 1) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_batch_plan_create: count must be at least 1");
    if (!imgs) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_batch_plan_create: null descriptor array");
    std::vector<Job> jobs((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        char where[64];
        snprintf(where, sizeof where, "ecc_batch_plan_create: image %d", i);
        ecc_status st = validate(ctx, imgs[i], nbins, where, &jobs[i], 4);
        if (st != ECC_OK) return st;
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    ecc_batch_plan* p = new (std::nothrow) ecc_batch_plan;
    if (!p) return fail(ctx, ECC_ERR_OUT_OF_MEMORY, "ecc_batch_plan_create: out of host memory");
    p->ctx = ctx;
    p->jobs = std::move(jobs);
    p->nbins = nbins;
    const ecc_status st = plan_upload(p, kDefaultBatchShape);
    if (st != ECC_OK) {
        if (p->dbuf) (void)hipFree(p->dbuf);
        delete p;
        return st;
    }
    *plan = p;
    return ECC_OK;
}

ecc_status ecc_batch_plan_launch(ecc_batch_plan* plan, void* hip_stream)
{
    if (!plan) return ECC_ERR_INVALID_ARG;
    ecc_ctx* ctx = plan->ctx;
    ctx->err.clear();
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    return launch_batch_kernels(ctx, plan->tables, (char*)plan->dbuf, true, (hipStream_t)hip_stream);
}

ecc_status ecc_batch_plan_destroy(ecc_batch_plan* plan)
{
    if (!plan) return ECC_OK;
    {
        DeviceGuard g(plan->ctx->device);
        if (plan->dbuf) (void)hipFree(plan->dbuf);
    }
    delete plan;
    return ECC_OK;
}

ecc_status ecc_batch_plan_autotune(ecc_batch_plan* plan, int32_t reps, void* hip_stream, ecc_batch_shape* chosen)
{
    if (!plan) return ECC_ERR_INVALID_ARG;
    ecc_ctx* ctx = plan->ctx;
    ctx->err.clear();
    if (reps < 1 || reps > 1000)
        return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_batch_plan_autotune: reps must be in [1, 1000]");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t stream = (hipStream_t)hip_stream;
    hipError_t e;
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
    // candidates: brick depths (3D planes, 2D rows) and workgroups per CU
    std::vector<ecc_batch_shape> cand;
    for (int wgs : {1, 2, 3, 4})
        for (const auto& d : {std::pair<int, int>{4, 32}, {8, 64}, {16, 128}})
            cand.push_back(ecc_batch_shape{d.first, d.second, wgs, 0, 0.0});
    const ecc_batch_shape before = plan->shape;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if ((e = hipEventCreate(&t0)) != hipSuccess || (e = hipEventCreate(&t1)) != hipSuccess) {
        if (t0) (void)hipEventDestroy(t0);
        return hip_fail(ctx, e, "hipEventCreate");
    }
    ecc_status st = ECC_OK;
    ecc_batch_shape best = before;
    best.ms = -1.0;
    for (auto& c : cand) {
        if ((st = plan_upload(plan, c)) != ECC_OK) break;
        // one untimed run, then `reps` timed ones
        if ((st = launch_batch_kernels(ctx, plan->tables, (char*)plan->dbuf, true, stream)) != ECC_OK) break;
        if ((e = hipEventRecord(t0, stream)) != hipSuccess) { st = hip_fail(ctx, e, "hipEventRecord"); break; }
        for (int r = 0; r < reps && st == ECC_OK; ++r)
            st = launch_batch_kernels(ctx, plan->tables, (char*)plan->dbuf, true, stream);
        if (st != ECC_OK) break;
        float ms = 0.f;
        if ((e = hipEventRecord(t1, stream)) != hipSuccess || (e = hipEventSynchronize(t1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, t0, t1)) != hipSuccess) {
            st = hip_fail(ctx, e, "batch timing");
            break;
        }
        c.ms = ms / reps;
        if (best.ms < 0 || c.ms < best.ms) best = c;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (st == ECC_OK && (e = hipStreamSynchronize(stream)) != hipSuccess) st = hip_fail(ctx, e, "hipStreamSynchronize");
    const ecc_status st2 = plan_upload(plan, st == ECC_OK ? best : before);
    if (st != ECC_OK) return st;
    if (st2 != ECC_OK) return st2;
    // the outputs hold the batch's ECCs
    if ((st = launch_batch_kernels(ctx, plan->tables, (char*)plan->dbuf, true, stream)) != ECC_OK) return st;
    if ((e = hipStreamSynchronize(stream)) != hipSuccess) return hip_fail(ctx, e, "hipStreamSynchronize");
    plan->shape = best;
    if (chosen) *chosen = best;
    return ECC_OK;
}

ecc_status ecc_set_launch_shape(ecc_ctx* ctx, const ecc_image* img, int32_t nbins, const ecc_launch_shape* shape)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!img || !shape) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_set_launch_shape: null pointer");
    if (shape->waves > ecc::kMaxWaves || shape->wgs_per_cu > 16 || shape->depth > 4096 ||
        shape->window > ecc::kMaxLdsBins ||
        (shape->copies != 0 && shape->copies != 2 && shape->copies != 4 && shape->copies != 8))
        return fail(ctx, ECC_ERR_INVALID_ARG,
                    "ecc_set_launch_shape: waves must be at most 9, wgs_per_cu at most 16, depth at most 4096, "
                    "window at most 4096, copies 0, 2, 4 or 8");
    Job j;
    ecc_status st = validate(ctx, *img, nbins, "ecc_set_launch_shape", &j, ECC_MAX_NDIM);
    if (st != ECC_OK) return st;
    ecc_launch_shape c = *shape;
    c.ms = 0.0;
    ctx->tuned[tune_key(ctx, j, nbins)] = c;
    return ECC_OK;
}

ecc_status ecc_autotune(ecc_ctx* ctx, const ecc_image* img, int32_t nbins, int32_t reps, void* hip_stream,
                        ecc_launch_shape* chosen)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!img) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_autotune: null descriptor");
    if (reps < 1 || reps > 1000) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_autotune: reps must be in [1, 1000]");
    Job j;
    ecc_status st = validate(ctx, *img, nbins, "ecc_autotune", &j, ECC_MAX_NDIM);
    if (st != ECC_OK) return st;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    hipStream_t stream = (hipStream_t)hip_stream;
    const TuneKey key = tune_key(ctx, j, nbins);
    ctx->tuned.erase(key);
    // candidates: the default shape, then waves, depth and workgroups per CU
    // around it (every shape gives the same result; only the time differs); an
    // image of 4 or more dimensions is tuned for its 3D passes (the shape of
    // its last three axes)
    Job shape_job = j;
    if (j.ndim >= 4) {
        shape_job.ndim = 3;
        shape_job.nw = 1;
        shape_job.nvox = j.g.n0 * j.g.n1 * j.g.n2;
    }
    const Sizes def = plan_sizes(ctx, shape_job, nbins);
    auto run = [&](const ecc_launch_shape* c) {
        return j.ndim >= 4 ? enqueue_nd(ctx, j, nbins, stream, false, c) : enqueue_one(ctx, j, nbins, stream, c);
    };
    const int64_t cols = (ecc::axis_positions(j.g.n2, ctx->construction) + ecc::kLaneCols - 1) / ecc::kLaneCols;
    std::vector<ecc_launch_shape> cand;
    auto add = [&](int waves, int64_t depth, int wgs, int32_t window = 0, int32_t copies = 0) {
        ecc_launch_shape c = {};
        c.waves = (int32_t)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(waves, ecc::kMaxWaves), cols));
        c.depth = std::max<int64_t>(1, depth);
        c.wgs_per_cu = wgs;
        c.window = window;
        c.copies = copies;
        for (const auto& e : cand)
            if (e.waves == c.waves && e.depth == c.depth && e.wgs_per_cu == c.wgs_per_cu && e.window == c.window &&
                e.copies == c.copies)
                return;
        cand.push_back(c);
    };
    const int def_wgs = j.ndim == 2 ? ECC_MAX_WGS_PER_CU_2D : ECC_MAX_WGS_PER_CU_3D;
    add(def.waves, def.depth, def_wgs);
    for (int wgs : {1, 2, 3, 4})
        for (int64_t dm : {1, 2, 4}) {
            add(def.waves, def.depth * dm / 2, wgs);
            if (def.waves > 4) add((def.waves + 1) / 2, def.depth * dm / 2, wgs);
        }
    // a 3D row whose default packs its narrow tail (one wave fewer than the
    // row's chunks, ecc::layout_3d): also one chunk with the tail in its last wave
    if (shape_job.ndim == 3 && def.waves + 1 == cols && cols <= ECC_MAX_WAVES_3D)
        for (int wgs : {2, 3, 4})
            for (int64_t dm : {1, 2}) add((int)cols, def.depth * dm, wgs);
    // 3D: for each workgroup count, the plane depth (between half and twice the
    // default) whose bricks split most evenly over the workgroups: the slowest
    // workgroup walks ceil(bricks / grid) bricks of depth planes plus about one
    // and a half planes of start-up each
    if (shape_job.ndim == 3) {
        const int64_t per_z = ecc::layout_3d(shape_job.g, ctx->construction, def.waves).per_z;
        const int resident = ecc::resident_wgs_per_cu(3, j.dtype, ctx->construction, def.window < nbins, def.waves,
                                                      def.lds_bytes);
        for (int wgs : {2, 3, 4}) {
            const int64_t grid = (int64_t)ctx->cu_count * std::min(wgs, resident);
            int64_t best_d = def.depth;
            double best_cost = HUGE_VAL;
            for (int64_t d = std::max<int64_t>(4, def.depth / 2); d <= 2 * def.depth; ++d) {
                const int64_t bricks = per_z * ((shape_job.g.n0 + d - 1) / d);
                const double cost = (double)((bricks + grid - 1) / grid) * ((double)d + 1.5);
                if (cost < best_cost) {
                    best_cost = cost;
                    best_d = d;
                }
            }
            add(def.waves, best_d, wgs);
        }
    }
    // the bins-per-pass split: half the window (two passes, half the LDS each)
    // at the default shape and with more workgroups per CU, which the smaller
    // LDS allows
    if (def.window >= 2048)
        for (int wgs : {def_wgs, def_wgs + 2}) add(def.waves, def.depth, wgs, def.window / 2);
    // histogram copies for narrow windows (few bins leave LDS for more)
    if (def.window <= 1024)
        for (int copies : {2, 4, 8}) add(def.waves, def.depth, def_wgs, 0, copies);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(ctx, e, "hipEventCreate(autotune)");
    }
    // Times `n` calls of shape c on the stream, in milliseconds per call.
    auto timed = [&](const ecc_launch_shape& c, int n, double* ms_per_call) -> ecc_status {
        ecc_status r = ECC_OK;
        if ((e = hipEventRecord(e0, stream)) != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
        for (int k = 0; k < n && r == ECC_OK; ++k) r = run(&c);
        if (r != ECC_OK) return r;
        if ((e = hipEventRecord(e1, stream)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
            return hip_fail(ctx, e, "hipEventSynchronize(autotune)");
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
        *ms_per_call = ms / n;
        return ECC_OK;
    };
    // The device's clocks rise over the first tenths of a second of load, which
    // would favour the candidates timed last: the default shape runs first
    // until 40 ms of calls (at most 400) have passed; then every candidate is
    // timed in two rounds (one warm-up call each the first time) and keeps the
    // faster of its two times.
    {
        double ms = 0.0, total = 0.0;
        for (int k = 0; k < 100 && total < 40.0 && st == ECC_OK; ++k) {
            st = timed(cand[0], 4, &ms);
            total += 4.0 * ms;
        }
    }
    for (auto& c : cand) c.ms = HUGE_VAL;
    for (int round = 0; round < 2 && st == ECC_OK; ++round) {
        for (auto& c : cand) {
            if (round == 0 && (st = run(&c)) != ECC_OK) break;   // warm-up, sizes the scratch
            double ms = 0.0;
            if ((st = timed(c, reps, &ms)) != ECC_OK) break;
            c.ms = std::min(c.ms, ms);
        }
    }
    ecc_launch_shape best = cand[0];
    for (const auto& c : cand)
        if (c.ms < best.ms) best = c;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != ECC_OK) return st;
    ctx->tuned[key] = best;
    if (chosen) *chosen = best;
    return ECC_OK;
}

ecc_status ecc_compute_streamed(ecc_ctx* ctx, const ecc_image* img, int32_t nbins, int64_t slab_planes,
                                void* hip_stream)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!img) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_compute_streamed: null descriptor");
    if (slab_planes < 0) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_compute_streamed: negative slab_planes");
    Job j;
    ecc_status st = validate(ctx, *img, nbins, "ecc_compute_streamed", &j, 4);
    if (st != ECC_OK) return st;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    if (j.ndim == 2) {   // a 2D image travels as one slab of one plane
        j.ndim = 3;
        j.g = {1, j.g.n1, j.g.n2};
    }
    return enqueue_streamed(ctx, j, nbins, slab_planes, (hipStream_t)hip_stream);
}

ecc_status ecc_smooth13(ecc_ctx* ctx, const float* in, float* out, int64_t n1, int64_t n2, const float* taps,
                        void* hip_stream)
{
    if (!ctx) return ECC_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!in || !out || !taps) return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_smooth13: null pointer");
    if (n1 < 1 || n2 < 1 || n1 > (int64_t(1) << 31) || n2 > (int64_t(1) << 31) || n1 * n2 > (int64_t(1) << 40))
        return fail(ctx, ECC_ERR_INVALID_ARG, "ecc_smooth13: dims out of range");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, ECC_ERR_DEVICE, "hipSetDevice failed");
    const size_t bytes = (size_t)n1 * (size_t)n2 * sizeof(float);
    hipError_t e;
    if (bytes > ctx->smooth_cap) {
        if (ctx->smooth_tmp) {
            if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
            (void)hipFree(ctx->smooth_tmp);
            ctx->smooth_tmp = nullptr;
            ctx->smooth_cap = 0;
        }
        if ((e = hipMalloc(&ctx->smooth_tmp, bytes)) != hipSuccess) {
            ctx->smooth_tmp = nullptr;
            return hip_fail(ctx, e, "hipMalloc(smoothing buffer)");
        }
        ctx->smooth_cap = bytes;
    }
    ecc::Taps13 w;
    for (int k = 0; k < 13; ++k) w.w[k] = taps[k];
    if ((e = ecc::launch_smooth13(in, out, (float*)ctx->smooth_tmp, n1, n2, w, (hipStream_t)hip_stream)) !=
        hipSuccess)
        return hip_fail(ctx, e, "smoothing launch");
    return ECC_OK;
}

}  // extern "C"
