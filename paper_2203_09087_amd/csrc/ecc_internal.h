// ecc_internal.h -- types shared by the host runtime and the kernels of the ECC
// library.  Not part of the public interface (include/ecc.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecc {

enum : int32_t { DT_U8 = 0, DT_U16 = 1, DT_F32 = 2 };
enum : int32_t { CONS_VERTEX = 0, CONS_TOP = 1 };

// Bin of a value (the library's reading of the paper's gray-level histogram
// index for data that is not 0..255 integers):
//   integer data: a = clamp(v, ilo, ihi) - ilo ; bin = floor(a * nbins / D),
//                 D = ihi-ilo+1 (bin = a when nbins == D), computed as the
//                 double product (a * nbins) * rcp with rcp = 1/D rounded up,
//                 which is exact because a * nbins < 2^32 and D <= 65536;
//   float data:   NaN -> nbins-1; flat range -> (x > hi ? nbins-1 : 0);
//                 otherwise clamp(floor(((double)x - lo) * scale), 0, nbins-1),
//                 scale = nbins / (hi - lo) (+inf for a flat range, which with
//                 the next double above lo as subtrahend gives the flat rule
//                 through the same formula).
struct BinParams {
    int32_t dtype;
    int32_t nbins;
    uint32_t ilo, ihi;  // integer range
    int32_t flat;       // float data, hi == lo
    int32_t ident;      // integer data, nbins == D = hi - lo + 1: bin = level - lo
    double lo, hi;      // the range used
    double base;        // float data: subtrahend (lo, or the next double above lo if flat)
    double scale;       // float data: nbins / (hi - lo), +inf if flat
    double rcp;         // integer data: 1 / D rounded up
};

// Geometry of one image: n0 slowest.  For 2D images n0 is 1.
struct Geom {
    int64_t n0, n1, n2;
};

// Histogram window: bins [bin_lo, bin_lo + width) are accumulated in LDS.
constexpr int kMaxLdsBins = 4096;

// Brick shapes of the wave kernels (64 x-lanes, 63 of them owned).  The
// ECC_* macros exist for tuning builds; the defaults are the shipped shapes.
#ifndef ECC_ROWS3
#define ECC_ROWS3 3
#endif
#ifndef ECC_CHUNK2
#define ECC_CHUNK2 16
#endif
#ifndef ECC_WAVES_PER_EU_3D
#define ECC_WAVES_PER_EU_3D 5   // resident waves per SIMD the 3D kernels are compiled for
#endif
#ifndef ECC_WAVES_PER_EU_BATCH
#define ECC_WAVES_PER_EU_BATCH 6   // the batched kernel: at most 80 vector registers, so two 9-wave workgroups fit a CU
#endif
#ifndef ECC_WAVES_PER_EU_2D
#define ECC_WAVES_PER_EU_2D 5   // resident waves per SIMD the 2D kernels are compiled for
#endif
#ifndef ECC_MAX_WAVES_3D
#define ECC_MAX_WAVES_3D 9   // waves per workgroup of a single 3D image (a whole row up to 567 positions)
#endif
#ifndef ECC_MAX_WGS_PER_CU_3D
#define ECC_MAX_WGS_PER_CU_3D 2   // resident workgroups per CU a single 3D image launches
#endif
#ifndef ECC_MAX_WGS_PER_CU_2D
#define ECC_MAX_WGS_PER_CU_2D 3   // resident workgroups per CU a single 2D image launches
#endif
// A key is 4 * bin: the LDS byte address of its counter.
constexpr int kKeyShift = 2;
// A workgroup histogram is kept in several copies, lane l of every wave adding to
// copy l mod copies: equal keys of neighbouring lanes (frequent in smooth images)
// then fall into different copies, each starting 8 words further in the bank
// cycle than the one before, so they do not collide in one LDS bank.  The merge
// adds the copies.  Two copies for wide windows; a narrow window affords more
// (hist_copies), which smooth data with few bins needs.  The LDS a launch takes
// is sized to its window and copies (dynamic shared memory), so a histogram of
// few bins leaves room for more workgroups.
constexpr int kHistCopies = 2;   // copies of a window wider than 1024 bins
constexpr int kMaxHistCopies = 8;
// Default copies for a window of `width` bins: 8 up to 256 bins, 4 up to 1024.
inline __host__ __device__ uint32_t hist_copies(int32_t width)
{
    return width <= 256 ? 8u : (width <= 1024 ? 4u : (uint32_t)kHistCopies);
}
// Words from one copy to the next for a window of `width` bins (a multiple of 32
// plus 8: the 8-bank offset; with windows the word after the window is spare).
inline __host__ __device__ uint32_t lds_stride(int32_t width)
{
    return ((uint32_t)width + 31u) / 32u * 32u + 8u;
}
// Sentinel key of a one-window launch of nbins bins: 4 (2^k - 1) with 2^k > nbins,
// so it is above every key (4 * bin, bin < nbins) and OR-ing it into a key gives it.
inline __host__ __device__ uint32_t lds_sentinel(int32_t nbins)
{
    uint32_t p = 1;
    while (p <= (uint32_t)nbins) p <<= 1;
    return 4u * (p - 1u);
}
// LDS words of a workgroup histogram: the copies and, with one window, spare
// words up to the second copy's sentinel word, which absorbs the counts of
// cells that do not exist (4096 bins: 12,296 words).
inline __host__ __device__ uint32_t lds_words(int32_t width, bool windowed, uint32_t sentinel, uint32_t copies)
{
    const uint32_t stride = lds_stride(width);
    return windowed ? copies * stride : stride * (copies - 1) + sentinel / 4u + 1u;
}
// Positions a wave owns along x (lanes 0..62; lane 63 only supplies lane 62's
// right neighbour).
constexpr int kLaneCols = 63;
// Positions along an axis of n voxels that carry a single or a pair (the cell
// types of the kernels): n for the vertex filtration; n + 1 lattice points for
// the top filtration (the first one before voxel 0).
inline __host__ __device__ int64_t axis_positions(int64_t n, int construction)
{
    return n + (construction == CONS_TOP ? 1 : 0);
}
constexpr int kRows3 = ECC_ROWS3;      // rows per 3D brick
constexpr int kChunk2 = ECC_CHUNK2;    // rows loaded together in the 2D kernel
// Waves per workgroup of the main kernels (x-chunk = waves * 63 position columns).
constexpr int kMaxWaves = 9;

// Workgroup bricks of a single 3D image (k_ecc_3d).  Ordinary bricks are an
// x-chunk of 63 * waves position columns x kRows3 rows (a strip) x `depth`
// planes, each wave on 63 columns of the chunk.  When the positions of a row
// leave a narrow tail after the full chunks (t < 32 columns), a wave on the
// tail would own t of its 63 lanes; instead the tail is packed: t + 1 lanes per
// strip (t owning, one supplying the right neighbour), floor(64 / (t + 1))
// strips per wave, for the strips whose rows (and the row after them) all lie
// in the image; the few other strips' tails run as ordinary bricks.  A 512-wide
// row then takes 8 waves of 63 columns and a packed tail of 8 instead of a
// ninth wave with 8 columns.
struct Layout3 {
    int64_t nxc;        // x-chunks of the ordinary bricks of each strip (full ones)
    int64_t nyb;        // strips
    int64_t t;          // positions of the tail (0: none)
    int64_t spw;        // tail strips per wave (0: the tail is not packed)
    int64_t sa, sb;     // strips [sa, sb) have packed tails
    int64_t npk;        // packed bricks per plane block
    int64_t per_z;      // bricks per plane block
};
inline __host__ __device__ Layout3 layout_3d(const Geom& g, int construction, int waves)
{
    Layout3 y = {};
    const int64_t cw = (int64_t)kLaneCols * waves;
    const int64_t xpos = axis_positions(g.n2, construction);
    const int64_t org = construction == CONS_TOP ? -1 : 0;
    y.nyb = (axis_positions(g.n1, construction) + kRows3 - 1) / kRows3;
    y.nxc = xpos / cw;
    y.t = xpos - y.nxc * cw;
    // strip s reads rows org + 3s .. org + 3s + 3 (the last one completes pairs)
    y.sa = org < 0 ? 1 : 0;
    y.sb = g.n1 - kRows3 - 1 - org >= 0 ? (g.n1 - kRows3 - 1 - org) / kRows3 + 1 : 0;
    if (y.sb > y.nyb) y.sb = y.nyb;
    const int64_t group = y.t + 1;
    // a lane's rows are up to (3 spw + 1) rows past the wave's first: 32-bit offsets
    const int64_t row_bytes = g.n2 * 4;
    const bool pack = y.t > 0 && group <= 32 && y.sb > y.sa &&
                      (kRows3 * (64 / group) + 1) * row_bytes < (int64_t(1) << 31);
    if (pack) {
        y.spw = 64 / group;
        const int64_t per_brick = y.spw * waves;
        y.npk = (y.sb - y.sa + per_brick - 1) / per_brick;
        y.per_z = y.nxc * y.nyb + y.npk + (y.nyb - (y.sb - y.sa));
    } else {
        if (y.t > 0) y.nxc += 1;
        y.t = 0;
        y.sa = y.sb = 0;
        y.per_z = y.nxc * y.nyb;
    }
    return y;
}

struct EccLaunch {
    const void* data;
    const void* data2;             // non-null (3D): count the elementwise max (min) of data and data2
    int ndim, dtype, construction;
    Geom g;
    const BinParams* params_dev;   // non-null: read the parameters from device memory
    BinParams params;              // used when params_dev is null
    int32_t bin_lo, width;
    int32_t windowed;              // nbins > width: skip bins outside the window
    int32_t grid;                  // number of workgroups
    int32_t waves;                 // waves per workgroup (x-chunk = 63 * waves position columns)
    int64_t depth;                 // planes (3D) or rows (2D) per workgroup brick
    // 3D slab of a larger volume (streaming): planes [0, z_own) of the g.n0 in
    // memory are counted (a plane beyond them is the collar the last one needs);
    // plane 0 is plane z_base of a volume of n0_global planes.  A whole image
    // has z_own = g.n0, z_base = 0, n0_global = g.n0.
    int64_t z_own, z_base, n0_global;
    // Several passes of the same shape in one launch (3D): workgroup row y of
    // the grid (grid x npass workgroups) counts the volume at data (and data2)
    // plus y * pass_stride bytes; its histograms go to partial rows y * grid ..
    int32_t npass;
    int64_t pass_stride;
    int32_t* partials;             // [grid * npass][width] workgroup histograms
    int32_t flush_add;             // add the workgroup histogram to its partial row (else write it)
    int32_t flush_sign;            // +1, or -1: the histogram enters its row negated
    int64_t* out;                  // the caller's output
    uint32_t* counter;             // counters[0]: the merge's; counters[1]: the fused merge's
    int32_t fused;                 // one window, few rows: the last workgroup merges and scans into out
    uint32_t hist_stride;          // LDS words between the histogram copies (lds_stride(width))
    uint32_t hist_copies;          // copies of the histogram (a power of two up to kMaxHistCopies)
    uint32_t sentinel;             // one-window sentinel key (lds_sentinel(nbins))
    uint32_t lds_bytes;            // dynamic LDS of the launch (lds_words * 4)
};
// Partial-row words (grid x window) up to which the histogram kernel merges its
// own rows (fused_merge_scan) instead of launching the two merge kernels.
constexpr int64_t kFusedMergeWords = int64_t(1) << 16;

// ---------------------------------------------------------------- batches

// One volume of a batch, as the batched kernels see it.  The first `count`
// entries are the batch's images (their outputs, ranges and min/max keys); a 2D
// or 3D image is also the volume that is counted.  A 4D image is counted as
// signed 3D volumes (its hyperplanes and the max/min of adjacent pairs) listed
// after the images, each naming its image as `owner`; its own entry is counted
// by none.
struct BatchImage {
    const void* data;
    const void* data2;    // a pair volume: count the max (vertex) or min (top) of data and data2
    Geom g;
    int32_t ndim, dtype;
    int32_t auto_range;   // parameters come from the min/max keys mm[2*owner], mm[2*owner+1]
    int32_t nxc;          // x-chunks of 63 * wpb position columns
    int32_t nyb;          // row blocks (3D: kRows3 rows; 2D: `depth` rows)
    int32_t wpb;          // waves per brick; a workgroup works on kBatchWaves / wpb bricks side by side
    int32_t sign;         // +1, or -1: the volume's histogram enters its image's rows negated
    int32_t owner;        // the image whose output, range and partial rows the volume uses
    int64_t depth;        // planes (3D) or rows (2D) per brick
    int64_t nvox;
    BinParams params;     // explicit or default range
    int64_t* out;         // the caller's output, nbins int64
};

// A run of consecutive bricks [b0, b1) of one volume (an index into the images)
// handled by one workgroup; its histogram lands in partial row `slot`.
struct BatchSeg {
    int32_t image;
    int32_t slot;
    int64_t b0, b1;
};

// A contiguous piece of one AUTO-range image for the batched min/max pass.
struct BatchPiece {
    int32_t image;
    int32_t pad;
    int64_t begin, end;   // element range
};

struct BatchLaunch {
    const BatchImage* images;
    int32_t count;
    int32_t dtype;              // the launch serves the images of this dtype
    const BatchSeg* segs;
    const int32_t* wg_seg;      // workgroup g runs segs[wg_seg[g] .. wg_seg[g+1])
    const int32_t* slot_off;    // image i owns partial rows slots[slot_off[i] .. slot_off[i+1])
    const int32_t* slots;
    uint32_t* mm;               // [count][2] min/max keys of AUTO images
    int32_t* partials;          // [nslots][width]
    int32_t nbins, bin_lo, width, windowed;
    int32_t grid, waves;
    int32_t pairs;              // the launch counts pair volumes (4D images)
    uint32_t hist_stride, hist_copies, sentinel, lds_bytes;   // LDS layout, as in EccLaunch
};

// Launchers (ecc_batch.hip).
hipError_t launch_minmax_batch(const BatchImage* images, const BatchPiece* pieces, int npieces, uint32_t* mm,
                               hipStream_t s);
hipError_t launch_ecc_batch(const BatchLaunch& B, int construction, hipStream_t s, hipEvent_t t0 = nullptr,
                            hipEvent_t t1 = nullptr);
// Sets mm[2i] = ~0, mm[2i+1] = 0 for the `count` images (a kernel, so that the
// enqueue stays valid inside a captured graph).
hipError_t launch_mm_init(uint32_t* mm, int count, hipStream_t s);
// Sums every image's partial rows into its out[bin_lo .. bin_lo+width) and, with
// `scan`, prefix-sums its out[0 .. nbins).
hipError_t launch_merge_batch(const BatchLaunch& B, bool scan, hipStream_t s);
// Bricks of one batch image for the batched launch shape (sets nxc, nyb, depth):
// 3D bricks of depth3 planes, 2D bricks of depth2 rows (a multiple of kChunk2).
int64_t batch_bricks(BatchImage& im, int construction, int waves, int depth3, int depth2);
// Voxels of one brick of a batch image whose shape batch_bricks has set (whole
// brick, including any part outside the image).
int64_t batch_brick_voxels(const BatchImage& im);
#ifndef ECC_BATCH_WAVES
#define ECC_BATCH_WAVES 9
#endif
constexpr int kBatchWaves = ECC_BATCH_WAVES;   // waves per workgroup of the batched kernel

// Launchers (ecc_kernels.hip: histogram kernels; ecc_reduce.hip: min/max,
// parameters, merge).  All enqueue on `s` and return the launch status.

// 13 smoothing taps (ecc_smooth.hip): tap k weights the neighbour at offset k - 6.
struct Taps13 {
    float w[13];
};
// Rows (in -> tmp), then columns (tmp -> out) of an n1 x n2 float image; out may be in.
hipError_t launch_smooth13(const float* in, float* out, float* tmp, int64_t n1, int64_t n2, const Taps13& w,
                           hipStream_t s);
hipError_t launch_minmax(const void* data, int dtype, int64_t nvox, uint32_t* mm_out, int blocks,
                         hipStream_t s);
// Elementwise max (take_max) or min of the n values at a and b into out, NaN
// taken as the largest float (the reduction of images of 5+ dimensions).
hipError_t launch_combine(const void* a, const void* b, void* out, int64_t n, int dtype, bool take_max,
                          hipStream_t s);
hipError_t launch_params_from_minmax(const uint32_t* mm, int blocks, int dtype, int32_t nbins,
                                     BinParams* out, hipStream_t s);
hipError_t launch_ecc(const EccLaunch& L, hipStream_t s, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
// Sums the `rows` partial histograms into out[bin_lo..bin_lo+width) (through
// `level2`, kLevel2Words int64 of scratch) and, with `scan`, prefix-sums
// out[0..nbins).  counters[0] is the merge's last-block counter, which the merge
// re-arms.
constexpr int kMergeGroups = 32;
// group sums (kMergeGroups x window) and per-group totals of 256-bin blocks
constexpr size_t kLevel2Words = (size_t)kMergeGroups * (kMaxLdsBins + kMaxLdsBins / 256);
constexpr int kCounterWords = 256;
// accumulate: add to out instead of writing it (slabs of a streamed volume, the
// 3D passes of a 4D image); sign -1: subtract the sums.
hipError_t launch_merge(const int32_t* partials, int rows, int32_t width, int32_t bin_lo, int64_t* level2,
                        int64_t* out, int32_t nbins, uint32_t* counters, bool accumulate, bool scan, int sign,
                        hipStream_t s);
// Folds `blocks` min/max key pairs into the running pair acc (first: start it).
hipError_t launch_mm_fold(const uint32_t* mm, int blocks, uint32_t* acc, bool first, hipStream_t s);

// Workgroup bricks of an image for a launch shape.
int64_t wg_bricks(int ndim, int construction, const Geom& g, int waves, int64_t depth);
// Workgroups of the main kernel variant (of `waves` waves, lds_bytes of dynamic
// LDS) that fit on one CU.
int resident_wgs_per_cu(int ndim, int dtype, int construction, bool windowed, int waves, uint32_t lds_bytes);

}  // namespace ecc
