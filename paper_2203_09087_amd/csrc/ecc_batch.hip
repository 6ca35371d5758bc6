// ecc_batch.hip -- the batched form: the ECCs of many images of uneven sizes and
// dimensions in one persistent launch.
//
// The host cuts the bricks of all images (in order) into one contiguous run per
// workgroup, balanced by work, and lists each run as segments of single images.
// A workgroup processes its segments in order with the same brick bodies as the
// single-image kernels, and writes one partial histogram row per segment.  The
// merge kernels then give every image the sum of its rows (and its prefix scan)
// without any atomic operation on the histogram bins, so the result of an image
// does not depend on the batch it is in.
#include <algorithm>

#include <hip/hip_ext.h>

#include "ecc_device.h"

namespace ecc {

namespace {

using namespace dev;

// Min/max keys of AUTO-range images: one block per piece, folded into the
// image's keys with atomics (the host uploads lo = ~0, hi = 0 first).
template <int DT>
__device__ void minmax_piece(const BatchImage& I, const BatchPiece& pc, uint32_t* mm)
{
    using T = typename ValT<DT>::T;
    const T* __restrict__ img = (const T*)I.data;
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (int64_t i = pc.begin + threadIdx.x; i < pc.end; i += kThreads) mm_take<DT>(img[i], lo, hi);
    block_minmax(lo, hi);
    if (threadIdx.x == 0) {
        atomicMin(&mm[2 * pc.image], lo);
        atomicMax(&mm[2 * pc.image + 1], hi);
    }
}

// Initial min/max keys of every image: lo = ~0, hi = 0.
__global__ __launch_bounds__(kThreads) void k_mm_init(uint32_t* mm, int count)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < count) {
        mm[2 * i] = 0xFFFFFFFFu;
        mm[2 * i + 1] = 0u;
    }
}

__global__ __launch_bounds__(kThreads) void k_minmax_batch(const BatchImage* images, const BatchPiece* pieces,
                                                           uint32_t* mm)
{
    const BatchPiece pc = pieces[blockIdx.x];
    const BatchImage& I = images[pc.image];
    switch (I.dtype) {
    case DT_U8: minmax_piece<DT_U8>(I, pc, mm); break;
    case DT_U16: minmax_piece<DT_U16>(I, pc, mm); break;
    default: minmax_piece<DT_F32>(I, pc, mm); break;
    }
}

// PAIRS: the launch holds pair volumes (their bricks load two hyperplanes).
template <int DT, int CONS, bool WIN, bool PAIRS>
__global__ __launch_bounds__(kMaxWaves * 64) __attribute__((amdgpu_waves_per_eu(ECC_WAVES_PER_EU_BATCH)))
void k_ecc_batch(BatchLaunch B)
{
    extern __shared__ __align__(16) int32_t hist[];
    const HistRef H = hist_ref(hist, B.bin_lo, B.width, B.hist_stride, B.sentinel, B.hist_copies);
    const int W = (int)(blockDim.x >> 6), wave = wave_id();
    const int s_end = B.wg_seg[blockIdx.x + 1];
    for (int si = B.wg_seg[blockIdx.x]; si < s_end; ++si) {
        // The tables are read with vector loads (the kernel also writes global
        // memory, so the scalar cache is not used for them): every value the
        // brick loops depend on is read back from the first lane, so that sizes,
        // offsets and pointers stay in scalar registers there.
        const BatchSeg S = B.segs[si];
        const int vol = (int)uniform_u32((uint32_t)S.image);
        const BatchImage& I = B.images[vol];
        const BinParams P = I.auto_range
                                ? params_from_keys(B.mm[2 * I.owner], B.mm[2 * I.owner + 1], DT, B.nbins)
                                : I.params;
        EccLaunch L;   // the fields the brick bodies read
        L.data = uniform_ptr(I.data);
        L.data2 = PAIRS ? uniform_ptr(I.data2) : nullptr;
        L.g = Geom{uniform_i64(I.g.n0), uniform_i64(I.g.n1), uniform_i64(I.g.n2)};
        L.depth = uniform_i64(I.depth);
        L.z_own = L.g.n0;
        L.z_base = 0;
        L.pass_stride = 0;
        L.n0_global = L.g.n0;
        const int ndim = (int)uniform_u32((uint32_t)I.ndim);
        zero_hist(H, B.width);
        // the workgroup's waves form W / wpb teams of wpb waves; team t takes
        // bricks b0 + t, b0 + t + teams, ... (waves beyond the last team idle)
        const int wpb = uniform_u32((uint32_t)I.wpb);
        const int teams = W / wpb, team = wave / wpb, xw = wave - team * wpb;
        const int64_t chunk = kLaneCols * (int64_t)wpb;
        const uint32_t nxc = uniform_u32((uint32_t)I.nxc);
        const int64_t b0 = uniform_i64(S.b0), b1 = uniform_i64(S.b1);
        if (team < teams && ndim == 3) {
            // per plane block: ordinary bricks (x-chunk fastest), packed tail
            // bricks, the tails of the strips not packed (layout_3d, as k_ecc_3d)
            const Layout3 Y = layout_3d(L.g, CONS, wpb);
            const int64_t per_z = Y.per_z, main = Y.nxc * Y.nyb;
            for (int64_t b = b0 + team; b < b1; b += teams) {
                // brick coordinates from the 64-bit index; each fits 32 bits
                const int64_t zb = b / per_z, r = b - zb * per_z;
                Brick3 K;
                if (r < main) {
                    K = chunk_brick_3d<DT, CONS, WIN>(L, H, chunk, (uint32_t)(r % nxc), (uint32_t)(r / nxc),
                                                      (uint32_t)zb, xw);
                } else if (r - main < Y.npk) {
                    K = tail_brick_3d<DT, CONS, WIN>(L, H, Y, wpb, (uint32_t)(r - main), (uint32_t)zb, xw);
                } else {
                    const int64_t e = r - main - Y.npk;   // the strips before sa, then those from sb on
                    K = chunk_brick_3d<DT, CONS, WIN>(L, H, chunk, nxc, (uint32_t)(e < Y.sa ? e : Y.sb + (e - Y.sa)),
                                                      (uint32_t)zb, xw);
                }
                if (PAIRS && L.data2) run_brick3<DT, CONS, WIN, true>(L, P, H, K);
                else run_brick3<DT, CONS, WIN>(L, P, H, K);
            }
        } else if (team < teams) {
            for (int64_t b = b0 + team; b < b1; b += teams) {
                const int64_t row = b / nxc;
                run_brick_2d<DT, CONS, WIN>(L, P, H, chunk, (uint32_t)(b - row * nxc), (uint32_t)row, xw);
            }
        }
        flush_hist(H, B.partials + (size_t)uniform_u32((uint32_t)S.slot) * (size_t)B.width, B.width, false,
                   (int)uniform_u32((uint32_t)I.sign));
    }
}

// Block (image i, bins y * 256 ..): out[bin_lo + j] = the sum of the image's
// partial rows.  16 rows are loaded before they are added (rows past the last
// re-read it and are dropped), so a wide image spread over many workgroups costs
// a few memory latencies, not one per row.
__global__ __launch_bounds__(kThreads) void k_merge_batch(BatchLaunch B)
{
    constexpr int K = 16;
    const int i = blockIdx.x;
    const int j = blockIdx.y * kThreads + threadIdx.x;
    if (j >= B.width) return;
    const int r0 = B.slot_off[i], r1 = B.slot_off[i + 1];
    int64_t s = 0;
    for (int base = r0; base < r1; base += K) {
        int32_t x[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
            x[k] = B.partials[(size_t)B.slots[min(base + k, r1 - 1)] * (size_t)B.width + j];
#pragma unroll
        for (int k = 0; k < K; ++k) s += base + k < r1 ? x[k] : 0;
    }
    B.images[i].out[B.bin_lo + j] = s;
}

// One block per image: out[0 .. nbins) prefix-summed in place.
__global__ __launch_bounds__(kThreads) void k_scan_batch(BatchLaunch B)
{
    block_scan_inplace(B.images[blockIdx.x].out, B.nbins);
}

template <class K>
hipError_t launch_batch_k(K kernel, const BatchLaunch& B, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    if (t0 || t1)
        hipExtLaunchKernelGGL(kernel, dim3(B.grid), dim3(B.waves * 64), B.lds_bytes, s, t0, t1, 0, B);
    else
        hipLaunchKernelGGL(kernel, dim3(B.grid), dim3(B.waves * 64), B.lds_bytes, s, B);
    return hipGetLastError();
}

template <int DT, int CONS, bool PAIRS>
hipError_t launch_batch_p(const BatchLaunch& B, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    return B.windowed ? launch_batch_k(k_ecc_batch<DT, CONS, true, PAIRS>, B, s, t0, t1)
                      : launch_batch_k(k_ecc_batch<DT, CONS, false, PAIRS>, B, s, t0, t1);
}

template <int DT, int CONS>
hipError_t launch_batch_w(const BatchLaunch& B, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    return B.pairs ? launch_batch_p<DT, CONS, true>(B, s, t0, t1) : launch_batch_p<DT, CONS, false>(B, s, t0, t1);
}

template <int CONS>
hipError_t launch_batch_d(const BatchLaunch& B, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    switch (B.dtype) {
    case DT_U8: return launch_batch_w<DT_U8, CONS>(B, s, t0, t1);
    case DT_U16: return launch_batch_w<DT_U16, CONS>(B, s, t0, t1);
    default: return launch_batch_w<DT_F32, CONS>(B, s, t0, t1);
    }
}

}  // namespace

int64_t batch_bricks(BatchImage& im, int construction, int waves, int depth3, int depth2)
{
    const int64_t xpos = axis_positions(im.g.n2, construction);
    const int64_t cols = (xpos + kLaneCols - 1) / kLaneCols;
    // waves per brick: the fraction of the workgroup's lanes that own a column,
    // (wave columns needed / wave columns covered) x (waves in teams / waves),
    // is largest (ties: the wider brick).  A 256-wide row takes 1 wave per
    // brick (9 teams, 81% of the lanes busy) rather than 5 (one team, 45%).
    int best = 1;
    double best_eff = -1.0;
    for (int w = (int)std::min<int64_t>(cols, waves); w >= 1; --w) {
        const int64_t nx = (cols + w - 1) / w;
        const double eff = (double)cols / (double)(nx * w) * (double)((waves / w) * w) / (double)waves;
        if (eff > best_eff + 1e-9) {
            best_eff = eff;
            best = w;
        }
    }
    im.wpb = best;
    const int64_t chunk = kLaneCols * (int64_t)im.wpb;
    im.nxc = (int32_t)((xpos + chunk - 1) / chunk);
    if (im.ndim == 3) {
        // the bricks of k_ecc_3d's layout for a workgroup of wpb waves (a narrow
        // row tail packed several strips per team, layout_3d)
        const Layout3 Y = layout_3d(im.g, construction, im.wpb);
        im.depth = depth3;
        im.nxc = (int32_t)Y.nxc;
        im.nyb = (int32_t)Y.nyb;
        return Y.per_z * ((im.g.n0 + im.depth - 1) / im.depth);
    }
    // whole chunks of rows per brick (the 2D brick body steps a chunk at a time)
    im.depth = ((int64_t)(depth2 < 1 ? 1 : depth2) + kChunk2 - 1) / kChunk2 * kChunk2;
    im.nyb = (int32_t)((im.g.n1 + im.depth - 1) / im.depth);
    return (int64_t)im.nxc * im.nyb;
}

int64_t batch_brick_voxels(const BatchImage& im)
{
    const int64_t cols = kLaneCols * (int64_t)im.wpb;
    return im.ndim == 3 ? cols * kRows3 * im.depth : cols * im.depth;
}

hipError_t launch_minmax_batch(const BatchImage* images, const BatchPiece* pieces, int npieces, uint32_t* mm,
                               hipStream_t s)
{
    if (npieces <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_minmax_batch, dim3(npieces), dim3(kThreads), 0, s, images, pieces, mm);
    return hipGetLastError();
}

hipError_t launch_mm_init(uint32_t* mm, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mm_init, dim3((count + kThreads - 1) / kThreads), dim3(kThreads), 0, s, mm, count);
    return hipGetLastError();
}

hipError_t launch_ecc_batch(const BatchLaunch& B, int construction, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    return construction == CONS_TOP ? launch_batch_d<CONS_TOP>(B, s, t0, t1) : launch_batch_d<CONS_VERTEX>(B, s, t0, t1);
}

hipError_t launch_merge_batch(const BatchLaunch& B, bool scan, hipStream_t s)
{
    if (B.count <= 0) return hipSuccess;
    const unsigned by = (unsigned)((B.width + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_merge_batch, dim3((unsigned)B.count, by), dim3(kThreads), 0, s, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !scan) return e;
    hipLaunchKernelGGL(k_scan_batch, dim3((unsigned)B.count), dim3(kThreads), 0, s, B);
    return hipGetLastError();
}

}  // namespace ecc
