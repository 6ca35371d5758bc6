// ecc_reduce.hip -- the small kernels around the histogram kernels of one
// image: the AUTO-range min/max pass and its binning parameters, and the merge of
// workgroup histograms with the prefix scan (Sec. 2.3: the ECC is the prefix sum
// of the VCEC).
#include "ecc_device.h"

namespace ecc {

namespace {

using namespace dev;

// ------------------------------------------------------------------- minmax

// Grid-stride min/max over the image with 16-byte loads; the unaligned head and
// the tail are read element by element.  Writes one (lo, hi) pair per block.
template <int DT>
__global__ __launch_bounds__(kThreads) void k_minmax(const void* data, int64_t nvox, uint32_t* mm)
{
    using T = typename ValT<DT>::T;
    constexpr int PER = 16 / (int)sizeof(T);
    const T* __restrict__ img = (const T*)data;
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    const int64_t tid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * kThreads;
    const uintptr_t addr = (uintptr_t)data;
    int64_t head = (int64_t)(((16 - (addr & 15)) & 15) / sizeof(T));
    if (head > nvox) head = nvox;
    if (tid < head) mm_take<DT>(img[tid], lo, hi);
    const int64_t nvec = (nvox - head) / PER;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4* __restrict__ vec = (const u32x4*)(img + head);
    for (int64_t i = tid; i < nvec; i += nthreads) {
        const u32x4 w = __builtin_nontemporal_load(vec + i);
        const T* e = (const T*)&w;
#pragma unroll
        for (int k = 0; k < PER; ++k) mm_take<DT>(e[k], lo, hi);
    }
    for (int64_t i = head + nvec * PER + tid; i < nvox; i += nthreads) mm_take<DT>(img[i], lo, hi);
    block_minmax(lo, hi);
    if (threadIdx.x == 0) {
        mm[2 * blockIdx.x] = lo;
        mm[2 * blockIdx.x + 1] = hi;
    }
}

// Elementwise max (take_max) or min of two hyperplanes of an image, for the
// reduction of an image of five or more dimensions one axis at a time (a cell
// that spans two adjacent hyperplanes takes the max of its vertices' values in
// the vertex filtration and the min of its voxels' in the top one, Sec. 2.1).
// The combined value must bin to the max (min) of the two bins, and binning is
// monotone with NaN in the last bin: NaN is taken as the largest float here.
template <int DT, bool MAX>
__global__ __launch_bounds__(kThreads) void k_combine(const void* a, const void* b, void* out, int64_t n)
{
    using T = typename ValT<DT>::T;
    const T* __restrict__ x = (const T*)a;
    const T* __restrict__ y = (const T*)b;
    T* __restrict__ z = (T*)out;
    const int64_t nthreads = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += nthreads) {
        const T u = x[i], v = y[i];
        if constexpr (DT == DT_F32) {
            if constexpr (MAX) z[i] = (u != u || u > v) ? u : v;    // v NaN: u > v fails, v wins
            else z[i] = (v != v || u < v) ? u : v;                  // u NaN: u < v fails, v wins
        } else {
            z[i] = MAX ? (u > v ? u : v) : (u < v ? u : v);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_params(const uint32_t* mm, int blocks, int dtype,
                                                     int32_t nbins, BinParams* out)
{
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (int i = threadIdx.x; i < blocks; i += kThreads) {
        lo = min(lo, mm[2 * i]);
        hi = max(hi, mm[2 * i + 1]);
    }
    block_minmax(lo, hi);
    if (threadIdx.x == 0) *out = params_from_keys(lo, hi, dtype, nbins);
}

// --------------------------------------------------------- merge and scan

// Merge of the workgroup histograms, in two launches with no fence between
// blocks of one launch (a device-scope release per block costs an L2 write-back
// on every XCD that takes part):
//   k_merge_groups: block (bx, g) sums rows [r0, r1) of group g for bins
//                   bx*256 .. +255 into level2[g] (int64), and with `btot` also
//                   the total of those 256 sums into btot[g][bx];
//   k_merge_final:  block bx adds the groups of its bins (negated with sign
//                   -1: the 4D path subtracts some 3D passes).  When the window is
//                   the whole histogram and `scan` is set, every block scans its
//                   own bins, offset by the totals of the blocks before it (from
//                   btot), so the ECC needs no last-block pass.  Otherwise the
//                   block writes the VCEC of its bins, and with `scan` the last
//                   block to finish prefix-sums out[0..nbins) and re-arms its
//                   counter (histograms wider than one LDS window).

// Sum of one value per thread across the wave, in every lane.
__device__ __forceinline__ int64_t wave_sum(int64_t v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Inclusive scan of `v` across the block plus the block-wide sum of `add`, in
// one LDS exchange of the wave totals (one barrier for the exchange, one before
// the buffer is used again).
__device__ __forceinline__ int64_t block_scan_plus(int64_t v, int64_t add)
{
    constexpr int W = kThreads / 64;
    __shared__ int64_t wscan[W], wadd[W];
    const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
    const int64_t inc = wave_scan(v);
    const int64_t a = wave_sum(add);
    if (lane == 63) wscan[w] = inc;
    if (lane == 0) wadd[w] = a;
    __syncthreads();
    int64_t before = 0, offset = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        before += k < w ? wscan[k] : 0;
        offset += wadd[k];
    }
    __syncthreads();
    return inc + before + offset;
}

// Sum of one value per thread across the block, in every thread.
__device__ __forceinline__ int64_t block_sum(int64_t v)
{
    constexpr int W = kThreads / 64;
    __shared__ int64_t ws[W];
    const int64_t a = wave_sum(v);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = a;
    __syncthreads();
    int64_t t = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) t += ws[k];
    __syncthreads();
    return t;
}

static_assert(kMaxLdsBins / kThreads <= kThreads, "k_merge_final gives each earlier block one thread");

__global__ __launch_bounds__(kThreads) void k_merge_groups(const int32_t* __restrict__ partials, int rows,
                                                           int32_t width, int64_t* __restrict__ level2,
                                                           int64_t* __restrict__ btot)
{
    const int j = blockIdx.x * kThreads + threadIdx.x;
    const int G = gridDim.y, g = blockIdx.y;
    const int r0 = (int)((int64_t)rows * g / G), r1 = (int)((int64_t)rows * (g + 1) / G);
    int64_t s = 0;
    if (j < width) {
#pragma unroll 8
        for (int r = r0; r < r1; ++r) s += partials[(size_t)r * (size_t)width + j];
        level2[(size_t)g * width + j] = s;
    }
    if (btot) {
        const int64_t total = block_sum(s);
        if (threadIdx.x == 0) btot[(size_t)g * gridDim.x + blockIdx.x] = total;
    }
}

__global__ __launch_bounds__(kThreads) void k_merge_final(const int64_t* __restrict__ level2,
                                                          const int64_t* __restrict__ btot, int groups,
                                                          int32_t width, int32_t bin_lo, int64_t* out,
                                                          int32_t nbins, uint32_t* counter, int accumulate,
                                                          int scan, int sign)
{
    const int j = blockIdx.x * kThreads + threadIdx.x;
    // Every row of level2 is loaded, those past `groups` too (they lie in the
    // buffer, and their values are dropped): a load under a condition becomes a
    // branch with a wait for each, and the latencies would add up.
    int64_t t = 0;
    if (j < width) {
        int64_t x[kMergeGroups];
#pragma unroll
        for (int g = 0; g < kMergeGroups; ++g) x[g] = level2[(size_t)g * width + j];
#pragma unroll
        for (int g = 0; g < kMergeGroups; ++g) t += g < groups ? x[g] : 0;
    }
    if (btot) {
        // offset = sum of the bins of the blocks before this one: thread b < this
        // block's index adds block b's group totals (blocks <= kThreads, since a
        // window holds at most kMaxLdsBins bins)
        int64_t part = 0;
        if ((int)threadIdx.x < (int)blockIdx.x) {
            int64_t x[kMergeGroups];
#pragma unroll
            for (int g = 0; g < kMergeGroups; ++g) x[g] = btot[(size_t)g * gridDim.x + threadIdx.x];
#pragma unroll
            for (int g = 0; g < kMergeGroups; ++g) part += g < groups ? x[g] : 0;
        }
        const int64_t v = block_scan_plus(t, part);
        if (j < width) out[bin_lo + j] = v;
        return;
    }
    if (j < width) out[bin_lo + j] = (accumulate ? out[bin_lo + j] : 0) + (sign < 0 ? -t : t);
    if (!scan) return;
    if (!last_to_arrive(counter, gridDim.x)) return;
    block_scan_inplace(out, nbins);
    if (threadIdx.x == 0) atomicExch(counter, 0u);
}

// Folds the per-block min/max keys of one slab into a running pair acc[0..1]
// (first: start the pair).
__global__ __launch_bounds__(kThreads) void k_mm_fold(const uint32_t* mm, int blocks, uint32_t* acc, int first)
{
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (int i = threadIdx.x; i < blocks; i += kThreads) {
        lo = min(lo, mm[2 * i]);
        hi = max(hi, mm[2 * i + 1]);
    }
    block_minmax(lo, hi);
    if (threadIdx.x == 0) {
        acc[0] = first ? lo : min(acc[0], lo);
        acc[1] = first ? hi : max(acc[1], hi);
    }
}

}  // namespace

hipError_t launch_mm_fold(const uint32_t* mm, int blocks, uint32_t* acc, bool first, hipStream_t s)
{
    hipLaunchKernelGGL(k_mm_fold, dim3(1), dim3(kThreads), 0, s, mm, blocks, acc, first ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_merge(const int32_t* partials, int rows, int32_t width, int32_t bin_lo, int64_t* level2,
                        int64_t* out, int32_t nbins, uint32_t* counters, bool accumulate, bool scan, int sign,
                        hipStream_t s)
{
    const unsigned bx = (unsigned)((width + kThreads - 1) / kThreads);
    const int groups = rows < kMergeGroups ? rows : kMergeGroups;
    // one window holding every bin, written afresh: blocks scan their own bins
    // (see k_merge_final)
    int64_t* btot = (scan && !accumulate && sign > 0 && bin_lo == 0 && width == nbins)
                        ? level2 + (size_t)kMergeGroups * width : nullptr;
    hipLaunchKernelGGL(k_merge_groups, dim3(bx, (unsigned)groups), dim3(kThreads), 0, s, partials, rows, width,
                       level2, btot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_final, dim3(bx), dim3(kThreads), 0, s, level2, btot, groups, width, bin_lo, out,
                       nbins, counters, accumulate ? 1 : 0, scan ? 1 : 0, sign < 0 ? -1 : 1);
    return hipGetLastError();
}

hipError_t launch_minmax(const void* data, int dtype, int64_t nvox, uint32_t* mm, int blocks,
                         hipStream_t s)
{
    switch (dtype) {
    case DT_U8: hipLaunchKernelGGL(k_minmax<DT_U8>, dim3(blocks), dim3(kThreads), 0, s, data, nvox, mm); break;
    case DT_U16: hipLaunchKernelGGL(k_minmax<DT_U16>, dim3(blocks), dim3(kThreads), 0, s, data, nvox, mm); break;
    default: hipLaunchKernelGGL(k_minmax<DT_F32>, dim3(blocks), dim3(kThreads), 0, s, data, nvox, mm); break;
    }
    return hipGetLastError();
}

hipError_t launch_combine(const void* a, const void* b, void* out, int64_t n, int dtype, bool take_max,
                          hipStream_t s)
{
    const unsigned blocks = (unsigned)std::min<int64_t>(4096, (n + kThreads - 1) / kThreads);
    const dim3 g(blocks > 0 ? blocks : 1), t(kThreads);
    switch (dtype * 2 + (take_max ? 1 : 0)) {
    case DT_U8 * 2: hipLaunchKernelGGL((k_combine<DT_U8, false>), g, t, 0, s, a, b, out, n); break;
    case DT_U8 * 2 + 1: hipLaunchKernelGGL((k_combine<DT_U8, true>), g, t, 0, s, a, b, out, n); break;
    case DT_U16 * 2: hipLaunchKernelGGL((k_combine<DT_U16, false>), g, t, 0, s, a, b, out, n); break;
    case DT_U16 * 2 + 1: hipLaunchKernelGGL((k_combine<DT_U16, true>), g, t, 0, s, a, b, out, n); break;
    case DT_F32 * 2: hipLaunchKernelGGL((k_combine<DT_F32, false>), g, t, 0, s, a, b, out, n); break;
    default: hipLaunchKernelGGL((k_combine<DT_F32, true>), g, t, 0, s, a, b, out, n); break;
    }
    return hipGetLastError();
}

hipError_t launch_params_from_minmax(const uint32_t* mm, int blocks, int dtype, int32_t nbins,
                                     BinParams* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_params, dim3(1), dim3(kThreads), 0, s, mm, blocks, dtype, nbins, out);
    return hipGetLastError();
}


}  // namespace ecc
