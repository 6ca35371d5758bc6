// ecc_device.h -- device-side building blocks shared by the single-image and
// the batched kernels (binning, wave helpers, type functions, brick bodies).
//
// What is computed (Wang, Wagner, Chen, SoCG 2022):
//   VCEC[j] = sum over cells of the cubical complex whose value has bin j of
//             (-1)^dim  (Sec. 2.3), and the ECC is its prefix sum (Eq. (1)).
//
// How the cells are counted here.  A cell of a d-dimensional cubical complex is
// a product of one choice per axis: a single position or a pair of adjacent
// positions.  Vertex filtration (voxels are vertices, a cell takes the largest
// value of its voxels): a single is one voxel index k (dimension 0 along the
// axis), a pair the edge {k, k+1} (dimension 1).  Top filtration (the paper's,
// Sec. 2.1: voxels are top cells, a face takes the smallest value of the voxels
// that contain it): a single is the voxel interval k (dimension 1), a pair the
// lattice point between voxels k-1 and k with voxel set {k-1, k} (dimension 0),
// the points before the first and after the last voxel included (their outside
// voxel is ignored).  Fix the choices on all axes but the first ("the marching
// axis") and take, at every position p of that axis, the max (vertex) or min
// (top) over the chosen voxels: a "type function" C(p).  The cells of that type
// are the 1D complex of C along the marching axis with an overall sign
// (-1)^(number of pairs) (vertex) or (-1)^(number of singles) (top), and a 1D
// complex is counted by crediting each interval {p, p+1} to the position that
// attains its value: position p adds +-(1 - [p wins its left interval] -
// [p wins its right interval]) at C(p) (vertex; the top filtration's points are
// credited the same way, with -1 for the voxel itself).  Both reduce to
//     count(p) = d(p) - d(p-1),   d(p) = -[C(p) > C(p+1)] = sign bit of C(p+1) - C(p),
// with C beyond the image = the sentinel and d(-1) = -1 (vertex ties go to the
// later position, top ties to the earlier one; the VCEC does not depend on
// either, since an interval's value is that of whichever position attains it).
// 3D: the marching axis is z and the types are the four choices in (y, x),
// two per axis; 2D: the marching axis is y and the types are the two in x.
// Every count is added to a workgroup histogram in LDS at the key of C(p).
// Nothing is compared position by position and no per-voxel cell logic remains:
// a type function is one max/min (the right neighbour through a DPP lane move),
// a count is two subtractions and a shift.
//
// Mapping to the hardware.  One wave handles 64 consecutive x positions; lanes
// 0..62 own theirs, lane 63 only supplies lane 62's right neighbour.  Rows and
// planes stay in registers while a wave walks its brick along the marching axis.
// Workgroup histograms are merged and prefix-scanned by a second kernel.
#pragma once

#include "ecc_internal.h"

namespace ecc {
namespace dev {


constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

// Sentinel key: above every key, below 2^31, and such that OR-ing it into any
// key gives the sentinel.  With windows it is the constant below (keys are
// bin << 2 with bins below 65535); with one window it is the launch's
// (lds_sentinel: bins below nbins), which is also the byte address of a spare
// LDS word that absorbs the counts of cells that do not exist, so they need no
// masking.
template <bool WIN>
__device__ __forceinline__ uint32_t sentinel_key(uint32_t one_window)
{
    return WIN ? 0x3FFFCu : one_window;
}

// ------------------------------------------------------------------ binning
//
// The kernels compare and store KEYS = 4 * bin: the order is that of the bins,
// and a key is directly the byte offset of its counter in the LDS histogram.

template <int DT> struct ValT;
template <> struct ValT<DT_U8> { using T = uint8_t; };
template <> struct ValT<DT_U16> { using T = uint16_t; };
template <> struct ValT<DT_F32> { using T = float; };

// Key (bin << kKeyShift, its LDS byte address) of one value, OR-ed with `oob`:
// 0, or the sentinel for lanes outside the image, which makes the key the
// sentinel.
// IDENT: integer data with nbins == hi - lo + 1, where the bin is the level.
template <int DT, bool IDENT>
__device__ __forceinline__ uint32_t key_of(typename ValT<DT>::T v, const BinParams& p, uint32_t oob)
{
    if constexpr (DT == DT_F32) {
        // clamp(floor(((double)x - lo) * scale), 0, nbins-1) without branches:
        // fmin maps NaN to nbins-1, and the saturating conversion clamps below.  A flat range
        // (hi == lo) carries scale = +inf and base = the next double above lo, so
        // x <= lo gives -inf -> 0, x > lo gives +inf or 0*inf = NaN -> nbins-1.
        const float x = v;
        double t = __dmul_rn(__dsub_rn((double)x, p.base), p.scale);
        t = __builtin_fmin(t, (double)(p.nbins - 1));
        // the conversion saturates: negative values and -inf give 0
        uint32_t b;
        asm("v_cvt_u32_f64 %0, %1" : "=v"(b) : "v"(t));
        return (b << kKeyShift) | oob;
    } else {
        uint32_t a = (uint32_t)v;
        a = min(max(a, p.ilo), p.ihi) - p.ilo;
        if constexpr (IDENT) return (a << kKeyShift) | oob;
        // floor(a * nbins / D): a * nbins < 2^32 is exact in double, and rcp is
        // 1/D rounded up, so the product never falls below an integer it should
        // reach and stays below the next one (a < D <= 65536).
        const uint32_t n = __umul24(a, (uint32_t)p.nbins);
        const uint32_t b = (uint32_t)__dmul_rn((double)n, p.rcp);
        return (b << kKeyShift) | oob;
    }
}

// Binning parameters from the min/max keys of an image (AUTO range).  Keys are
// order-preserving: integers as themselves, finite floats through the sign-flip
// map; lo_key > hi_key means no (finite) value was seen, which gives [0, 0].
__device__ __forceinline__ double key_to_double(uint32_t k, int dtype)
{
    if (dtype != DT_F32) return (double)k;
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return (double)__uint_as_float(u);
}

__device__ __forceinline__ BinParams params_from_keys(uint32_t lo_key, uint32_t hi_key, int dtype, int32_t nbins)
{
    BinParams p = {};
    p.dtype = dtype;
    p.nbins = nbins;
    const bool empty = lo_key > hi_key;
    const double dlo = empty ? 0.0 : key_to_double(lo_key, dtype);
    const double dhi = empty ? 0.0 : key_to_double(hi_key, dtype);
    p.lo = dlo;
    p.hi = dhi;
    if (dtype == DT_F32) {
        p.flat = (dhi == dlo) ? 1 : 0;
        p.scale = p.flat ? __builtin_inf() : __ddiv_rn((double)nbins, __dsub_rn(dhi, dlo));
        // next double above lo (lo is finite): the subtrahend of a flat range
        const double up = dlo == 0.0 ? __longlong_as_double(1ll)
                                     : __longlong_as_double(__double_as_longlong(dlo) + (dlo > 0.0 ? 1 : -1));
        p.base = p.flat ? up : dlo;
    } else {
        const uint32_t ilo = (uint32_t)dlo, ihi = (uint32_t)dhi;
        const uint32_t D = ihi - ilo + 1u;
        p.ilo = ilo;
        p.ihi = ihi;
        p.ident = ((uint32_t)nbins == D) ? 1 : 0;
        // 1/D rounded up: one step above the correctly rounded quotient
        p.rcp = __longlong_as_double(__double_as_longlong(__ddiv_rn(1.0, (double)D)) + 1);
    }
    return p;
}

// Folds one value into running min/max keys (non-finite floats are skipped).
template <int DT>
__device__ __forceinline__ void mm_take(typename ValT<DT>::T v, uint32_t& lo, uint32_t& hi)
{
    if constexpr (DT == DT_F32) {
        const uint32_t u = __float_as_uint(v);
        const uint32_t k = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
        const bool fin = (u & 0x7F800000u) != 0x7F800000u;
        lo = fin ? min(lo, k) : lo;
        hi = fin ? max(hi, k) : hi;
    } else {
        const uint32_t k = (uint32_t)v;
        lo = min(lo, k);
        hi = max(hi, k);
    }
}

// Block-wide min/max of (lo, hi); the result is valid in thread 0.
__device__ __forceinline__ void block_minmax(uint32_t& lo, uint32_t& hi)
{
    __shared__ uint32_t slo[kThreads], shi[kThreads];
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            slo[threadIdx.x] = min(slo[threadIdx.x], slo[threadIdx.x + s]);
            shi[threadIdx.x] = max(shi[threadIdx.x], shi[threadIdx.x + s]);
        }
        __syncthreads();
    }
    lo = slo[0];
    hi = shi[0];
}

// Inclusive prefix sum of v[0..n) by one block of kThreads threads.  The values
// pass through LDS in chunks of kScanChunk: coalesced loads, a sequential scan
// of kScanPer values per thread, a scan of the thread totals, coalesced stores.
constexpr int kScanPer = 16;
constexpr int kScanChunk = kThreads * kScanPer;

__device__ __forceinline__ void block_scan_inplace(int64_t* v, int32_t n)
{
    __shared__ int64_t buf[kScanChunk];
    __shared__ int64_t tot[kThreads];
    const int t = threadIdx.x;
    int64_t carry = 0;
    for (int32_t base = 0; base < n; base += kScanChunk) {
        const int m = min(kScanChunk, n - base);
        // every load is issued before any is used (indices past the chunk
        // re-read its last value, which is dropped)
        int64_t x[kScanPer];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) x[k] = v[base + min(k * kThreads + t, m - 1)];
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int i = k * kThreads + t;
            buf[i] = i < m ? x[k] : 0;
        }
        __syncthreads();
        int64_t run = 0;
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            run += buf[t * kScanPer + k];
            buf[t * kScanPer + k] = run;
        }
        tot[t] = run;
        __syncthreads();
        for (int off = 1; off < kThreads; off <<= 1) {
            const int64_t add = t >= off ? tot[t - off] : 0;
            __syncthreads();
            tot[t] += add;
            __syncthreads();
        }
        const int64_t before = carry + (t > 0 ? tot[t - 1] : 0);
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) buf[t * kScanPer + k] += before;
        carry += tot[kThreads - 1];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kScanPer; ++k) {
            const int i = k * kThreads + t;
            if (i < m) v[base + i] = buf[i];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// lane i <- lane i+1 (lane 63 gets 0; it owns no position)
__device__ __forceinline__ uint32_t from_right(uint32_t v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x130 /* wave_shl:1 */, 0xF, 0xF, true);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// ---------------------------------------------------------- type functions

// The pair operation of the filtration: a vertex-filtration cell takes the
// largest key of its voxels, a top-filtration face the smallest of the voxels
// that contain it (voxels outside the image carry the sentinel, so a vertex
// cell that leaves the image and a top face with no voxel inside get it too).
template <int CONS>
__device__ __forceinline__ uint32_t op2(uint32_t a, uint32_t b)
{
    return CONS == CONS_VERTEX ? max(a, b) : min(a, b);
}

// op2 of this lane's key and its right neighbour's (lane 63: meaningless, never counted)
template <int CONS>
__device__ __forceinline__ uint32_t op_right(uint32_t a)
{
    return op2<CONS>(a, from_right(a));
}

struct HistRef {
    int32_t* hist;     // LDS: `copies` copies of the window's counters (`stride` words apart)
                       // and spare words (lds_words)
    uint32_t key_lo;   // key of the first bin of the window (windowed launches)
    uint32_t key_span; // keys in the window: also the byte offset of the spare word that
                       // absorbs keys outside the window (windowed launches)
    uint32_t copy;     // byte offset of this lane's copy (odd lanes: the second)
    uint32_t stride;   // words from one copy to the next
    uint32_t sm;       // the sentinel key of a one-window launch
    uint32_t copies;   // copies (a power of two; lane l adds to copy l mod copies)
};

__device__ __forceinline__ HistRef hist_ref(int32_t* hist, int32_t bin_lo, int32_t width, uint32_t stride,
                                            uint32_t sm, uint32_t copies)
{
    return HistRef{hist, (uint32_t)bin_lo << kKeyShift, (uint32_t)width << kKeyShift,
                   (__lane_id() & (copies - 1u)) * stride * 4u, stride, sm, copies};
}

// Adds v to the counter of `key` in this lane's copy.  One window: the key is the
// counter's byte address in the copy (the sentinel's address is a spare word).
// Windows: keys outside the window (the sentinel included; below it the
// subtraction wraps) go to the spare word after the window.
template <bool WIN>
__device__ __forceinline__ void hist_add(const HistRef& H, uint32_t key, int32_t v)
{
    uint32_t a = key;
    if constexpr (WIN) a = min(key - H.key_lo, H.key_span);
    atomicAdd((int32_t*)((char*)H.hist + (a + H.copy)), v);
}

// One step of a type function along the marching axis.  The type's cells at
// position p (value `cur`) and on the interval from p to p+1 (value op2(cur,
// next)) are counted at key `cur` as SIGN * (d - dp): d = -[cur > next] is the
// sign bit of next - cur (every key is below 2^31), dp the previous step's d,
// and the interval from p to p+1 goes to the side that attains op2 (vertex:
// p wins with cur > next, ties to the later position; top: p wins with
// cur <= next, ties to the earlier one; both give d).  Returns the count and
// leaves d in dp.
template <int SIGN>
__device__ __forceinline__ int32_t step_count(uint32_t cur, uint32_t next, int32_t& dp)
{
    const int32_t d = (int32_t)(next - cur) >> 31;
    const int32_t c = SIGN > 0 ? d - dp : dp - d;
    dp = d;
    return c;
}

// True in every thread of the block that is the last of `total` to arrive.
__device__ __forceinline__ bool last_to_arrive(uint32_t* counter, uint32_t total)
{
    __shared__ bool last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == total - 1;
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// Inclusive scan of one value per thread across the wave (lanes shift by 1, 2,
// 4, ... 32).
__device__ __forceinline__ int64_t wave_scan(int64_t v)
{
    const int lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int64_t u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    return v;
}

// Merge of a small single-window launch inside the histogram kernel: the last
// workgroup to finish (all partial rows written and fenced) sums the rows into
// int64 counts in its LDS (the histogram's space, free after the flush), scans
// them and writes the ECC to out[0..width), then re-arms the counter.  It saves
// the two merge launches where the rows are few enough for one workgroup.
__device__ __forceinline__ void fused_merge_scan(int32_t* hist, const int32_t* partials, int width, int64_t* out,
                                                 uint32_t* counter)
{
    const uint32_t rows = gridDim.x * gridDim.y;
    if (!last_to_arrive(counter, rows)) return;
    __shared__ int64_t wave_tot[kMaxWaves];
    const int bd = (int)blockDim.x, t = (int)threadIdx.x;
    uint64_t* acc = reinterpret_cast<uint64_t*>(hist);
    for (int j = t; j < width; j += bd) acc[j] = 0;
    __syncthreads();
    // the rows as one flat array, 16 loads in flight per thread; element i adds
    // to bin i mod width (tracked incrementally)
    constexpr int U = 16;
    const int64_t total = (int64_t)rows * width;
    const int step = bd % width;
    int j = t % width;
    for (int64_t i0 = t; i0 < total; i0 += (int64_t)bd * U) {
        int32_t x[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int64_t i = i0 + (int64_t)k * bd;
            x[k] = i < total ? partials[i] : 0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (x[k] != 0) atomicAdd((unsigned long long*)&acc[j], (unsigned long long)(int64_t)x[k]);
            j += step;
            if (j >= width) j -= width;
        }
    }
    __syncthreads();
    // each thread scans a contiguous run of bins, then adds the runs before it
    const int per = (width + bd - 1) / bd;
    const int j0 = min(t * per, width), j1 = min(j0 + per, width);
    int64_t run = 0;
    for (int b = j0; b < j1; ++b) {
        run += (int64_t)acc[b];
        acc[b] = (uint64_t)run;
    }
    const int64_t inc = wave_scan(run);
    const int w = t >> 6;
    if ((t & 63) == 63) wave_tot[w] = inc;
    __syncthreads();
    int64_t before = inc - run;
    for (int k = 0; k < w; ++k) before += wave_tot[k];
    for (int b = j0; b < j1; ++b) out[b] = (int64_t)acc[b] + before;
    if (t == 0) atomicExch(counter, 0u);
}

// ------------------------------------------------------------ main kernels

__device__ __forceinline__ void zero_hist(const HistRef& H, int width)
{
    for (uint32_t c = 0; c < H.copies; ++c)
        for (int j = threadIdx.x; j < width; j += blockDim.x) H.hist[c * H.stride + j] = 0;
    __syncthreads();
}

// The workgroup's count of bin j of the window: the sum of its copies.
__device__ __forceinline__ int32_t hist_value(const HistRef& H, int j)
{
    int32_t t = H.hist[j];
    for (uint32_t c = 1; c < H.copies; ++c) t += H.hist[c * H.stride + j];
    return t;
}

// Writes the workgroup histogram (negated with sign -1) to dst[0..width), or
// adds it to what dst holds (add).
__device__ __forceinline__ void flush_hist(const HistRef& H, int32_t* dst, int width, bool add = false,
                                           int sign = 1)
{
    __syncthreads();
    if (!add) {
        for (int j = threadIdx.x; j < width; j += blockDim.x) {
            const int32_t t = hist_value(H, j);
            dst[j] = sign < 0 ? -t : t;
        }
        return;
    }
    // adding: a round of the row's old values is loaded before any is written
    // (indices past the row re-read its last word, which is dropped)
    constexpr int R = 8;
    const int step = (int)blockDim.x;
    for (int j0 = (int)threadIdx.x; j0 < width; j0 += R * step) {
        int32_t old[R];
#pragma unroll
        for (int k = 0; k < R; ++k) old[k] = dst[min(j0 + k * step, width - 1)];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int j = j0 + k * step;
            if (j < width) {
                const int32_t t = hist_value(H, j);
                dst[j] = old[k] + (sign < 0 ? -t : t);
            }
        }
    }
}

// Values the whole wave shares, read back from the first lane so that the
// compiler treats them as uniform: the binning parameters may come from device
// memory, and brick coordinates come out of integer divisions that the compiler
// expands into vector arithmetic.  Without this, branches on them are lowered
// as divergent and the row masks that depend on them leave scalar registers.
__device__ __forceinline__ bool uniform_flag(int32_t f) { return __builtin_amdgcn_readfirstlane(f) != 0; }
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ int64_t uniform_i64(int64_t v)
{
    const uint32_t lo = uniform_u32((uint32_t)v), hi = uniform_u32((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double uniform_f64(double v)
{
    return __longlong_as_double((long long)uniform_i64((int64_t)__double_as_longlong(v)));
}
// The binning parameters that key_of reads, read back from the first lane.
// Loaded through a pointer they arrive in vector registers (the kernels also
// write global memory, so the compiler does not load them through the scalar
// cache); as uniform values they stay in scalar registers, which the binning's
// fp64 operations read directly, and leave the vector registers to the brick
// loop.
// (Float data only: the integer kernels have fewer vector registers in use and
// are short of scalar ones, and take the parameters as they are.)
template <int DT>
__device__ __forceinline__ BinParams load_params(const EccLaunch& L)
{
    if constexpr (DT == DT_F32) {
        BinParams p = L.params_dev ? *L.params_dev : L.params;
        p.nbins = (int32_t)uniform_u32((uint32_t)p.nbins);
        p.base = uniform_f64(p.base);
        p.scale = uniform_f64(p.scale);
        return p;
    } else {
        return L.params_dev ? *L.params_dev : L.params;
    }
}
__device__ __forceinline__ const void* uniform_ptr(const void* p) { return (const void*)uniform_i64((int64_t)p); }

// Raw buffer loads: one 32-bit per-lane byte offset (the column) plus one scalar
// byte offset (the row) against a resource whose base is the brick's first row.
// The base is the same for the whole wave; reading it back from the first lane
// lets the compiler keep the resource in scalar registers (otherwise it may not
// prove uniformity and wraps every load in a loop over distinct resources).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_at(const void* base)
{
    const uint64_t a = (uint64_t)base;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32));
    void* u = (void*)(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(u, (short)0, -1, 0x00020000);
}

template <typename T> __device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ uint8_t buffer_load<uint8_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b8(r, (int)voff, (int)soff, 0);
}
template <> __device__ __forceinline__ uint16_t buffer_load<uint16_t>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
}
template <> __device__ __forceinline__ float buffer_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

// Advances a scalar offset by `step`; the empty asm keeps the compiler from
// precomputing every row's offset into its own register.
__device__ __forceinline__ uint32_t advance(uint32_t off, uint32_t step)
{
    off += step;
    asm volatile("" : "+s"(off));
    return off;
}

// Lanes of a wave: lane l sits at position column x0 + l of its chunk; lanes
// 0..62 own their position, lane 63 only supplies lane 62's right neighbour.
constexpr uint64_t kOwnLanes = 0x7FFFFFFFFFFFFFFFull;

// The planes of one 3D brick.  Row r of the brick (0 <= r <= kRows3) is image
// row ys + r; rows 0 .. kRows3-1 are the brick's, row kRows3 only completes the
// pairs of row kRows3-1.  FULL: every row read lies inside the image.  Otherwise
// the rows outside [0, n1) read the nearest row inside (every load in bounds)
// and take the sentinel key, without branches.  Plane indices are 32-bit.
// Types of a row (one per choice of a single position or a pair in y and in x):
//   T0 = row r, T1 = op2(row r, row r+1), T2 = op2(T0, right), T3 = op2(T1, right)
// with signs +, -, -, + in both filtrations (two type axes).  Planes are the
// marching axis: plane z of the brick counts every type against plane z+1.
// PAIR: the volume is the elementwise max (vertex) or min (top) of L.data and
// L.data2, taken on the keys (the bins' order, so exactly the bin of the max or
// min value): the combined hyperplanes of a 4D image.
template <int DT, int CONS, bool WIN, bool FULL, bool IDENT, bool PAIR>
__device__ __forceinline__ void brick_3d(const EccLaunch& L, const BinParams& P, const HistRef& H, int64_t ys,
                                         uint32_t z0, uint32_t zend, uint32_t xob, uint32_t oob, uint64_t own_x,
                                         int r_lo, int r_hi)
{
    constexpr int NR = kRows3;
    const uint32_t SM = sentinel_key<WIN>(H.sm);
    using T = typename ValT<DT>::T;
    const uint32_t n0 = (uint32_t)L.g.n0;
    const int64_t n1 = L.g.n1, n2 = L.g.n2;
    const uint32_t row_bytes = (uint32_t)(n2 * (int64_t)sizeof(T));
    // the launch's pass (one volume of several of the same shape, pass_stride apart)
    const int64_t pass_off = (int64_t)blockIdx.y * L.pass_stride;
    const char* img = (const char*)L.data + pass_off;
    const char* img2 = PAIR ? (const char*)L.data2 + pass_off : nullptr;
    // first row read: ys, or the first row inside the image
    const int64_t ybase = ys + (FULL ? 0 : r_lo);
    constexpr int NR2 = PAIR ? NR + 1 : 1;

    // the brick's first row in plane 0, and the bytes from plane to plane
    const int64_t first_row = ybase * (int64_t)row_bytes;
    const int64_t plane_bytes = n1 * (int64_t)row_bytes;
    auto load_plane = [&](uint32_t z, T (&raw)[NR + 1], T (&raw2)[NR2]) {
        const int64_t off = first_row + (int64_t)z * plane_bytes;
        const __amdgpu_buffer_rsrc_t rs = rsrc_at(img + off);
        __amdgpu_buffer_rsrc_t rs2 = rs;
        if constexpr (PAIR) rs2 = rsrc_at(img2 + off);
        uint32_t soff = 0;
#pragma unroll
        for (int r = 0; r < NR + 1; ++r) {
            raw[r] = buffer_load<T>(rs, xob, soff);
            if constexpr (PAIR) raw2[r] = buffer_load<T>(rs2, xob, soff);
            // advance while the next row still lies inside the image
            if (FULL || (r >= r_lo && r + 1 < r_hi)) soff = advance(soff, row_bytes);
        }
    };
    auto keys = [&](const T (&raw)[NR + 1], const T (&raw2)[NR2], uint32_t (&K)[NR + 1]) {
#pragma unroll
        for (int r = 0; r < NR + 1; ++r) {
            const uint32_t outside = (FULL || (r >= r_lo && r < r_hi)) ? 0u : SM;
            K[r] = key_of<DT, IDENT>(raw[r], P, oob | outside);
            if constexpr (PAIR) K[r] = op2<CONS>(K[r], key_of<DT, IDENT>(raw2[r], P, oob | outside));
        }
    };

    // lanes that add, per row and kind of y choice (single: T0, T2; pair: T1, T3):
    // a row's cells of a kind exist only inside the image's positions -- vertex:
    // singles at rows [0, n1), pairs at rows [0, n1 - 1); top: singles at rows
    // [0, n1), pairs (lattice points) at rows [-1, n1).  Counts of cells that do
    // not exist would all go to the one spare word and collide there.
    uint64_t own1[NR], own2[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        own1[r] = (FULL || (r >= r_lo && r < r_hi)) ? own_x : 0ull;
        own2[r] = (FULL || (CONS == CONS_TOP ? r < r_hi : r + 1 < r_hi)) ? own_x : 0ull;
    }
    // One step of the marching axis: the types of the next plane (keys K) go to
    // Cn, each type of the current plane (Cc, previous d in Dc) is counted
    // against them, and the new d goes to Dn.  Two register sets alternate from
    // step to step, so no state is copied.
    auto plane_step = [&](const uint32_t (&K)[NR + 1], const uint32_t (&Cc)[NR][4], uint32_t (&Cn)[NR][4],
                          const int32_t (&Dc)[NR][4], int32_t (&Dn)[NR][4]) {
        // every count of the step first, then all adds under one lane mask: a
        // mask switch per row would cut the step into blocks that the compiler
        // cannot schedule across
        int32_t c[NR][4];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const uint32_t b = op2<CONS>(K[r], K[r + 1]);
            Cn[r][0] = K[r];
            Cn[r][1] = b;
            Cn[r][2] = op_right<CONS>(K[r]);
            Cn[r][3] = op_right<CONS>(b);
            int32_t d[4] = {Dc[r][0], Dc[r][1], Dc[r][2], Dc[r][3]};
            c[r][0] = step_count<+1>(Cc[r][0], Cn[r][0], d[0]);
            c[r][1] = step_count<-1>(Cc[r][1], Cn[r][1], d[1]);
            c[r][2] = step_count<-1>(Cc[r][2], Cn[r][2], d[2]);
            c[r][3] = step_count<+1>(Cc[r][3], Cn[r][3], d[3]);
#pragma unroll
            for (int t = 0; t < 4; ++t) Dn[r][t] = d[t];
        }
        if (FULL) {
            if (lane_bit(own_x)) {
#pragma unroll
                for (int r = 0; r < NR; ++r)
#pragma unroll
                    for (int t = 0; t < 4; ++t) hist_add<WIN>(H, Cc[r][t], c[r][t]);
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                if (lane_bit(own1[r])) {
                    hist_add<WIN>(H, Cc[r][0], c[r][0]);
                    hist_add<WIN>(H, Cc[r][2], c[r][2]);
                }
                if (lane_bit(own2[r])) {
                    hist_add<WIN>(H, Cc[r][1], c[r][1]);
                    hist_add<WIN>(H, Cc[r][3], c[r][3]);
                }
            }
        }
    };
    // the keys of plane z (the sentinel past the volume's last plane)
    auto plane_keys = [&](uint32_t z, const T (&raw)[NR + 1], const T (&raw2)[NR2], uint32_t (&K)[NR + 1]) {
        if (z < n0) {
            keys(raw, raw2, K);
        } else {
#pragma unroll
            for (int r = 0; r < NR + 1; ++r) K[r] = SM;
        }
    };
    // the next brick's first plane (zend) starts with d = 0: its count there
    // lacks the -d of this brick's last step, which is added here
    auto end_adds = [&](const uint32_t (&Cc)[NR][4], const int32_t (&Dc)[NR][4]) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (lane_bit(own1[r])) {
                hist_add<WIN>(H, Cc[r][0], -Dc[r][0]);
                hist_add<WIN>(H, Cc[r][2], Dc[r][2]);
            }
            if (lane_bit(own2[r])) {
                hist_add<WIN>(H, Cc[r][1], Dc[r][1]);
                hist_add<WIN>(H, Cc[r][3], -Dc[r][3]);
            }
        }
    };

    uint32_t Ca[NR][4], Cb[NR][4];   // types of the current plane (the sets alternate)
    int32_t Da[NR][4], Db[NR][4];    // d of each type's previous step
    T raw[NR + 1], raw2[NR2];        // loads of the next plane, issued a step ahead
    {
        uint32_t K[NR + 1];
        load_plane(z0, raw, raw2);
        keys(raw, raw2, K);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const uint32_t b = op2<CONS>(K[r], K[r + 1]);
            Ca[r][0] = K[r];
            Ca[r][1] = b;
            Ca[r][2] = op_right<CONS>(K[r]);
            Ca[r][3] = op_right<CONS>(b);
        }
    }
    // the volume's first plane has nothing before it (d = -1: it wins the
    // interval before it); a later brick's first plane gets the rest of its
    // count from the brick before it (end_adds).  A type whose cells do not exist
    // (its value is the sentinel in every plane) starts with d = 0, so all its
    // counts are 0: they may land on any word, the other copy's counters included.
    if (L.z_base + (int64_t)z0 == 0) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int t = 0; t < 4; ++t) Da[r][t] = Ca[r][t] == SM ? 0 : -1;
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int t = 0; t < 4; ++t) Da[r][t] = 0;
    }
    if (z0 + 1 < n0) load_plane(z0 + 1, raw, raw2);
    bool odd = false;   // the last step wrote the b set
    for (uint32_t z = z0; z < zend; z += 2) {
        {
            uint32_t K[NR + 1];
            plane_keys(z + 1, raw, raw2, K);
            if (z + 1 < zend && z + 2 < n0) load_plane(z + 2, raw, raw2);
            plane_step(K, Ca, Cb, Da, Db);
        }
        if (z + 1 < zend) {
            uint32_t K[NR + 1];
            plane_keys(z + 2, raw, raw2, K);
            if (z + 2 < zend && z + 3 < n0) load_plane(z + 3, raw, raw2);
            plane_step(K, Cb, Ca, Db, Da);
        } else {
            odd = true;
        }
    }
    if (L.z_base + (int64_t)zend < L.n0_global) {
        if (odd) end_adds(Cb, Db);
        else end_adds(Ca, Da);
    }
}

// The rows [y0, yend) of one 2D brick for one wave: rows are the marching axis,
// loaded in chunks of kChunk2, the next chunk loading while the current one is
// counted.  Types of a row: T0 = the row, T1 = op2(T0, right), with signs +, -
// (vertex) or -, + (top: a single position is a voxel, of dimension 1 along x).
// yend - y0 is a multiple of kChunk2 unless yend == n1 (the rows past the image
// carry the sentinel and count into the spare word).  Row indices are 32-bit.
template <int DT, int CONS, bool WIN, bool IDENT>
__device__ __forceinline__ void brick_2d(const void* data, uint32_t n1, int64_t n2, const BinParams& P,
                                         const HistRef& H, uint32_t y0, uint32_t yend, uint32_t xo, uint32_t oob,
                                         uint64_t own_x)
{
    constexpr uint32_t CH = kChunk2;
    constexpr uint32_t kGroup2 = 8;   // rows whose adds share one lane mask
    static_assert(CH % kGroup2 == 0, "row chunks hold whole groups");
    const uint32_t SM = sentinel_key<WIN>(H.sm);
    constexpr int S0 = CONS == CONS_VERTEX ? 1 : -1;
    using T = typename ValT<DT>::T;
    const T* __restrict__ img = (const T*)data;
    const uint32_t row_bytes = (uint32_t)(n2 * (int64_t)sizeof(T));
    const uint32_t xob = xo * (uint32_t)sizeof(T);
    // rows ys .. ys+CH-1 (those inside the image)
    auto load_chunk = [&](uint32_t ys, T (&raw)[CH]) {
        const __amdgpu_buffer_rsrc_t rs = rsrc_at(img + (int64_t)ys * n2);
        uint32_t soff = 0;
#pragma unroll
        for (uint32_t k = 0; k < CH; ++k) {
            raw[k] = (ys + k < n1) ? buffer_load<T>(rs, xob, soff) : T(0);
            soff = advance(soff, row_bytes);
        }
    };
    // the same when every row lies in the image (no per-row checks)
    auto load_chunk_full = [&](uint32_t ys, T (&raw)[CH]) {
        const __amdgpu_buffer_rsrc_t rs = rsrc_at(img + (int64_t)ys * n2);
        uint32_t soff = 0;
#pragma unroll
        for (uint32_t k = 0; k < CH; ++k) {
            raw[k] = buffer_load<T>(rs, xob, soff);
            soff = advance(soff, row_bytes);
        }
    };
    uint32_t c0, c1;   // types of the current row
    int32_t d0, d1;    // d of the previous step
    {
        const uint32_t k = key_of<DT, IDENT>(img[(int64_t)y0 * n2 + xo], P, oob);
        c0 = k;
        c1 = op_right<CONS>(k);
        // the image's first row wins the interval before it (d = -1); a type
        // whose cells do not exist (the sentinel) starts with d = 0, so all its
        // counts are 0 (they may land on any word, the other copy's included)
        d0 = (y0 == 0 && c0 != SM) ? -1 : 0;
        d1 = (y0 == 0 && c1 != SM) ? -1 : 0;
    }
    T raw[CH];
    if (y0 + CH < n1) load_chunk_full(y0 + 1, raw);
    else load_chunk(y0 + 1, raw);
    for (uint32_t y = y0; y < yend; y += CH) {
        // uniform per chunk: the rows below (y+1 .. y+CH) all lie in the image
        uint32_t b[CH];
        if (y + CH < n1) {
#pragma unroll
            for (uint32_t k = 0; k < CH; ++k) b[k] = key_of<DT, IDENT>(raw[k], P, oob);
        } else {
#pragma unroll
            for (uint32_t k = 0; k < CH; ++k)
                b[k] = (y + 1 + k < n1) ? key_of<DT, IDENT>(raw[k], P, oob) : SM;
        }
        if (y + CH < yend) {
            if (y + 2 * CH < n1) load_chunk_full(y + CH + 1, raw);
            else load_chunk(y + CH + 1, raw);
        }
        // the counts of a group of rows first, then their adds under one lane
        // mask (rows past the image, at the end of the last chunk, have no cells)
#pragma unroll
        for (uint32_t g = 0; g < CH; g += kGroup2) {
            uint32_t a0[kGroup2], a1[kGroup2];
            int32_t e0[kGroup2], e1[kGroup2];
#pragma unroll
            for (uint32_t k = 0; k < kGroup2; ++k) {
                const uint32_t n0 = b[g + k], n1v = op_right<CONS>(b[g + k]);
                a0[k] = c0;
                a1[k] = c1;
                e0[k] = step_count<S0>(c0, n0, d0);
                e1[k] = step_count<-S0>(c1, n1v, d1);
                c0 = n0;
                c1 = n1v;
            }
            if (y + g + kGroup2 <= n1) {
                if (lane_bit(own_x)) {
#pragma unroll
                    for (uint32_t k = 0; k < kGroup2; ++k) {
                        hist_add<WIN>(H, a0[k], e0[k]);
                        hist_add<WIN>(H, a1[k], e1[k]);
                    }
                }
            } else {
#pragma unroll
                for (uint32_t k = 0; k < kGroup2; ++k) {
                    if (lane_bit(y + g + k < n1 ? own_x : 0ull)) {
                        hist_add<WIN>(H, a0[k], e0[k]);
                        hist_add<WIN>(H, a1[k], e1[k]);
                    }
                }
            }
        }
    }
    // the next brick's first row (yend) starts with d = 0: the -d of this
    // brick's last step is added here
    if (yend < n1 && lane_bit(own_x)) {
        hist_add<WIN>(H, c0, S0 > 0 ? -d0 : d0);
        hist_add<WIN>(H, c1, S0 > 0 ? d1 : -d1);
    }
}

// Column placement of one wave inside a workgroup brick whose first lane sits
// at position column x0: lane l at column x0 + 63 * wave + l.
struct WaveCols {
    bool active;       // the wave owns at least one position column (columns below n2)
    uint32_t oob;      // 0 if this lane's column lies inside the image, else the sentinel
    uint64_t own;      // lanes 0..62 at columns below n2: the lanes that add (a lane past
                       // the image only has cells that do not exist, whose counts would all
                       // go to the one spare word and collide there)
    uint32_t xo;       // this lane's column, clamped into the image (what it loads)
};

// Index of this wave in its workgroup, known to the compiler to be wave-uniform.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

template <bool WIN>
__device__ __forceinline__ WaveCols wave_cols(int64_t x0, int wave, int64_t n2, uint32_t sm)
{
    WaveCols w;
    const int64_t first = x0 + (int64_t)wave * kLaneCols;
    w.active = first < n2;
    const int64_t x = first + (int64_t)lane_id();
    const bool x_ok = x >= 0 && x < n2;
    w.oob = x_ok ? 0u : sentinel_key<WIN>(sm);
    w.own = ballot(x < n2) & kOwnLanes;
    w.xo = (uint32_t)(x < 0 ? 0 : (x >= n2 ? n2 - 1 : x));
    return w;
}

// Where one wave works in a 3D brick: its first row ys (row r of the brick is
// image row ys + r), planes [z0, zend), the lane's byte offset in a row (xob)
// and out-of-image mask (oob), the lanes that add (own), and the rows [r_lo,
// r_hi) of the brick that lie in the image.
struct Brick3 {
    bool active;
    int64_t ys;
    uint32_t z0, zend, xob, oob;
    uint64_t own;
    int r_lo, r_hi;
};

// The planes of plane block zb.
__device__ __forceinline__ void brick_planes(const EccLaunch& L, uint32_t zb, Brick3& B)
{
    B.z0 = zb * (uint32_t)L.depth;
    const int64_t z_own = L.z_own;   // planes counted (the image's, or a slab's)
    B.zend = ((int64_t)B.z0 + L.depth < z_own) ? B.z0 + (uint32_t)L.depth : (uint32_t)z_own;
}

// An ordinary 3D workgroup brick (x-chunk xc, strip yb, plane block zb) for
// wave xw.  Position columns and rows start at -1 for the top filtration (the
// lattice point before voxel 0).
template <int DT, int CONS, bool WIN>
__device__ __forceinline__ Brick3 chunk_brick_3d(const EccLaunch& L, const HistRef& H, int64_t chunk, uint32_t xc,
                                                 uint32_t yb, uint32_t zb, int xw)
{
    xc = uniform_u32(xc);
    yb = uniform_u32(yb);
    zb = uniform_u32(zb);
    constexpr int NR = kRows3;
    constexpr int64_t org = CONS == CONS_TOP ? -1 : 0;
    using T = typename ValT<DT>::T;
    const int64_t n1 = L.g.n1, n2 = L.g.n2;
    const WaveCols w = wave_cols<WIN>(org + (int64_t)xc * chunk, xw, n2, H.sm);
    Brick3 B;
    B.active = w.active;
    B.xob = w.xo * (uint32_t)sizeof(T);
    B.oob = w.oob;
    B.own = w.own;
    B.ys = org + (int64_t)yb * NR;
    brick_planes(L, zb, B);
    // rows r in [r_lo, r_hi) of the brick lie inside the image
    B.r_lo = B.ys < 0 ? (int)(-B.ys) : 0;
    B.r_hi = (int)((n1 - B.ys) < NR + 1 ? (n1 - B.ys) : NR + 1);
    return B;
}

// A packed tail brick (packed brick pk of plane block zb, Layout3) for wave xw:
// tail strips s0 .. s0 + spw - 1, lane l on strip s0 + l / (t + 1) and position
// column tail_start + l % (t + 1); the lanes at l % (t + 1) == t only supply
// their left neighbours' right ones.  Every strip's rows lie in the image, so the
// brick is a full one, each lane's row offset folded into its column offset.
template <int DT, int CONS, bool WIN>
__device__ __forceinline__ Brick3 tail_brick_3d(const EccLaunch& L, const HistRef& H, const Layout3& Y, int waves,
                                                uint32_t pk, uint32_t zb, int xw)
{
    pk = uniform_u32(pk);
    zb = uniform_u32(zb);
    constexpr int NR = kRows3;
    constexpr int64_t org = CONS == CONS_TOP ? -1 : 0;
    using T = typename ValT<DT>::T;
    const int64_t n2 = L.g.n2;
    const int64_t s0 = Y.sa + ((int64_t)pk * waves + xw) * Y.spw;   // the wave's first strip
    Brick3 B;
    B.active = s0 < Y.sb;
    const uint32_t group = (uint32_t)Y.t + 1u;
    // the lane's place, computed here for each brick: the empty asm keeps the
    // compiler from hoisting these per-lane values out of the brick loop, where
    // they would hold registers through every brick's body
    uint32_t lane = lane_id();
    asm volatile("" : "+v"(lane));
    uint32_t q = lane / group;
    const uint32_t j = lane - q * group;
    const bool strip_ok = q < (uint32_t)Y.spw && s0 + (int64_t)q < Y.sb;
    if (!strip_ok) q = 0;   // reads the wave's first strip, adds nothing
    const int64_t x = org + Y.nxc * kLaneCols * waves + (int64_t)j;
    const bool x_ok = x >= 0 && x < n2;
    B.oob = x_ok ? 0u : sentinel_key<WIN>(H.sm);
    B.own = ballot(strip_ok && j < (uint32_t)Y.t);
    const uint32_t xo = (uint32_t)(x < 0 ? 0 : (x >= n2 ? n2 - 1 : x));
    const uint32_t row_bytes = (uint32_t)(n2 * (int64_t)sizeof(T));
    B.xob = xo * (uint32_t)sizeof(T) + q * (uint32_t)NR * row_bytes;
    B.ys = org + s0 * NR;
    brick_planes(L, zb, B);
    B.r_lo = 0;
    B.r_hi = NR + 1;
    return B;
}

// Runs a 3D brick (the body is inlined once for every kind of brick).
template <int DT, int CONS, bool WIN, bool PAIR = false>
__device__ __forceinline__ void run_brick3(const EccLaunch& L, const BinParams& P, const HistRef& H, const Brick3& B)
{
    constexpr int NR = kRows3;
    if (!B.active) return;
    const bool full = B.r_lo == 0 && B.r_hi == NR + 1;
    const int64_t ys = B.ys;
    const uint32_t z0 = B.z0, ze = B.zend, xob = B.xob, oob = B.oob;
    const uint64_t own = B.own;
    if (DT != DT_F32 && uniform_flag(P.ident)) {
        if (full) brick_3d<DT, CONS, WIN, true, true, PAIR>(L, P, H, ys, z0, ze, xob, oob, own, B.r_lo, B.r_hi);
        else brick_3d<DT, CONS, WIN, false, true, PAIR>(L, P, H, ys, z0, ze, xob, oob, own, B.r_lo, B.r_hi);
    } else {
        if (full) brick_3d<DT, CONS, WIN, true, false, PAIR>(L, P, H, ys, z0, ze, xob, oob, own, B.r_lo, B.r_hi);
        else brick_3d<DT, CONS, WIN, false, false, PAIR>(L, P, H, ys, z0, ze, xob, oob, own, B.r_lo, B.r_hi);
    }
}

// One 2D workgroup brick (x-chunk xc, row block yb) for this wave.
template <int DT, int CONS, bool WIN>
__device__ __forceinline__ void run_brick_2d(const EccLaunch& L, const BinParams& P, const HistRef& H,
                                             int64_t chunk, uint32_t xc, uint32_t yb, int xw)
{
    xc = uniform_u32(xc);
    yb = uniform_u32(yb);
    constexpr int64_t org = CONS == CONS_TOP ? -1 : 0;
    const int64_t n1 = L.g.n1, n2 = L.g.n2;
    const WaveCols w = wave_cols<WIN>(org + (int64_t)xc * chunk, xw, n2, H.sm);
    if (!w.active) return;
    const uint32_t y0 = yb * (uint32_t)L.depth;
    const uint32_t yend = (int64_t)y0 + L.depth < n1 ? y0 + (uint32_t)L.depth : (uint32_t)n1;
    if (DT != DT_F32 && uniform_flag(P.ident))
        brick_2d<DT, CONS, WIN, true>(L.data, (uint32_t)n1, n2, P, H, y0, yend, w.xo, w.oob, w.own);
    else
        brick_2d<DT, CONS, WIN, false>(L.data, (uint32_t)n1, n2, P, H, y0, yend, w.xo, w.oob, w.own);
}

}  // namespace dev
}  // namespace ecc
