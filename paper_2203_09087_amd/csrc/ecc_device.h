// ecc_device.h -- device-side building blocks shared by the single-image and
// the batched kernels (binning, wave helpers, the 2D row step, brick bodies).
//
// What is computed (Wang, Wagner, Chen, SoCG 2022):
//   VCEC[j] = sum over cells of the cubical complex whose value has bin j of
//             (-1)^dim  (Sec. 2.3), and the ECC is its prefix sum (Eq. (1)).
// Each cell is credited to the voxel that completes it (Sec. 2.3, "Faces
// introduced by a voxel"; Algorithm 1), so every voxel adds one signed count to
// the histogram at its own bin.
//
// Who completes a cell.  In the vertex filtration a cell's value is the largest
// bin among its vertices; voxel v completes it if v beats every other vertex,
// "beats" = larger bin, ties won by the later raster position.  In the top
// filtration (the paper's) a face takes the smallest bin among the voxels that
// contain it; v introduces it if v beats them all with "beats" = smaller bin,
// ties won by the earlier position (the paper's tie-break).  Between two voxels
// inside the image exactly one of "v beats u (vertex)" and "v beats u (top)"
// holds, and a voxel outside the image loses every top comparison and wins
// every vertex one (it belongs to no vertex cell).  So one bit per neighbour,
//     w(u) = [v wins the vertex comparison against u]   (0 for u outside),
// serves both filtrations: x = w (vertex) or x = ~w (top).
//
// 2D: around a pixel, the 9 cells that contain it are summed as
//     P(x) = 1 - sum_{i in (t, r, b, l)} x(e_i) & ~(x(e_{i-1}) & x(d_{i-1,i}))
// (e = edge neighbours in cyclic order, d = the diagonal between two of them).
// The vertex VCEC of an image is sum_v P(w)(v) at bin(v); the top VCEC is
// sum_v P(~w)(v).
//
// 3D: a cell is (2D cell) x (z-vertex or z-edge).  Its value is the max (vertex)
// or min (top) over its voxels, so the cells over the z-edge [z, z+1] behave like
// the 2D complex of the plane max(P_z, P_{z+1}) (vertex) and the faces at the
// lattice point z like the 2D complex of min(P_{z-1}, P_z) (top):
//   vertex:  VCEC = sum_z V2(P_z) - sum_{z<n-1} V2(max(P_z, P_{z+1}))
//   top:     VCEC = sum_z c_z T2(P_z) + sum_{z<n-1} T2(min(P_z, P_{z+1})),
//            c_z = -1 + [z == 0] + [z == n-1]
// so the 3D kernel solves two 2D problems per plane.
//
// Mapping to the hardware.  One wave handles a brick of 64 consecutive x
// positions; lanes 0 and 63 are halo (read, never credited), lanes 1..62 own their
// voxel.  Neighbours along x come from the adjacent lane through DPP; every
// comparison is one v_cmp whose result is a 64-bit lane mask in SGPRs, and all of
// the cell logic runs on the scalar unit, 64 voxels per instruction.  Only the
// comparisons a voxel makes with its right and lower neighbours are evaluated;
// the ones with its left and upper neighbours are the complements of the
// neighbours' results, shifted by one lane.  The per-voxel signed count is
// assembled with carry-in adds (v_addc/v_subb with the mask as carry) and added
// to a workgroup histogram in LDS by one ds_add per row (lanes that own no voxel
// add into a spare word of their own, which is cheaper than masking the add).
// Workgroup histograms are merged and prefix-scanned by a second kernel.
#pragma once

#include "ecc_internal.h"

namespace ecc {
namespace dev {


constexpr uint32_t kSentinel = 0xFFFFFFFFu;   // above every key
constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr uint64_t kOwnLanes = 0x7FFFFFFFFFFFFFFEull;   // lanes 1..62

// ------------------------------------------------------------------ binning
//
// The kernels compare and store KEYS = 4 * bin: the order is that of the bins,
// and a key is directly the byte offset of its counter in the LDS histogram.

template <int DT> struct ValT;
template <> struct ValT<DT_U8> { using T = uint8_t; };
template <> struct ValT<DT_U16> { using T = uint16_t; };
template <> struct ValT<DT_F32> { using T = float; };

// Key (bin << kKeyShift, its LDS byte address) of one value, OR-ed with `oob`:
// 0, or ~0 for lanes outside the image, which makes the key the sentinel.
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

// lane i <- lane i+1 (lane 63 gets 0; it is never owned)
__device__ __forceinline__ uint32_t from_right(uint32_t v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x130 /* wave_shl:1 */, 0xF, 0xF, true);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ bool lane_bit(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }


// acc - [lane bit of m]
__device__ __forceinline__ int32_t sub_bit(int32_t acc, uint64_t m)
{
    int32_t r;
    uint64_t carry;
    asm("v_subb_co_u32_e64 %0, %1, %2, 0, %3" : "=v"(r), "=s"(carry) : "v"(acc), "s"(m));
    return r;
}

// acc + [lane bit of m]
__device__ __forceinline__ int32_t add_bit(int32_t acc, uint64_t m)
{
    int32_t r;
    uint64_t carry;
    asm("v_addc_co_u32_e64 %0, %1, %2, 0, %3" : "=v"(r), "=s"(carry) : "v"(acc), "s"(m));
    return r;
}

// ------------------------------------------------- one row of a 2D problem

// State carried from row to row of one 2D problem (one wave, 64 columns).
struct RowState {
    uint32_t c;        // keys of the current row
    uint32_t c_right;  // keys of the current row, one lane to the right
    uint64_t fb;       // previous row: [above(x) > current(x)]
    uint64_t fbr;      // previous row: [above(x) > current(x+1)]
    uint64_t q;        // previous row: [current(x) >= above(x+1)]
};

__device__ __forceinline__ void row_start(RowState& s, uint32_t above, uint32_t cur)
{
    s.c = cur;
    s.c_right = from_right(cur);
    const uint32_t above_right = from_right(above);
    s.fb = ballot(above > cur);
    s.fbr = ballot(above > s.c_right);
    s.q = ballot(cur >= above_right);
}

struct HistRef {
    int32_t* hist;     // LDS: kMaxLdsBins counters, then one spare word per lane
    uint32_t key_lo;   // key of the first bin of the window
    uint32_t key_span; // keys in the window
    uint32_t spare;    // byte offset of this lane's spare word (absorbs adds that do not count)
};

__device__ __forceinline__ uint32_t spare_offset() { return (uint32_t)(kMaxLdsBins + lane_id()) * 4u; }

__device__ __forceinline__ HistRef hist_ref(int32_t* hist, int32_t bin_lo, int32_t width)
{
    return HistRef{hist, (uint32_t)bin_lo << kKeyShift, (uint32_t)width << kKeyShift, spare_offset()};
}

__device__ __forceinline__ void hist_add(const HistRef& H, uint32_t key, int32_t v)
{
    atomicAdd((int32_t*)((char*)H.hist + key), v);
}

// Credits the current row (owned lanes `own`) with sign SIGN and advances the
// state to `below`.
template <int CONS, int SIGN, bool WIN, bool CHECK = true>
__device__ __forceinline__ void row_step(RowState& s, uint32_t below, uint64_t own, const HistRef& H)
{
    const uint32_t c = s.c;
    // The four comparisons of this row pair.  The lower-left one comes out of q
    // shifted by a lane, [c(x) > b(x-1)] = ~[b(x-1) >= c(x)], which saves moving
    // the lower row to the left; the next row reads q itself as its upper-right
    // comparison.
    const uint32_t b_right = from_right(below);
    const uint64_t fr = ballot(c > s.c_right);
    const uint64_t fbr = ballot(c > b_right);
    const uint64_t q = ballot(below >= s.c_right);
    const uint64_t fb = ballot(c > below);
    if (!CHECK || own) {
        // vertex-comparison bits of the 8 neighbours (later voxels win ties)
        uint64_t er = fr, eb = fb, dbr = fbr, dbl = ~(q << 1);
        uint64_t el = ~(fr << 1), et = ~s.fb, dtl = ~(s.fbr << 1), dtr = s.q;
        if constexpr (CONS == CONS_TOP) {
            er = ~er; eb = ~eb; dbr = ~dbr; dbl = ~dbl;
            el = ~el; et = ~et; dtl = ~dtl; dtr = ~dtr;
        }
        const uint64_t tt = et & ~(el & dtl);
        const uint64_t tr = er & ~(et & dtr);
        const uint64_t tb = eb & ~(er & dbr);
        const uint64_t tl = el & ~(eb & dbl);
        int32_t v;
        if constexpr (SIGN > 0) v = sub_bit(sub_bit(sub_bit(sub_bit(1, tt), tr), tb), tl);
        else v = add_bit(add_bit(add_bit(add_bit(-1, tt), tr), tb), tl);
        // every lane adds; lanes that do not count add into their spare word
        uint32_t key = c;
        bool hit = lane_bit(own);
        if constexpr (WIN) {
            key -= H.key_lo;
            hit = hit && key < H.key_span;
        }
        hist_add(H, hit ? key : H.spare, v);
    }
    s.fb = fb;
    s.fbr = fbr;
    s.q = q;
    s.c = below;
    s.c_right = b_right;
}

// ------------------------------------------------------------ main kernels

__device__ __forceinline__ void zero_hist(int32_t* hist, int width)
{
    for (int j = threadIdx.x; j < width; j += blockDim.x) hist[j] = 0;
    __syncthreads();
}

// Writes the workgroup histogram (negated with sign -1) to dst[0..width), or
// adds it to what dst holds (add).
__device__ __forceinline__ void flush_hist(const int32_t* hist, int32_t* dst, int width, bool add = false,
                                           int sign = 1)
{
    __syncthreads();
    if (!add) {
        for (int j = threadIdx.x; j < width; j += blockDim.x) {
            const int32_t t = hist[j];
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
                const int32_t t = hist[j];
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

// One plane step of a 3D brick: problem A on plane z with sign SA (0: skipped)
// and, with HASB, problem B on the combined plane of z and z+1 with sign SB.
// The two problems are independent and are advanced row by row together.
template <int CONS, bool WIN, bool FULL, int SA, bool HASB, int NR>
__device__ __forceinline__ void plane_step(const uint32_t (&Bc)[NR + 2], const uint32_t (&Bn)[NR + 2],
                                           uint64_t own_x, int rows_owned, const HistRef& H)
{
    constexpr int SB = (CONS == CONS_TOP) ? +1 : -1;
    auto comb = [&](int r) -> uint32_t {
        return (CONS == CONS_TOP) ? min(Bc[r], Bn[r]) : max(Bc[r], Bn[r]);
    };
    RowState sa, sb;
    if constexpr (SA != 0) row_start(sa, Bc[0], Bc[1]);
    if constexpr (HASB) row_start(sb, comb(0), comb(1));
#pragma unroll
    for (int r = 1; r <= NR; ++r) {
        const uint64_t own = (FULL || r <= rows_owned) ? own_x : 0ull;
        if constexpr (SA != 0) row_step<CONS, SA, WIN, false>(sa, Bc[r + 1], own, H);
        if constexpr (HASB) row_step<CONS, SB, WIN, false>(sb, comb(r + 1), own, H);
    }
}

// The planes of one 3D brick.  Row r of the brick is image row y0 - 1 + r.
// FULL: every row of the brick and its halo lies inside the image.  Otherwise
// the rows outside [0, n1) read the nearest row inside (so every load is in
// bounds) and take the sentinel key, and rows past the brick's owned rows count
// nothing; both without branches, so boundary bricks cost about what inner ones
// do.  Plane indices are 32-bit (see brick_2d).
// PAIR: the volume is the elementwise max (vertex) or min (top) of L.data and
// L.data2, taken on the keys (the bins' order, so exactly the bin of the max or
// min value): the combined hyperplanes of a 4D image.
template <int DT, int CONS, bool WIN, bool FULL, bool IDENT, bool PAIR>
__device__ __forceinline__ void brick_3d(const EccLaunch& L, const BinParams& P, const HistRef& H, int64_t y0,
                                         uint32_t z0, uint32_t zend, uint32_t xob, uint32_t oob, uint64_t own_x,
                                         int rows_owned, int r_lo, int r_hi)
{
    constexpr int NR = kRows3;
    using T = typename ValT<DT>::T;
    const uint32_t n0 = (uint32_t)L.g.n0;
    const int64_t n1 = L.g.n1, n2 = L.g.n2;
    const uint32_t row_bytes = (uint32_t)(n2 * (int64_t)sizeof(T));
    const char* img = (const char*)L.data;
    const char* img2 = (const char*)L.data2;
    // first row read: y0 - 1, or the first row inside the image
    const int64_t ybase = y0 - 1 + (FULL ? 0 : r_lo);
    constexpr int NR2 = PAIR ? NR + 2 : 1;

    auto load_plane = [&](uint32_t z, T (&raw)[NR + 2], T (&raw2)[NR2]) {
        const int64_t off = ((int64_t)z * n1 + ybase) * (int64_t)row_bytes;
        const __amdgpu_buffer_rsrc_t rs = rsrc_at(img + off);
        __amdgpu_buffer_rsrc_t rs2 = rs;
        if constexpr (PAIR) rs2 = rsrc_at(img2 + off);
        uint32_t soff = 0;
#pragma unroll
        for (int r = 0; r < NR + 2; ++r) {
            raw[r] = buffer_load<T>(rs, xob, soff);
            if constexpr (PAIR) raw2[r] = buffer_load<T>(rs2, xob, soff);
            // advance while the next row still lies inside the image
            if (FULL || (r >= r_lo && r + 1 < r_hi)) soff = advance(soff, row_bytes);
        }
    };
    auto keys = [&](const T (&raw)[NR + 2], const T (&raw2)[NR2], uint32_t (&B)[NR + 2]) {
#pragma unroll
        for (int r = 0; r < NR + 2; ++r) {
            const uint32_t outside = (FULL || (r >= r_lo && r < r_hi)) ? 0u : ~0u;
            B[r] = key_of<DT, IDENT>(raw[r], P, oob | outside);
            if constexpr (PAIR) {
                const uint32_t k2 = key_of<DT, IDENT>(raw2[r], P, oob | outside);
                B[r] = CONS == CONS_VERTEX ? max(B[r], k2) : min(B[r], k2);
            }
        }
    };

    uint32_t Bc[NR + 2], Bn[NR + 2];
    T raw[NR + 2], raw2[NR2];
    load_plane(z0, raw, raw2);
    keys(raw, raw2, Bc);
    for (uint32_t z = z0; z < zend; ++z) {
        // the next plane's loads are waited for here; other waves' arithmetic
        // covers their latency (a plane prefetched one step ahead measured no gain)
        const bool has1 = z + 1 < n0;
        if (has1) {
            load_plane(z + 1, raw, raw2);
            keys(raw, raw2, Bn);
        }
        if constexpr (CONS == CONS_VERTEX) {
            if (has1) plane_step<CONS, WIN, FULL, +1, true, NR>(Bc, Bn, own_x, rows_owned, H);
            else plane_step<CONS, WIN, FULL, +1, false, NR>(Bc, Bn, own_x, rows_owned, H);
        } else {
            // top filtration: plane z enters with -1 + [z == 0] + [z == n0-1]
            // (positions in the whole volume)
            const int64_t zg = L.z_base + (int64_t)z;
            const int ca = -1 + (zg == 0) + (zg == L.n0_global - 1);
            if (has1) {
                if (ca < 0) plane_step<CONS, WIN, FULL, -1, true, NR>(Bc, Bn, own_x, rows_owned, H);
                else plane_step<CONS, WIN, FULL, 0, true, NR>(Bc, Bn, own_x, rows_owned, H);
            } else {
                if (ca > 0) plane_step<CONS, WIN, FULL, +1, false, NR>(Bc, Bn, own_x, rows_owned, H);
                else if (ca < 0) plane_step<CONS, WIN, FULL, -1, false, NR>(Bc, Bn, own_x, rows_owned, H);
            }
        }
#pragma unroll
        for (int r = 0; r < NR + 2; ++r) Bc[r] = Bn[r];
    }
}

// The rows [y0, yend) of one 2D brick for one wave: rows are streamed in chunks
// of kChunk2, the next chunk loading while the current one is processed.
// Row indices are 32-bit (the scalar unit compares 32-bit values only; 64-bit
// loop bounds would move the loop, and every mask derived from it, to vector
// registers).  Rows are at most 2^31, so y + 2 * kChunk2 does not wrap.
template <int DT, int CONS, bool WIN, bool IDENT>
__device__ __forceinline__ void brick_2d(const void* data, uint32_t n1, int64_t n2, const BinParams& P,
                                         const HistRef& H, uint32_t y0, uint32_t yend, uint32_t xo, uint32_t oob,
                                         uint64_t own_x)
{
    constexpr uint32_t CH = kChunk2;
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
    RowState s;
    {
        const uint32_t above = y0 == 0 ? kSentinel : key_of<DT, IDENT>(img[(int64_t)(y0 - 1) * n2 + xo], P, oob);
        row_start(s, above, key_of<DT, IDENT>(img[(int64_t)y0 * n2 + xo], P, oob));
    }
    T raw[CH];
    if (y0 + CH < n1) load_chunk_full(y0 + 1, raw);
    else load_chunk(y0 + 1, raw);
    for (uint32_t y = y0; y < yend; y += CH) {
        // Uniform per chunk: the rows below (y+1 .. y+CH) all lie in the image,
        // and the rows owned (y .. y+CH-1) all lie in the brick.
        const bool keys_full = y + CH < n1;
        const bool own_full = y + CH <= yend;
        uint32_t b[CH];
        if (keys_full) {
#pragma unroll
            for (uint32_t k = 0; k < CH; ++k) b[k] = key_of<DT, IDENT>(raw[k], P, oob);
        } else {
#pragma unroll
            for (uint32_t k = 0; k < CH; ++k)
                b[k] = (y + 1 + k < n1) ? key_of<DT, IDENT>(raw[k], P, oob) : kSentinel;
        }
        if (y + CH < yend) {
            if (y + 2 * CH < n1) load_chunk_full(y + CH + 1, raw);
            else load_chunk(y + CH + 1, raw);
        }
        if (own_full) {
#pragma unroll
            for (uint32_t k = 0; k < CH; ++k) row_step<CONS, +1, WIN, false>(s, b[k], own_x, H);
        } else {
            // rows past the brick run with no owned lanes (a branch around
            // them here would make the compiler treat the row state as divergent)
#pragma unroll
            for (uint32_t k = 0; k < CH; ++k) {
                const uint64_t own = (y + k < yend) ? own_x : 0ull;
                row_step<CONS, +1, WIN, false>(s, b[k], own, H);
            }
        }
    }
}

// Column placement of one wave inside a workgroup brick: lane 0 and lane 63 are
// halo, lanes 1..62 own columns x0 + 62 * wave + lane - 1.
struct WaveCols {
    bool active;       // the wave owns at least one column of the image
    uint32_t oob;      // 0 if this lane's column lies inside the image, else ~0
    uint64_t own_x;    // owned lanes
    uint32_t xo;       // this lane's column, clamped into the image
};

// Index of this wave in its workgroup, known to the compiler to be wave-uniform.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

__device__ __forceinline__ WaveCols wave_cols(int64_t x0, int wave, int64_t n2)
{
    WaveCols w;
    const int64_t first = x0 + (int64_t)wave * 62;
    w.active = first < n2;
    const int64_t x = first - 1 + (int64_t)lane_id();
    const bool x_ok = x >= 0 && x < n2;
    const uint64_t xmask = ballot(x_ok);
    w.oob = x_ok ? 0u : ~0u;
    w.own_x = xmask & kOwnLanes;
    w.xo = (uint32_t)(x < 0 ? 0 : (x >= n2 ? n2 - 1 : x));
    return w;
}

// One 3D workgroup brick (x-chunk xc, row block yb, plane block zb) for this wave.
// `xw`: this wave's place among the waves of the brick (columns xw*62 ..).
template <int DT, int CONS, bool WIN, bool PAIR = false>
__device__ __forceinline__ void run_brick_3d(const EccLaunch& L, const BinParams& P, const HistRef& H,
                                             int64_t chunk, uint32_t xc, uint32_t yb, uint32_t zb, int xw)
{
    xc = uniform_u32(xc);
    yb = uniform_u32(yb);
    zb = uniform_u32(zb);
    constexpr int NR = kRows3;
    using T = typename ValT<DT>::T;
    const int64_t n1 = L.g.n1, n2 = L.g.n2;
    const WaveCols w = wave_cols((int64_t)xc * chunk, xw, n2);
    if (!w.active) return;
    const uint32_t xob = w.xo * (uint32_t)sizeof(T);
    const int64_t y0 = (int64_t)yb * NR;
    const int rows_owned = (int)((n1 - y0) < NR ? (n1 - y0) : NR);
    const uint32_t z0 = zb * (uint32_t)L.depth;
    const int64_t z_own = L.z_own;   // planes counted (the image's, or a slab's)
    const uint32_t zend = ((int64_t)z0 + L.depth < z_own) ? z0 + (uint32_t)L.depth : (uint32_t)z_own;
    // rows r in [r_lo, r_hi) of the brick (row r is y0 - 1 + r) lie inside the image
    const int r_lo = (y0 == 0) ? 1 : 0;
    const int r_hi = (int)((n1 - (y0 - 1)) < NR + 2 ? (n1 - (y0 - 1)) : NR + 2);
    const bool full = r_lo == 0 && r_hi == NR + 2;
    if (DT != DT_F32 && uniform_flag(P.ident)) {
        if (full) brick_3d<DT, CONS, WIN, true, true, PAIR>(L, P, H, y0, z0, zend, xob, w.oob, w.own_x, rows_owned, r_lo, r_hi);
        else brick_3d<DT, CONS, WIN, false, true, PAIR>(L, P, H, y0, z0, zend, xob, w.oob, w.own_x, rows_owned, r_lo, r_hi);
    } else {
        if (full) brick_3d<DT, CONS, WIN, true, false, PAIR>(L, P, H, y0, z0, zend, xob, w.oob, w.own_x, rows_owned, r_lo, r_hi);
        else brick_3d<DT, CONS, WIN, false, false, PAIR>(L, P, H, y0, z0, zend, xob, w.oob, w.own_x, rows_owned, r_lo, r_hi);
    }
}

// One 2D workgroup brick (x-chunk xc, row block yb) for this wave.
template <int DT, int CONS, bool WIN>
__device__ __forceinline__ void run_brick_2d(const EccLaunch& L, const BinParams& P, const HistRef& H,
                                             int64_t chunk, uint32_t xc, uint32_t yb, int xw)
{
    xc = uniform_u32(xc);
    yb = uniform_u32(yb);
    const int64_t n1 = L.g.n1, n2 = L.g.n2;
    const WaveCols w = wave_cols((int64_t)xc * chunk, xw, n2);
    if (!w.active) return;
    const uint32_t y0 = yb * (uint32_t)L.depth;
    const uint32_t yend = (int64_t)y0 + L.depth < n1 ? y0 + (uint32_t)L.depth : (uint32_t)n1;
    if (DT != DT_F32 && uniform_flag(P.ident))
        brick_2d<DT, CONS, WIN, true>(L.data, (uint32_t)n1, n2, P, H, y0, yend, w.xo, w.oob, w.own_x);
    else
        brick_2d<DT, CONS, WIN, false>(L.data, (uint32_t)n1, n2, P, H, y0, yend, w.xo, w.oob, w.own_x);
}

}  // namespace dev
}  // namespace ecc
