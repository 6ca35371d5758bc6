// ecc_kernels.hip -- gfx950 kernels of the ECC library (first, LDS-tiled path).
//
// Per voxel v the kernel adds to VCEC[bin(v)] the signed count of the cells that
// v completes (Sec. 2.3 "Faces introduced by a voxel", Algorithm 1).  Which voxel
// completes a cell is decided by comparing bins with a fixed tie-break, so each
// cell is credited exactly once:
//   vertex filtration - v completes a cell if it beats every other vertex of it,
//                       "beats" = larger bin, ties won by the later raster index;
//   top filtration    - v introduces a face if it beats every other voxel that
//                       contains it, "beats" = smaller bin, ties won by the earlier
//                       raster index (the rule of Sec. 2.3).
// Voxels outside the image never win against v in the top filtration (the
// paper's +infinity collar) and the cells they would belong to do not exist in
// the vertex filtration; both are the same bit "v beats u" being 0 resp. 1, so a
// sentinel key larger than every bin serves both.
//
// Let w(u) = [v wins the vertex comparison against neighbour u].  In the top
// filtration v wins against u exactly when it does not in the vertex one, so
// x = w (vertex) or x = ~w (top) and the contribution is
//     sum_{o in {-1,0,1}^d} (-1)^{nnz(o)} prod_{0 != delta <= o} x(delta)
// times (-1)^d for the top filtration.  In 2D the sum collapses (around the
// 4-cycle of edge neighbours t, r, b, l) to
//     P(x) = 1 - sum_i x(e_i) & ~(x(e_{i-1}) & x(diag_{i-1,i}))
// and in 3D, splitting the cells by their z extent,
//     C(x) = P(x0) - x(-z) P(x0 & x-) - x(+z) P(x0 & x+)
// where x0, x-, x+ are the 8 in-plane bits of planes z, z-1, z+1.
#include "ecc_internal.h"

namespace ecc {

namespace {

constexpr uint32_t kSentinel = 0xFFFFu;   // larger than every bin (nbins <= 65535)
constexpr int kThreads = 256;

// ------------------------------------------------------------------ binning

template <int DT> struct ValT;
template <> struct ValT<DT_U8> { using T = uint8_t; };
template <> struct ValT<DT_U16> { using T = uint16_t; };
template <> struct ValT<DT_F32> { using T = float; };

template <int DT>
__device__ __forceinline__ uint32_t bin_of(typename ValT<DT>::T v, const BinParams& p)
{
    if constexpr (DT == DT_F32) {
        const float x = v;
        if (x != x) return (uint32_t)(p.nbins - 1);
        if (p.flat) return ((double)x > p.hi) ? (uint32_t)(p.nbins - 1) : 0u;
        const double t = __dmul_rn(__dsub_rn((double)x, p.lo), p.scale);
        if (!(t >= 0.0)) return 0u;
        if (t >= (double)p.nbins) return (uint32_t)(p.nbins - 1);
        return (uint32_t)t;   // t in [0, nbins): truncation is floor
    } else {
        uint32_t a = (uint32_t)v;
        a = a < p.ilo ? p.ilo : (a > p.ihi ? p.ihi : a);
        a -= p.ilo;
        return a * p.q0 + __umulhi(a, p.magic);
    }
}

// ------------------------------------------------------- local contribution

// 2D planar sum over the 9 cells around a voxel; E bit i = x(edge i) for the
// cycle (t, r, b, l), D bit i = x(diagonal between edge i and edge i+1).
__device__ __forceinline__ int planar(uint32_t E, uint32_t D)
{
    const uint32_t X = E & D;
    const uint32_t Xr = ((X << 1) | (X >> 3)) & 0xFu;   // bit i <- bit i-1
    return 1 - __popc(E & ~Xr & 0xFu);
}

// ------------------------------------------------------------ tiled kernel

template <int NDIM> struct Tile;
template <> struct Tile<2> { static constexpr int X = 64, Y = 32, Z = 1; };
template <> struct Tile<3> { static constexpr int X = 32, Y = 8, Z = 8; };

template <int NDIM, int DT, int CONS>
__global__ __launch_bounds__(kThreads) void k_hist_tile(HistLaunch L)
{
    using TL = Tile<NDIM>;
    constexpr int HX = TL::X + 2, HY = TL::Y + 2, HZ = (NDIM == 3) ? TL::Z + 2 : 1;
    constexpr int HALO_N = HX * HY * HZ;
    constexpr int TILE_N = TL::X * TL::Y * TL::Z;
    __shared__ uint16_t tile[HALO_N];
    extern __shared__ int32_t hist[];

    using T = typename ValT<DT>::T;
    const T* __restrict__ img = (const T*)L.data;
    const BinParams P = L.params_dev ? *L.params_dev : L.params;
    const int64_t n0 = L.g.n0, n1 = L.g.n1, n2 = L.g.n2;
    const int64_t tx = (n2 + TL::X - 1) / TL::X;
    const int64_t ty = (n1 + TL::Y - 1) / TL::Y;
    const int64_t tz = (NDIM == 3) ? (n0 + TL::Z - 1) / TL::Z : 1;
    const int64_t ntiles = tx * ty * tz;
    const int tid = threadIdx.x;

    for (int j = tid; j < L.width; j += kThreads) hist[j] = 0;

    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t bx = t % tx, by = (t / tx) % ty, bz = t / (tx * ty);
        const int64_t x0 = bx * TL::X, y0 = by * TL::Y, z0 = bz * TL::Z;
        __syncthreads();   // previous tile fully consumed (and hist zeroed)
        for (int i = tid; i < HALO_N; i += kThreads) {
            const int hx = i % HX, hy = (i / HX) % HY, hz = i / (HX * HY);
            const int64_t gx = x0 - 1 + hx, gy = y0 - 1 + hy;
            const int64_t gz = (NDIM == 3) ? z0 - 1 + hz : 0;
            uint32_t key = kSentinel;
            if (gx >= 0 && gx < n2 && gy >= 0 && gy < n1 && gz >= 0 && gz < n0)
                key = bin_of<DT>(img[(gz * n1 + gy) * n2 + gx], P);
            tile[i] = (uint16_t)key;
        }
        __syncthreads();
        for (int v = tid; v < TILE_N; v += kThreads) {
            const int lx = v % TL::X, ly = (v / TL::X) % TL::Y, lz = v / (TL::X * TL::Y);
            if (x0 + lx >= n2 || y0 + ly >= n1 || z0 + lz >= ((NDIM == 3) ? n0 : 1)) continue;
            const int ci = ((NDIM == 3 ? lz + 1 : 0) * HY + ly + 1) * HX + lx + 1;
            const uint32_t c = tile[ci];
            // w(dz,dy,dx) = [c beats the neighbour in the vertex filtration]
            auto w = [&](int dz, int dy, int dx) -> uint32_t {
                const uint32_t n = tile[ci + (dz * HY + dy) * HX + dx];
                const bool later = dz > 0 || (dz == 0 && (dy > 0 || (dy == 0 && dx > 0)));
                return later ? (c > n ? 1u : 0u) : (c >= n ? 1u : 0u);
            };
            auto edges = [&](int dz) -> uint32_t {
                return w(dz, -1, 0) | (w(dz, 0, 1) << 1) | (w(dz, 1, 0) << 2) | (w(dz, 0, -1) << 3);
            };
            auto diags = [&](int dz) -> uint32_t {
                return w(dz, -1, 1) | (w(dz, 1, 1) << 1) | (w(dz, 1, -1) << 2) | (w(dz, -1, -1) << 3);
            };
            int contrib;
            const uint32_t flip = (CONS == CONS_TOP) ? 0xFu : 0u;
            const uint32_t E0 = edges(0) ^ flip, D0 = diags(0) ^ flip;
            if constexpr (NDIM == 2) {
                contrib = planar(E0, D0);
            } else {
                const uint32_t Em = edges(-1) ^ flip, Dm = diags(-1) ^ flip;
                const uint32_t Ep = edges(1) ^ flip, Dp = diags(1) ^ flip;
                const uint32_t zm = w(-1, 0, 0) ^ (flip & 1u), zp = w(1, 0, 0) ^ (flip & 1u);
                contrib = planar(E0, D0) - (int)zm * planar(E0 & Em, D0 & Dm)
                          - (int)zp * planar(E0 & Ep, D0 & Dp);
                if (CONS == CONS_TOP) contrib = -contrib;
            }
            const int b = (int)c - L.bin_lo;
            if (contrib != 0 && b >= 0 && b < L.width) atomicAdd(&hist[b], contrib);
        }
    }
    __syncthreads();
    int32_t* dst = L.partials + (size_t)blockIdx.x * (size_t)L.width;
    for (int j = tid; j < L.width; j += kThreads) dst[j] = hist[j];
}

// ------------------------------------------------------------------- minmax

// Order-preserving 32-bit keys: integers as themselves; finite floats through
// the usual sign-flip map.  Non-finite floats are skipped.
template <int DT>
__global__ __launch_bounds__(kThreads) void k_minmax(const void* data, int64_t nvox, uint32_t* mm)
{
    using T = typename ValT<DT>::T;
    const T* __restrict__ img = (const T*)data;
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nvox;
         i += (int64_t)gridDim.x * kThreads) {
        uint32_t k;
        if constexpr (DT == DT_F32) {
            const float f = img[i];
            if (!isfinite(f)) continue;
            const uint32_t u = __float_as_uint(f);
            k = (u & 0x80000000u) ? ~u : (u | 0x80000000u);
        } else {
            k = (uint32_t)img[i];
        }
        lo = min(lo, k);
        hi = max(hi, k);
    }
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
    if (threadIdx.x == 0) {
        mm[2 * blockIdx.x] = slo[0];
        mm[2 * blockIdx.x + 1] = shi[0];
    }
}

__device__ double key_to_double(uint32_t k, int dtype)
{
    if (dtype != DT_F32) return (double)k;
    const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return (double)__uint_as_float(u);
}

__global__ __launch_bounds__(kThreads) void k_params(const uint32_t* mm, int blocks, int dtype,
                                                     int32_t nbins, BinParams* out)
{
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (int i = threadIdx.x; i < blocks; i += kThreads) {
        lo = min(lo, mm[2 * i]);
        hi = max(hi, mm[2 * i + 1]);
    }
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
    if (threadIdx.x != 0) return;
    BinParams p = {};
    p.dtype = dtype;
    p.nbins = nbins;
    const bool empty = slo[0] > shi[0];   // no (finite) value at all
    const double dlo = empty ? 0.0 : key_to_double(slo[0], dtype);
    const double dhi = empty ? 0.0 : key_to_double(shi[0], dtype);
    if (dtype == DT_F32) {
        p.lo = dlo;
        p.hi = dhi;
        p.flat = (dhi == dlo) ? 1 : 0;
        p.scale = p.flat ? 0.0 : __ddiv_rn((double)nbins, __dsub_rn(dhi, dlo));
    } else {
        const uint32_t ilo = (uint32_t)dlo, ihi = (uint32_t)dhi;
        const uint64_t D = (uint64_t)(ihi - ilo) + 1u;
        p.ilo = ilo;
        p.ihi = ihi;
        p.q0 = (uint32_t)((uint64_t)nbins / D);
        const uint64_t r = (uint64_t)nbins % D;
        p.magic = (uint32_t)(((r << 32) / D) + 1u);
        p.lo = dlo;
        p.hi = dhi;
    }
    *out = p;
}

// --------------------------------------------------------- reduce and scan

__global__ __launch_bounds__(kThreads) void k_reduce(const int32_t* partials, int grid,
                                                     int32_t width, int64_t* out)
{
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= width) return;
    int64_t s = 0;
    for (int w = 0; w < grid; ++w) s += partials[(size_t)w * (size_t)width + j];
    out[j] = s;
}

constexpr int kScanThreads = 1024;

__global__ __launch_bounds__(kScanThreads) void k_scan(int64_t* v, int32_t n)
{
    __shared__ int64_t part[kScanThreads];
    const int per = (n + kScanThreads - 1) / kScanThreads;
    const int b = threadIdx.x * per;
    const int e = min(n, b + per);
    int64_t s = 0;
    for (int i = b; i < e; ++i) s += v[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int64_t add = (threadIdx.x >= (unsigned)off) ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int64_t acc = part[threadIdx.x] - s;   // exclusive prefix of this chunk
    for (int i = b; i < e; ++i) { acc += v[i]; v[i] = acc; }
}

}  // namespace

int64_t hist_tiles(int ndim, const Geom& g)
{
    if (ndim == 2)
        return ((g.n2 + Tile<2>::X - 1) / Tile<2>::X) * ((g.n1 + Tile<2>::Y - 1) / Tile<2>::Y);
    return ((g.n2 + Tile<3>::X - 1) / Tile<3>::X) * ((g.n1 + Tile<3>::Y - 1) / Tile<3>::Y) *
           ((g.n0 + Tile<3>::Z - 1) / Tile<3>::Z);
}

template <int NDIM, int DT, int CONS>
static hipError_t launch_hist_t(const HistLaunch& L, hipStream_t s)
{
    const size_t lds = (size_t)L.width * sizeof(int32_t);
    hipLaunchKernelGGL((k_hist_tile<NDIM, DT, CONS>), dim3(L.grid), dim3(kThreads), lds, s, L);
    return hipGetLastError();
}

template <int NDIM, int DT>
static hipError_t launch_hist_c(const HistLaunch& L, hipStream_t s)
{
    return L.construction == CONS_TOP ? launch_hist_t<NDIM, DT, CONS_TOP>(L, s)
                                      : launch_hist_t<NDIM, DT, CONS_VERTEX>(L, s);
}

template <int NDIM>
static hipError_t launch_hist_d(const HistLaunch& L, hipStream_t s)
{
    switch (L.dtype) {
    case DT_U8: return launch_hist_c<NDIM, DT_U8>(L, s);
    case DT_U16: return launch_hist_c<NDIM, DT_U16>(L, s);
    default: return launch_hist_c<NDIM, DT_F32>(L, s);
    }
}

hipError_t launch_hist(const HistLaunch& L, hipStream_t s)
{
    return L.ndim == 2 ? launch_hist_d<2>(L, s) : launch_hist_d<3>(L, s);
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

hipError_t launch_params_from_minmax(const uint32_t* mm, int blocks, int dtype, int32_t nbins,
                                     BinParams* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_params, dim3(1), dim3(kThreads), 0, s, mm, blocks, dtype, nbins, out);
    return hipGetLastError();
}

hipError_t launch_reduce(const int32_t* partials, int grid, int32_t width, int64_t* out_window,
                         hipStream_t s)
{
    const int blocks = (width + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_reduce, dim3(blocks), dim3(kThreads), 0, s, partials, grid, width, out_window);
    return hipGetLastError();
}

hipError_t launch_scan(int64_t* out, int32_t nbins, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, out, nbins);
    return hipGetLastError();
}

}  // namespace ecc
