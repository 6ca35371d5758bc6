// ecc_smooth.hip -- separable 13-tap smoothing of a 2D float32 image, the
// smoothing step of the smoothing + ECC pipeline (Sec. 5, "Pipeline").
//
// Two launches: rows (in -> tmp), then columns (tmp -> out).  Each output is
// the sum over k = 0..12, in that order and starting from 0, of w[k] times the
// neighbour at offset k - 6 along the axis (border pixels repeated), every
// product and sum rounded once in float32 (__fmul_rn / __fadd_rn, no fused
// multiply-add).  The row pass stages a row segment plus its 12-pixel halo in
// LDS; the column pass reads 13 rows with coalesced loads (neighbouring
// threads, neighbouring columns).
#include "ecc_internal.h"

namespace ecc {

namespace {

constexpr int kSmoothThreads = 256;

__global__ __launch_bounds__(kSmoothThreads) void k_smooth_rows(const float* __restrict__ in, float* __restrict__ tmp,
                                                                int64_t n1, int64_t n2, Taps13 w)
{
    __shared__ float tile[kSmoothThreads + 12];
    const int64_t x0 = (int64_t)blockIdx.x * kSmoothThreads;
    const int64_t x = x0 + threadIdx.x;
    for (int64_t y = blockIdx.y; y < n1; y += gridDim.y) {
        const float* row = in + y * n2;
        for (int i = threadIdx.x; i < kSmoothThreads + 12; i += kSmoothThreads) {
            int64_t xi = x0 + i - 6;
            xi = xi < 0 ? 0 : (xi >= n2 ? n2 - 1 : xi);
            tile[i] = row[xi];
        }
        __syncthreads();
        if (x < n2) {
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < 13; ++k) acc = __fadd_rn(acc, __fmul_rn(w.w[k], tile[threadIdx.x + k]));
            tmp[y * n2 + x] = acc;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kSmoothThreads) void k_smooth_cols(const float* __restrict__ tmp, float* __restrict__ out,
                                                                int64_t n1, int64_t n2, Taps13 w)
{
    const int64_t x = (int64_t)blockIdx.x * kSmoothThreads + threadIdx.x;
    if (x >= n2) return;
    for (int64_t y = blockIdx.y; y < n1; y += gridDim.y) {
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < 13; ++k) {
            int64_t yy = y + k - 6;
            yy = yy < 0 ? 0 : (yy >= n1 ? n1 - 1 : yy);
            acc = __fadd_rn(acc, __fmul_rn(w.w[k], tmp[yy * n2 + x]));
        }
        out[y * n2 + x] = acc;
    }
}

}  // namespace

hipError_t launch_smooth13(const float* in, float* out, float* tmp, int64_t n1, int64_t n2, const Taps13& w,
                           hipStream_t s)
{
    const dim3 grid((unsigned)((n2 + kSmoothThreads - 1) / kSmoothThreads), (unsigned)(n1 < 65535 ? n1 : 65535));
    hipLaunchKernelGGL(k_smooth_rows, grid, dim3(kSmoothThreads), 0, s, in, tmp, n1, n2, w);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_smooth_cols, grid, dim3(kSmoothThreads), 0, s, tmp, out, n1, n2, w);
    return hipGetLastError();
}

}  // namespace ecc
