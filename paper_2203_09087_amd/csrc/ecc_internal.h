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
//   integer data: a = clamp(v, ilo, ihi) - ilo ; bin = a*q0 + floor(a*r/D) with
//                 D = ihi-ilo+1, nbins = q0*D + r, the second term computed
//                 exactly as umulhi(a, magic), magic = floor(r*2^32/D) + 1
//                 (exact because a*D < 2^32);
//   float data:   NaN -> nbins-1; flat range -> (x > hi ? nbins-1 : 0);
//                 otherwise clamp(floor(((double)x - lo) * scale), 0, nbins-1).
struct BinParams {
    int32_t dtype;
    int32_t nbins;
    uint32_t ilo, ihi, q0, magic;
    int32_t flat;
    int32_t pad;
    double lo, hi, scale;
};

// Geometry of one image: n[0] slowest.  For 2D images n[0] is 1.
struct Geom {
    int64_t n0, n1, n2;
};

// Histogram window: bins [bin_lo, bin_lo + width) are accumulated in LDS.
constexpr int kMaxLdsBins = 8192;

struct HistLaunch {
    const void* data;
    int ndim, dtype, construction;
    Geom g;
    const BinParams* params_dev;   // non-null: read the parameters from device memory
    BinParams params;              // used when params_dev is null
    int32_t bin_lo, width;
    int32_t* partials;             // [grid][width]
    int grid;                      // number of workgroups
};

// Launchers (ecc_kernels.hip).  All enqueue on `s` and return the launch status.
hipError_t launch_minmax(const void* data, int dtype, int64_t nvox, uint32_t* mm_out, int blocks,
                         hipStream_t s);
hipError_t launch_params_from_minmax(const uint32_t* mm, int blocks, int dtype, int32_t nbins,
                                     BinParams* out, hipStream_t s);
hipError_t launch_hist(const HistLaunch& L, hipStream_t s);
hipError_t launch_reduce(const int32_t* partials, int grid, int32_t width, int64_t* out_window,
                         hipStream_t s);
hipError_t launch_scan(int64_t* out, int32_t nbins, hipStream_t s);

int64_t hist_tiles(int ndim, const Geom& g);

}  // namespace ecc
