// ecc_kernels.hip -- the histogram kernels of the ECC library for one image (2D
// and 3D) and their launchers.  The method and its mapping to the hardware are
// described in ecc_device.h; the min/max pass and the merge are in
// ecc_reduce.hip.
#include <map>
#include <mutex>
#include <tuple>

#include <hip/hip_ext.h>

#include "ecc_device.h"

namespace ecc {

namespace {

using namespace dev;

// 3D images.  A workgroup brick is a contiguous x-chunk (the workgroup's waves
// side by side, each 64 lanes wide with 63 owned) x kRows3 rows x L.depth planes.
// All waves of a workgroup read the same rows at about the same time, so every
// plane step of a workgroup reads whole row segments of memory.
template <int DT, int CONS, bool WIN, bool PAIR>
__global__ __launch_bounds__(kMaxWaves * 64) __attribute__((amdgpu_waves_per_eu(ECC_WAVES_PER_EU_3D))) void k_ecc_3d(EccLaunch L)
{
    extern __shared__ __align__(16) int32_t hist[];
    const BinParams P = load_params<DT>(L);
    const HistRef H = hist_ref(hist, L.bin_lo, L.width, L.hist_stride, L.sentinel, L.hist_copies);
    zero_hist(H, L.width);
    const int waves = (int)(blockDim.x >> 6);
    const int64_t chunk = (int64_t)waves * kLaneCols;
    // per plane block: the ordinary bricks (x-chunk fastest), then the packed
    // tail bricks, then the tails of the strips not packed (Layout3)
    const Layout3 Y = layout_3d(L.g, CONS, waves);
    const uint32_t nxc = (uint32_t)Y.nxc, nyb = (uint32_t)Y.nyb, per_z = (uint32_t)Y.per_z;
    const uint32_t main = nxc * nyb, npk = (uint32_t)Y.npk, sa = (uint32_t)Y.sa, sb = (uint32_t)Y.sb;
    const uint32_t nzb = (uint32_t)((L.z_own + L.depth - 1) / L.depth);
    const uint32_t nbricks = per_z * nzb;
    for (uint32_t brick = blockIdx.x; brick < nbricks; brick += gridDim.x) {
        const uint32_t zb = brick / per_z, r = brick - zb * per_z;
        Brick3 B;
        if (r < main) {
            B = chunk_brick_3d<DT, CONS, WIN>(L, H, chunk, r % nxc, r / nxc, zb, wave_id());
        } else if (r - main < npk) {
            B = tail_brick_3d<DT, CONS, WIN>(L, H, Y, waves, r - main, zb, wave_id());
        } else {
            const uint32_t e = r - main - npk;   // the strips before sa, then those from sb on
            B = chunk_brick_3d<DT, CONS, WIN>(L, H, chunk, nxc, e < sa ? e : sb + (e - sa), zb, wave_id());
        }
        run_brick3<DT, CONS, WIN, PAIR>(L, P, H, B);
    }
    flush_hist(H, L.partials + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * (size_t)L.width, L.width, L.flush_add != 0, L.flush_sign);
    if (L.fused) fused_merge_scan(hist, L.partials, L.width, L.out, L.counter + 1);
}

// 2D images.  A workgroup brick is a contiguous x-chunk x L.depth rows.
template <int DT, int CONS, bool WIN>
__global__ __launch_bounds__(kMaxWaves * 64) __attribute__((amdgpu_waves_per_eu(ECC_WAVES_PER_EU_2D))) void k_ecc_2d(EccLaunch L)
{
    extern __shared__ __align__(16) int32_t hist[];
    const BinParams P = L.params_dev ? *L.params_dev : L.params;
    const HistRef H = hist_ref(hist, L.bin_lo, L.width, L.hist_stride, L.sentinel, L.hist_copies);
    zero_hist(H, L.width);
    const int64_t chunk = (int64_t)(blockDim.x >> 6) * kLaneCols;
    const uint32_t nxc = (uint32_t)((axis_positions(L.g.n2, CONS) + chunk - 1) / chunk);
    const uint32_t nyb = (uint32_t)((L.g.n1 + L.depth - 1) / L.depth);
    const uint32_t nbricks = nxc * nyb;
    for (uint32_t brick = blockIdx.x; brick < nbricks; brick += gridDim.x)
        run_brick_2d<DT, CONS, WIN>(L, P, H, chunk, brick % nxc, brick / nxc, wave_id());
    flush_hist(H, L.partials + (size_t)blockIdx.x * (size_t)L.width, L.width, L.flush_add != 0, L.flush_sign);
    if (L.fused) fused_merge_scan(hist, L.partials, L.width, L.out, L.counter + 1);
}

}  // namespace

// ----------------------------------------------------------------- launchers


int64_t wg_bricks(int ndim, int construction, const Geom& g, int waves, int64_t depth)
{
    const int64_t chunk = (int64_t)waves * kLaneCols;
    const int64_t nxc = (axis_positions(g.n2, construction) + chunk - 1) / chunk;
    if (ndim == 2) return nxc * ((g.n1 + depth - 1) / depth);
    return layout_3d(g, construction, waves).per_z * ((g.n0 + depth - 1) / depth);
}

template <class K>
static hipError_t launch_k(K kernel, const EccLaunch& L, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    const dim3 grid((unsigned)L.grid, (unsigned)(L.npass > 1 ? L.npass : 1));
    if (t0 || t1)
        hipExtLaunchKernelGGL(kernel, grid, dim3(L.waves * 64), L.lds_bytes, s, t0, t1, 0, L);
    else
        hipLaunchKernelGGL(kernel, grid, dim3(L.waves * 64), L.lds_bytes, s, L);
    return hipGetLastError();
}

template <int NDIM, int DT, int CONS, bool WIN>
static hipError_t launch_t(const EccLaunch& L, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    if constexpr (NDIM == 2) return launch_k(k_ecc_2d<DT, CONS, WIN>, L, s, t0, t1);
    else if (L.data2) return launch_k(k_ecc_3d<DT, CONS, WIN, true>, L, s, t0, t1);
    else return launch_k(k_ecc_3d<DT, CONS, WIN, false>, L, s, t0, t1);
}

template <int NDIM, int DT, int CONS>
static hipError_t launch_w(const EccLaunch& L, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    return L.windowed ? launch_t<NDIM, DT, CONS, true>(L, s, t0, t1) : launch_t<NDIM, DT, CONS, false>(L, s, t0, t1);
}

template <int NDIM, int DT>
static hipError_t launch_c(const EccLaunch& L, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    return L.construction == CONS_TOP ? launch_w<NDIM, DT, CONS_TOP>(L, s, t0, t1)
                                      : launch_w<NDIM, DT, CONS_VERTEX>(L, s, t0, t1);
}

template <int NDIM>
static hipError_t launch_d(const EccLaunch& L, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    switch (L.dtype) {
    case DT_U8: return launch_c<NDIM, DT_U8>(L, s, t0, t1);
    case DT_U16: return launch_c<NDIM, DT_U16>(L, s, t0, t1);
    default: return launch_c<NDIM, DT_F32>(L, s, t0, t1);
    }
}

hipError_t launch_ecc(const EccLaunch& L, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    return L.ndim == 2 ? launch_d<2>(L, s, t0, t1) : launch_d<3>(L, s, t0, t1);
}

template <int NDIM, int DT, int CONS, bool WIN>
static const void* kernel_of()
{
    if constexpr (NDIM == 2) return (const void*)k_ecc_2d<DT, CONS, WIN>;
    else return (const void*)k_ecc_3d<DT, CONS, WIN, false>;
}

template <int NDIM, int DT, int CONS>
static const void* kernel_w(bool win)
{
    return win ? kernel_of<NDIM, DT, CONS, true>() : kernel_of<NDIM, DT, CONS, false>();
}

template <int NDIM, int DT>
static const void* kernel_c(int cons, bool win)
{
    return cons == CONS_TOP ? kernel_w<NDIM, DT, CONS_TOP>(win) : kernel_w<NDIM, DT, CONS_VERTEX>(win);
}

template <int NDIM>
static const void* kernel_d(int dtype, int cons, bool win)
{
    switch (dtype) {
    case DT_U8: return kernel_c<NDIM, DT_U8>(cons, win);
    case DT_U16: return kernel_c<NDIM, DT_U16>(cons, win);
    default: return kernel_c<NDIM, DT_F32>(cons, win);
    }
}

int resident_wgs_per_cu(int ndim, int dtype, int construction, bool windowed, int waves, uint32_t lds_bytes)
{
    // the answer only depends on the LDS in steps of the allocation granule
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, uint32_t>, int> cache;
    const uint32_t lds = (lds_bytes + 511u) / 512u * 512u;
    const auto key = std::make_tuple(ndim == 3, dtype, construction == CONS_TOP, windowed ? 1 : 0, waves, lds);
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    const void* k = ndim == 2 ? kernel_d<2>(dtype, construction, windowed) : kernel_d<3>(dtype, construction, windowed);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, waves * 64, lds) != hipSuccess || n < 1) n = 1;
    cache[key] = n;
    return n;
}


}  // namespace ecc
