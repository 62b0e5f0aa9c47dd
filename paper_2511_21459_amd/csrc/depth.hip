// RGB-D fusion of one map (Sec. 3.1 "Cameras", Eq. 2; Eq. 3, Eq. 5; Sec. 3.2.1).
//
// One frame is two launches on the map's stream: k_alloc_depth (pixel tiles, then cull
// workgroups; the last one also runs the allocation-side frame hand-off) and k_integrate_depth
// (update tasks over the per-level queues; workgroup 0 also runs the update-side hand-off).
#include <algorithm>
#include <cmath>
#include <mutex>

#include "mrh_depth.h"

namespace mrh {


// Frame sizes the kernels accept: pixel indices are 32-bit and pixel coordinates exact in FP32.
bool depth_size_ok(int32_t width, int32_t height) {
    return width > 0 && height > 0 && width < (1 << 24) && height < (1 << 24) &&
           (int64_t)width * (int64_t)height <= (int64_t)INT32_MAX;
}

// Point the frame at the map's tile-maximum buffer, growing it when the frame has more tiles.
mrh_status attach_tiles(mrh_map* map, int32_t width, int32_t height, DepthFrame& f) {
    f.tiles_x = (width + 15) / 16;
    f.tiles_y = (height + 15) / 16;
    const size_t need = (size_t)f.tiles_x * (size_t)f.tiles_y;
    if (need > map->tile_cap) {
        if (map->tile_max) {
            mrh_status st = check_hip(map, hipStreamSynchronize(map->stream), "tile buffer");
            if (st != MRH_OK) return st;
            (void)hipFree(map->tile_max);
            map->tile_max = nullptr;
            map->tile_cap = 0;
        }
        mrh_status st = check_hip(map, hipMalloc((void**)&map->tile_max, need * sizeof(float)), "tile buffer");
        if (st != MRH_OK) return st;
        map->tile_cap = need;
    }
    f.tile_max = map->tile_max;
    return MRH_OK;
}

bool make_depth_frame(const mrh_config& cfg, const float* depth, int32_t width, int32_t height, const double K[4],
                      const double T_ws[16], DepthFrame& f) {
    if (!pose_from(T_ws, f.P)) return false;
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(K[i])) return false;
    if (K[0] == 0.0 || K[1] == 0.0) return false;
    f.fx = K[0];
    f.fy = K[1];
    f.cx = K[2];
    f.cy = K[3];
    f.ifx = 1.0 / f.fx;
    f.ify = 1.0 / f.fy;
    f.width = width;
    f.height = height;
    f.depth = depth;
    f.fxf = (float)f.fx;
    f.fyf = (float)f.fy;
    f.cxf = (float)f.cx;
    f.cyf = (float)f.cy;
    // side planes of the pixel frustum u in [-1/2, W - 1/2), v in [-1/2, H - 1/2) (camera frame),
    // and the largest ray length factor over the image for the range bound
    const double al = (-0.5 - f.cx) / f.fx, ar = ((double)width - 0.5 - f.cx) / f.fx;
    const double at = (-0.5 - f.cy) / f.fy, ab = ((double)height - 0.5 - f.cy) / f.fy;
    const double lo_x = std::min(al, ar), hi_x = std::max(al, ar), lo_y = std::min(at, ab), hi_y = std::max(at, ab);
    auto set_plane = [&](int p, double a0, double a1, double a2) {
        const double nrm = std::sqrt(a0 * a0 + a1 * a1 + a2 * a2);
        f.plane[p][0] = a0 / nrm;
        f.plane[p][1] = a1 / nrm;
        f.plane[p][2] = a2 / nrm;
    };
    set_plane(0, 1.0, 0.0, -lo_x);
    set_plane(1, -1.0, 0.0, hi_x);
    set_plane(2, 0.0, 1.0, -lo_y);
    set_plane(3, 0.0, -1.0, hi_y);
    double lam = 1.0;
    for (double xx : {lo_x, hi_x})
        for (double yy : {lo_y, hi_y}) lam = std::max(lam, std::sqrt(1.0 + xx * xx + yy * yy));
    f.cull_range = lam * (cfg.max_depth + cfg.tau) * (1.0 + 1e-9) + 1e-6;
    return true;
}

// Workgroups [0, tiles): pixel tiles; [tiles, gridDim): cull.
__global__ __launch_bounds__(256) void k_alloc_depth(const DevMap* __restrict__ pm, DepthFrame f, uint32_t tiles_x, uint32_t tiles) {
    const DevMap& m = *pm;
    if (blockIdx.x == gridDim.x - 1) alloc_duties(m, f.parity);
    if (blockIdx.x >= tiles) depth_cull(m, f, blockIdx.x - tiles, gridDim.x - tiles);
    else depth_alloc_tile(m, f, blockIdx.x, tiles_x);
}

template <int ST>
__global__ __launch_bounds__(256) void k_integrate_depth(const DevMap* __restrict__ pm, DepthFrame f) {
    const DevMap& m = *pm;
    const uint32_t wave = uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    if (blockIdx.x == 0) update_duties(m, f.parity);
    const TaskCounts n = frame_task_counts(m, true, f.parity);
    const uint32_t ntask = update_task_count(n);
    TaskStats ts;
    for (uint32_t t = wave; t < ntask; t += nwaves) ts.add(depth_update_task<ST>(m, f, t, n));
    flush_task_stats(m, ts, true);
}

}  // namespace mrh

using namespace mrh;

namespace mrh {
// The two launches of one RGB-D frame; the frame descriptor is returned for a launch that follows
// on the same frame (colour).
mrh_status integrate_depth_frame(mrh_map* map, const float* depth_dev, int32_t width, int32_t height,
                                 const double K[4], const double T_ws[16], DepthFrame* frame_out) {
    if (!map || !depth_dev || !K || !T_ws || !depth_size_ok(width, height)) return MRH_ERR_INVALID_ARG;
    DepthFrame f;
    if (!make_depth_frame(map->cfg, depth_dev, width, height, K, T_ws, f))
        return set_error(map, MRH_ERR_INVALID_ARG, "non-finite pose or intrinsics, or zero focal length");
    const mrh_status ts = attach_tiles(map, width, height, f);
    if (ts != MRH_OK) return ts;
    f.parity = (int32_t)(map->frames & 1u);
    map->frames += 1;
    const uint32_t tiles_x = (uint32_t)(width + 15) / 16, tiles = tiles_x * (uint32_t)((height + 15) / 16);
    const uint32_t cull_groups = 128;
    launch(map, K_ALLOC_DEPTH, [&] {
        hipLaunchKernelGGL(k_alloc_depth, dim3(tiles + cull_groups), dim3(256), 0, map->stream, map->dmd, f, tiles_x,
                           tiles);
    });
    launch(map, K_INTEGRATE_DEPTH, [&] {
        const dim3 g(1024), b(256);
        switch (map->cfg.storage) {
            case MRH_STORE_F16: hipLaunchKernelGGL(k_integrate_depth<MRH_STORE_F16>, g, b, 0, map->stream, map->dmd, f); break;
            case MRH_STORE_BF16: hipLaunchKernelGGL(k_integrate_depth<MRH_STORE_BF16>, g, b, 0, map->stream, map->dmd, f); break;
            default: hipLaunchKernelGGL(k_integrate_depth<MRH_STORE_F32>, g, b, 0, map->stream, map->dmd, f);
        }
    });
    if (frame_out) *frame_out = f;
    return check_hip(map, hipGetLastError(), "integrate_depth");
}
}  // namespace mrh

extern "C" mrh_status mrh_integrate_depth(mrh_map* map, const float* depth_dev, int32_t width, int32_t height,
                                          const double K[4], const double T_ws[16]) {
    if (map && map->cfg.color)
        return set_error(map, MRH_ERR_INVALID_ARG, "a map with colour fuses RGB-D frames through mrh_integrate_rgbd");
    return integrate_depth_frame(map, depth_dev, width, height, K, T_ws, nullptr);
}

// ---- the variant that allocates nothing ------------------------------------------------------
// The per-tile depth summary lives in a fixed device array instead of the map's growable buffer.
// Each GPU holds its own copy for the life of the process; its address is looked up once per
// device (the array's name is not a device address in host code).
namespace mrh {
constexpr size_t kScratchTiles = 65536;  // 16 x 16 pixel tiles: frames of up to 4096 x 4096 pixels
constexpr int kScratchDevices = 64;
}  // namespace mrh

static __device__ __align__(256) float scratch[mrh::kScratchTiles];

static float* g_scratch_ptr[mrh::kScratchDevices];
static std::once_flag g_scratch_once[mrh::kScratchDevices];
static hipError_t g_scratch_err[mrh::kScratchDevices];

// Device address of `scratch` on `device`, resolved with that device current (once per device).
static hipError_t scratch_address(int device, float** out) {
    if (device < 0 || device >= mrh::kScratchDevices) return hipErrorInvalidDevice;
    std::call_once(g_scratch_once[device], [device] {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess && prev != device) e = hipSetDevice(device);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess) g_scratch_ptr[device] = static_cast<float*>(p);
        if (prev != device) (void)hipSetDevice(prev);
        g_scratch_err[device] = e;
    });
    *out = g_scratch_ptr[device];
    return g_scratch_err[device];
}

extern "C" mrh_status mrh_integrate_depth_noalloc(mrh_map* map, const float* depth_dev, int32_t width, int32_t height,
                                                  const double K[4], const double T_ws[16]) {
    if (!map || !depth_dev || !K || !T_ws || !depth_size_ok(width, height)) return MRH_ERR_INVALID_ARG;
    if (map->cfg.color)
        return set_error(map, MRH_ERR_INVALID_ARG, "a map with colour fuses RGB-D frames through mrh_integrate_rgbd");
    const size_t tiles_need = (size_t)((width + 15) / 16) * (size_t)((height + 15) / 16);
    if (tiles_need > kScratchTiles)
        return set_error(map, MRH_ERR_INVALID_ARG, "frame of %d x %d pixels has %zu tiles; the no-allocation entry point "
                         "takes at most %zu (4096 x 4096 pixels)", width, height, tiles_need, kScratchTiles);
    DepthFrame f;
    if (!make_depth_frame(map->cfg, depth_dev, width, height, K, T_ws, f))
        return set_error(map, MRH_ERR_INVALID_ARG, "non-finite pose or intrinsics, or zero focal length");
    float* tiles_dev = nullptr;
    const mrh_status sa = check_hip(map, scratch_address(map->device, &tiles_dev), "scratch address");
    if (sa != MRH_OK) return sa;
    f.tiles_x = (width + 15) / 16;
    f.tiles_y = (height + 15) / 16;
    f.tile_max = tiles_dev;
    f.parity = (int32_t)(map->frames & 1u);
    map->frames += 1;
    const uint32_t tiles_x = (uint32_t)f.tiles_x, tiles = (uint32_t)tiles_need;
    const uint32_t cull_groups = 128;
    // launched directly: the launch profiler's events are created on demand, which allocates
    hipLaunchKernelGGL(k_alloc_depth, dim3(tiles + cull_groups), dim3(256), 0, map->stream, map->dmd, f, tiles_x, tiles);
    const dim3 g(1024), b(256);
    switch (map->cfg.storage) {
        case MRH_STORE_F16: hipLaunchKernelGGL(k_integrate_depth<MRH_STORE_F16>, g, b, 0, map->stream, map->dmd, f); break;
        case MRH_STORE_BF16: hipLaunchKernelGGL(k_integrate_depth<MRH_STORE_BF16>, g, b, 0, map->stream, map->dmd, f); break;
        default: hipLaunchKernelGGL(k_integrate_depth<MRH_STORE_F32>, g, b, 0, map->stream, map->dmd, f);
    }
    return check_hip(map, hipGetLastError(), "integrate_depth_noalloc");
}

extern "C" mrh_status mrh_integrate_depth_sequence(mrh_map* map, const float* depth_dev, int32_t n_frames, int32_t width,
                                                   int32_t height, const double K[4], const double* T_ws) {
    if (!map || !depth_dev || !K || !T_ws || n_frames < 0 || !depth_size_ok(width, height)) return MRH_ERR_INVALID_ARG;
    DepthFrame f;
    for (int32_t k = 0; k < n_frames; ++k)
        if (!make_depth_frame(map->cfg, depth_dev, width, height, K, T_ws + 16 * k, f))
            return set_error(map, MRH_ERR_INVALID_ARG, "frame %d: non-finite pose or intrinsics", k);
    const size_t pix = (size_t)width * (size_t)height;
    for (int32_t k = 0; k < n_frames; ++k) {
        const mrh_status st = mrh_integrate_depth(map, depth_dev + pix * (size_t)k, width, height, K, T_ws + 16 * k);
        if (st != MRH_OK) return st;
    }
    return MRH_OK;
}
