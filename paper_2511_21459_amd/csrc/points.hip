// LiDAR fusion of one map (Sec. 3.1 "3D Point Cloud", Eq. 1; Eq. 3, Eq. 5; Sec. 3.2.1).
//
// One scan is four launches on the map's stream: k_alloc_points (its last workgroup also runs the
// allocation-side frame hand-off), k_rays, k_touch_queue (the touched blocks onto the per-level
// update queues) and k_apply_points (update tasks over those queues; workgroup 0 also runs the
// update-side hand-off).
#include <cmath>

#include "mrh_points.h"

namespace mrh {


__global__ __launch_bounds__(256) void k_alloc_points(const DevMap* __restrict__ pm, ScanParams sp) {
    if (blockIdx.x == gridDim.x - 1) alloc_duties(*pm, sp.parity);
    points_alloc_chunk(*pm, sp, blockIdx.x);
}

template <int ST>
__global__ __launch_bounds__(256) void k_rays(const DevMap* __restrict__ pm, ScanParams sp) {
    __shared__ unsigned long long tab[kSatSlots];
    points_ray_chunk<ST, false>(*pm, sp, blockIdx.x, tab);
}

// After the ray launch: the touched blocks onto the update queues (workgroup w takes block ids
// w * 256 * kTouchPerThread onwards).
__global__ __launch_bounds__(256) void k_touch_queue(const DevMap* __restrict__ pm, int par) {
    const DevMap& m = *pm;
    const uint32_t nb = min(m.ctr->n_blocks, m.max_blocks);
    const uint32_t per = blockDim.x * (uint32_t)kTouchPerThread;
    for (uint32_t first = blockIdx.x * per; first < nb; first += gridDim.x * per)
        queue_touched(m, first, min(per, nb - first), par);
}

template <int ST>
__global__ __launch_bounds__(256) void k_apply_points(const DevMap* __restrict__ pm, int par) {
    const DevMap& m = *pm;
    if (blockIdx.x == 0) update_duties(m, par);
    const uint32_t wave = uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const TaskCounts n = frame_task_counts(m, false, par);
    const uint32_t ntask = update_task_count(n);
    // merges of level-0 / level-1 blocks are recorded and done in batches (see run_deferred)
    __shared__ uint32_t dbuf[4][4 * kDefer];
    DeferList dl{dbuf[uniform(threadIdx.x >> 6)], 0u};
    unsigned long long m0 = 0, m1 = 0;
    TaskStats as;
    for (uint32_t t = wave; t < ntask; t += nwaves) {
        as.add_uniform(points_update_task<ST, true>(m, t, n, par, &dl));
        if (dl.full()) run_deferred<ST>(m, dl, par, m0, m1);
    }
    run_deferred<ST>(m, dl, par, m0, m1);
    as.merge0 += m0;
    as.merge1 += m1;
    flush_task_stats(m, as, false);
}

// Blocks a ray's walk can visit: the guard of the block walk bounds it by 4 + the sum over the
// axes of the cells the segment spans (carving: up to max_range + tau long; otherwise 2 tau).
static int32_t ray_block_cap(const mrh_config& c) {
    const double len = c.carve ? c.max_range + c.tau : 2.0 * c.tau;
    const double cells = 1.7320508075688772 * len / (8.0 * c.voxel) + 8.0;
    return cells < 1024.0 ? (int32_t)cells : 1024;
}

// LiDAR state of a map: accumulators (first scan) and per-ray block-key buffers for n rays.
mrh_status ensure_lidar(mrh_map* map, int64_t n) {
    DevMap& d = map->dm;
    mrh_status st = MRH_OK;
    bool changed = false;
    auto alloc = [&](void** p, size_t bytes, const char* what) {
        if (st != MRH_OK) return;
        st = check_hip(map, hipMalloc(p, bytes), what);
        if (st == MRH_OK) st = check_hip(map, hipMemsetAsync(*p, 0, bytes, map->stream), what);
        changed = true;
    };
    if (!map->lidar_ready) {
        alloc((void**)&d.btouch, (size_t)d.max_blocks * 8, "touch masks");
        for (int l = 0; l < map->cfg.levels; ++l) {
            const size_t nv = (size_t)d.heap_cap[l] * (size_t)(side_of(l) * side_of(l) * side_of(l));
            alloc((void**)&d.acc_sat[l], nv * 4, "scan accumulators");
            alloc((void**)&d.acc_band[l], nv * 4, "scan accumulators");
            alloc((void**)&d.acc_s1[l], nv * 8, "scan accumulators");
            alloc((void**)&d.acc_s2[l], nv * 8, "scan accumulators");
        }
        d.rcap_k = ray_block_cap(map->cfg);
        if (st == MRH_OK) map->lidar_ready = true;
    }
    if (st == MRH_OK && n > map->rcap_n) {
        st = check_hip(map, hipStreamSynchronize(map->stream), "ray buffers");
        if (d.rslots) (void)hipFree(d.rslots);
        if (d.rcount) (void)hipFree(d.rcount);
        d.rslots = nullptr;
        d.rcount = nullptr;
        map->rcap_n = 0;
        alloc((void**)&d.rslots, (size_t)n * (size_t)d.rcap_k * 4, "ray block slots");
        alloc((void**)&d.rcount, (size_t)n * 4, "ray block counts");
        if (st == MRH_OK) map->rcap_n = n;
    }
    if (st == MRH_OK && changed) st = upload_descriptor(map);
    return st;
}

}  // namespace mrh

using namespace mrh;

extern "C" mrh_status mrh_integrate_points(mrh_map* map, const float* xyz_dev, int64_t n, const double T_ws[16]) {
    if (!map || !T_ws || n < 0 || (n > 0 && !xyz_dev)) return MRH_ERR_INVALID_ARG;
    if (map->cfg.color) return set_error(map, MRH_ERR_INVALID_ARG, "a map with colour fuses RGB-D frames only");
    ScanParams sp;
    if (!pose_from(T_ws, sp.P)) return set_error(map, MRH_ERR_INVALID_ARG, "non-finite pose");
    sp.xyz = xyz_dev;
    sp.n = n;
    mrh_status st = ensure_lidar(map, n);
    if (st != MRH_OK) return st;
    sp.parity = (int32_t)(map->frames & 1u);
    map->frames += 1;
    const int par = sp.parity;
    // the allocation and update launches always run (they carry the frame hand-off)
    const unsigned agrid = n > 0 ? (unsigned)((n + kAllocRaysPerGroup - 1) / kAllocRaysPerGroup) : 1u;
    launch(map, K_ALLOC_POINTS,
           [&] { hipLaunchKernelGGL(k_alloc_points, dim3(agrid), dim3(256), 0, map->stream, map->dmd, sp); });
    if (n > 0) {
        const unsigned rgrid = (unsigned)((n + kRaysPerGroup - 1) / kRaysPerGroup);
        launch(map, K_RAYS, [&] {
            switch (map->cfg.storage) {
                case MRH_STORE_F16: hipLaunchKernelGGL(k_rays<MRH_STORE_F16>, dim3(rgrid), dim3(256), 0, map->stream, map->dmd, sp); break;
                case MRH_STORE_BF16: hipLaunchKernelGGL(k_rays<MRH_STORE_BF16>, dim3(rgrid), dim3(256), 0, map->stream, map->dmd, sp); break;
                default: hipLaunchKernelGGL(k_rays<MRH_STORE_F32>, dim3(rgrid), dim3(256), 0, map->stream, map->dmd, sp);
            }
            hipLaunchKernelGGL(k_touch_queue, dim3(1024), dim3(256), 0, map->stream, map->dmd, par);
        });
    }
    launch(map, K_APPLY_POINTS, [&] {
        const dim3 g(1024), b(256);
        switch (map->cfg.storage) {
            case MRH_STORE_F16: hipLaunchKernelGGL(k_apply_points<MRH_STORE_F16>, g, b, 0, map->stream, map->dmd, par); break;
            case MRH_STORE_BF16: hipLaunchKernelGGL(k_apply_points<MRH_STORE_BF16>, g, b, 0, map->stream, map->dmd, par); break;
            default: hipLaunchKernelGGL(k_apply_points<MRH_STORE_F32>, g, b, 0, map->stream, map->dmd, par);
        }
    });
    return check_hip(map, hipGetLastError(), "integrate_points");
}

extern "C" mrh_status mrh_integrate_points_sequence(mrh_map* map, const float* xyz_dev, int32_t n_frames, int64_t n,
                                                    const double* T_ws) {
    if (!map || !T_ws || n_frames < 0 || n < 0 || (n > 0 && !xyz_dev)) return MRH_ERR_INVALID_ARG;
    Pose P;
    for (int32_t k = 0; k < n_frames; ++k)
        if (!pose_from(T_ws + 16 * k, P)) return set_error(map, MRH_ERR_INVALID_ARG, "scan %d: non-finite pose", k);
    for (int32_t k = 0; k < n_frames; ++k) {
        const mrh_status st = mrh_integrate_points(map, xyz_dev + (size_t)3 * (size_t)n * (size_t)k, n, T_ws + 16 * k);
        if (st != MRH_OK) return st;
    }
    return MRH_OK;
}
