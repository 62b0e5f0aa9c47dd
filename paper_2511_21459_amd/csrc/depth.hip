// RGB-D fusion (Sec. 3.1 "Cameras", Eq. 2; Eq. 3 and Eq. 5; Sec. 3.2.1 merging criterion).
//
// One frame is three launches on the map's stream:
//   k_alloc_depth      pixel workgroups: back-projection, band walk over the block lattice, lookup,
//                      wave-deduplicated lock-free insert, ballot/prefix-sum ids and heap slots for
//                      new blocks (queued for the update); cull workgroups: one thread per block
//                      that existed at the frame's start, conservative frustum test, visible blocks
//                      queued per level
//   k_integrate_depth  one task per queued level-0 or level-1 block (a wave), 8 level-2 or 64
//                      level-3 blocks per wave: per-voxel projection and update, block variance
//                      bookkeeping and the merge of a block whose mean variance fell below the
//                      threshold
//   k_finalize         freed slots back to their stacks, statistics
#include <cmath>

#include "mrh_update.h"

namespace mrh {

void launch_finalize(mrh_map* m);

struct DepthFrame {
    Pose P;
    double fx, fy, cx, cy, ifx, ify;
    int32_t width, height;
    // conservative culling of whole blocks (camera frame): side-plane normals and a range bound
    double plane[4][3];
    double cull_range;
};

// ---------------------------------------------------------------------------------------------
// allocation
// ---------------------------------------------------------------------------------------------

__device__ inline bool block_visible(const DevMap& m, const DepthFrame& f, int64_t bx, int64_t by, int64_t bz);

// Workgroups [0, tiles): 16 x 16 pixel tiles, each wave a 16 x 4 strip (good key reuse).
// Workgroups [tiles, gridDim): one thread per block that existed at the frame's start.
__global__ __launch_bounds__(256) void k_alloc_depth(DevMap m, DepthFrame f, const float* __restrict__ depth,
                                                     uint32_t tiles_x, uint32_t tiles) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    if (blockIdx.x >= tiles) {
        // conservative frustum cull of the existing blocks
        const uint32_t n = m.ctr->n_prev;
        const uint32_t stride = (gridDim.x - tiles) * blockDim.x;
        for (uint32_t base = (blockIdx.x - tiles) * blockDim.x; base < n; base += stride) {
            const uint32_t id = base + threadIdx.x;
            int level = -1;
            if (id < n) {
                const uint32_t info = m.binfo[id];
                if (!(info & kNoBlockBit)) {
                    int32_t bx, by, bz;
                    unpack_key(m.bkey[id], bx, by, bz);
                    if ((info & kNewBit) || block_visible(m, f, bx, by, bz)) level = (int)((info >> kLevelShift) & 3u);
                }
            }
            for (int lv = 0; lv < 4; ++lv) {
                const unsigned long long msk = __ballot(level == lv);
                if (!msk) continue;
                const int f0 = __ffsll((long long)msk) - 1;
                uint32_t vb = 0;
                if (lane == f0) vb = atomicAdd(&m.ctr->vis_n[lv], (uint32_t)__popcll(msk));
                vb = (uint32_t)__shfl((int)vb, f0);
                if (level == lv) m.vis[lv][vb + rank_in_mask(msk)] = id;
            }
        }
        return;
    }
    const int u = (blockIdx.x % tiles_x) * 16 + (lane & 15);
    const int v = (blockIdx.x / tiles_x) * 16 + wave * 4 + (lane >> 4);
    bool ok = u < f.width && v < f.height;
    double d = 0.0;
    if (ok) {
        d = (double)depth[(int64_t)v * f.width + u];
        ok = __builtin_isfinite(d) && d > 0.0 && d <= m.max_depth;
    }
    Walk w;
    bool in_range = false;
    if (ok) {
        // back-projection of the pixel centre and the truncation band along the sensor ray
        const double ps[3] = {(((double)u - f.cx) * f.ifx) * d, (((double)v - f.cy) * f.ify) * d, d};
        double pw[3], n[3];
        pose_apply(f.P, ps, pw);
        unit_direction(pw, f.P.t, n);
        const double a[3] = {pw[0] - m.tau * n[0], pw[1] - m.tau * n[1], pw[2] - m.tau * n[2]};
        const double e[3] = {pw[0] + m.tau * n[0], pw[1] + m.tau * n[1], pw[2] + m.tau * n[2]};
        in_range = segment_in_range(a, e, m.invB);
        if (in_range) w.init(a, e, m.invB);
    }
    __shared__ uint32_t cnt[2];
    if (threadIdx.x == 0) cnt[0] = cnt[1] = 0;
    __syncthreads();
    const unsigned long long vmask = __ballot(ok), dmask = __ballot(ok && !in_range);
    if (lane == 0) {
        atomicAdd(&cnt[0], (uint32_t)__popcll(vmask));
        atomicAdd(&cnt[1], (uint32_t)__popcll(dmask));
    }
    bool active = in_range;
    while (__ballot(active)) {
        const unsigned long long key = active ? pack_key(w.c0, w.c1, w.c2) : 0ull;
        insert_keys(m, active, key, true);
        if (active) active = w.next();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        stat_add(m, S_VALID, cnt[0]);
        stat_add(m, S_DROPPED, cnt[1]);
    }
}

// ---------------------------------------------------------------------------------------------
// projective update
// ---------------------------------------------------------------------------------------------

// Observation for the voxel whose camera-frame centre is x (Eq. 2 with the gate at -tau and
// truncation at +tau).  Returns false when the voxel is not updated.
__device__ inline bool project_observe(const DevMap& m, const DepthFrame& f, const float* __restrict__ depth,
                                       double x0, double x1, double x2, float& obs) {
    if (!(x2 > 0.0)) return false;
    const double iz = 1.0 / x2;
    const double uu = (f.fx * (x0 * iz)) + f.cx;
    const double vv = (f.fy * (x1 * iz)) + f.cy;
    const double fu = __builtin_floor(uu + 0.5), fv = __builtin_floor(vv + 0.5);
    if (!(fu >= 0.0 && fu <= (double)(f.width - 1) && fv >= 0.0 && fv <= (double)(f.height - 1))) return false;
    const double d = (double)depth[(int64_t)fv * f.width + (int64_t)fu];
    if (!(__builtin_isfinite(d) && d > 0.0 && d <= m.max_depth)) return false;
    double raw;
    if (m.form == MRH_FORM_RANGE) {
        const double nx = __builtin_sqrt((x0 * x0 + x1 * x1) + x2 * x2);
        raw = nx * ((d * iz) - 1.0);
    } else {
        raw = d - x2;
    }
    if (raw < -m.tau) return false;
    obs = (float)(raw < m.tau ? raw : m.tau);
    return true;
}

__device__ inline bool block_visible(const DevMap& m, const DepthFrame& f, int64_t bx, int64_t by, int64_t bz) {
    const double hb = 0.5 * m.B;
    const double c[3] = {(double)bx * m.B + hb, (double)by * m.B + hb, (double)bz * m.B + hb};
    const double d0 = c[0] - f.P.t[0], d1 = c[1] - f.P.t[1], d2 = c[2] - f.P.t[2];
    double x[3];
    for (int r = 0; r < 3; ++r) x[r] = (f.P.R[0][r] * d0 + f.P.R[1][r] * d1) + f.P.R[2][r] * d2;
    const double rb = m.B * 0.8660254037844387 * (1.0 + 1e-9) + 1e-9;
    if (x[2] < -rb) return false;
    if (__builtin_sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) - rb > f.cull_range) return false;
    for (int p = 0; p < 4; ++p)
        if (f.plane[p][0] * x[0] + f.plane[p][1] * x[1] + f.plane[p][2] * x[2] < -rb) return false;
    return true;
}

// Statistics gathered by one wave over its tasks: obs / fresh / merges[0..1] are wave-uniform,
// lane_obs / lane_merges (packed blocks) are per lane.
struct TaskStats {
    unsigned long long obs = 0, fresh = 0, merges[2] = {0, 0}, lane_obs = 0, lane_merges = 0;
};

// Level-0 block: lane l owns the 2x2x2 group of Morton positions 8l .. 8l+7.
__device__ inline void integrate_fine_block(const DevMap& m, const DepthFrame& f, const float* __restrict__ depth,
                                            uint32_t id, TaskStats& ts) {
    const int lane = lane_id();
    const uint32_t info = m.binfo[id];
    int32_t bx, by, bz;
    unpack_key(m.bkey[id], bx, by, bz);
    const bool fresh = (info & kNewBit) != 0;
    int I, J, K;
    demorton3(lane, I, J, K);
    const double nu = m.nu[0];
    // camera-frame products of R^T (c - t), one per axis coordinate of this lane's group
    double px[2][3], py[2][3], pz[2][3];
    for (int s = 0; s < 2; ++s) {
        const double cx = (double)bx * m.B + ((double)(2 * I + s) + 0.5) * nu;
        const double cy = (double)by * m.B + ((double)(2 * J + s) + 0.5) * nu;
        const double cz = (double)bz * m.B + ((double)(2 * K + s) + 0.5) * nu;
        const double dx = cx - f.P.t[0], dy = cy - f.P.t[1], dz = cz - f.P.t[2];
        for (int r = 0; r < 3; ++r) {
            px[s][r] = f.P.R[0][r] * dx;
            py[s][r] = f.P.R[1][r] * dy;
            pz[s][r] = f.P.R[2][r] * dz;
        }
    }
    float obs[8];
    uint32_t upd = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int a = q & 1, b = (q >> 1) & 1, c = (q >> 2) & 1;
        const double x0 = (px[a][0] + py[b][0]) + pz[c][0];
        const double x1 = (px[a][1] + py[b][1]) + pz[c][1];
        const double x2 = (px[a][2] + py[b][2]) + pz[c][2];
        if (project_observe(m, f, depth, x0, x1, x2, obs[q])) upd |= 1u << q;
    }
    const int nupd = wave_sum((int)__popc(upd));
    if (nupd == 0 && !fresh) return;
    ts.obs += (unsigned long long)nupd;
    if (fresh) ts.fresh += (unsigned long long)nupd;

    const size_t base = (size_t)(info & kSlotMask) * 512 + (size_t)lane * 8;
    float D[8], S2[8];
    uint32_t W[8];
    bool have = false;
    if (fresh) {
        for (int q = 0; q < 8; ++q) D[q] = 0.f, S2[q] = 0.f, W[q] = 0u;
        have = true;
    } else if (upd) {
        load_group(m, base, D, W, S2);
        have = true;
    }
    double dsum = 0.0;
    int dcnt = 0;
    for (int q = 0; q < 8; ++q) {
        if (!(upd & (1u << q))) continue;
        const double before = var_term(m, W[q], S2[q]);
        const int cb = var_count(m, W[q]);
        welford(obs[q], D[q], W[q], S2[q]);
        dsum += var_term(m, W[q], S2[q]) - before;
        dcnt += var_count(m, W[q]) - cb;
    }
    ts.merges[0] += (unsigned long long)finish_fine(m, id, info, D, W, S2, have, upd != 0 || fresh, nupd, dsum, dcnt);
}

// Camera-frame centre of voxel (i, j, k) of block b at `level`, canonical FP64.
__device__ inline void voxel_camera(const DevMap& m, const DepthFrame& f, int64_t bx, int64_t by, int64_t bz, int level,
                                    int i, int j, int k, double& x0, double& x1, double& x2) {
    const double nu = m.nu[level];
    const double c0 = (double)bx * m.B + ((double)i + 0.5) * nu;
    const double c1 = (double)by * m.B + ((double)j + 0.5) * nu;
    const double c2 = (double)bz * m.B + ((double)k + 0.5) * nu;
    const double d0 = c0 - f.P.t[0], d1 = c1 - f.P.t[1], d2 = c2 - f.P.t[2];
    x0 = (f.P.R[0][0] * d0 + f.P.R[1][0] * d1) + f.P.R[2][0] * d2;
    x1 = (f.P.R[0][1] * d0 + f.P.R[1][1] * d1) + f.P.R[2][1] * d2;
    x2 = (f.P.R[0][2] * d0 + f.P.R[1][2] * d1) + f.P.R[2][2] * d2;
}

// Level-1 block: lane l owns the voxel at Morton position l.
__device__ inline void integrate_level1_block(const DevMap& m, const DepthFrame& f, const float* __restrict__ depth,
                                              uint32_t id, TaskStats& ts) {
    const int lane = lane_id();
    const uint32_t info = m.binfo[id];
    int32_t bx, by, bz;
    unpack_key(m.bkey[id], bx, by, bz);
    int i, j, k;
    demorton3(lane, i, j, k);
    double x0, x1, x2;
    voxel_camera(m, f, bx, by, bz, 1, i, j, k, x0, x1, x2);
    float obs = 0.f;
    const bool upd = project_observe(m, f, depth, x0, x1, x2, obs);
    const int nupd = __popcll(__ballot(upd));
    if (nupd == 0) return;
    ts.obs += (unsigned long long)nupd;
    const size_t at = (size_t)(info & kSlotMask) * 64 + lane;
    float D = m.D[1][at], S2 = m.S2[1][at];
    uint32_t W = m.W[1][at];
    double dsum = 0.0;
    int dcnt = 0;
    if (upd) {
        const double before = var_term(m, W, S2);
        const int cb = var_count(m, W);
        welford(obs, D, W, S2);
        dsum = var_term(m, W, S2) - before;
        dcnt = var_count(m, W) - cb;
    }
    ts.merges[1] += (unsigned long long)finish_coarse(m, id, info, 1, D, W, S2, upd, nupd, dsum, dcnt);
}

// 64 / seg blocks of `level` (2: seg = 8 voxels, 3: seg = 1 voxel) per wave.
__device__ inline void integrate_packed_blocks(const DevMap& m, const DepthFrame& f, const float* __restrict__ depth,
                                               const uint32_t* list, uint32_t count, uint32_t group, int level,
                                               TaskStats& ts) {
    const int lane = lane_id();
    const int seg = level == 2 ? 8 : 1;
    const uint32_t bi = group * (uint32_t)(64 / seg) + (uint32_t)(lane / seg);
    const bool live = bi < count;
    uint32_t id = 0, info = 0;
    bool upd = false;
    float obs = 0.f;
    if (live) {
        id = list[bi];
        info = m.binfo[id];
        int32_t bx, by, bz;
        unpack_key(m.bkey[id], bx, by, bz);
        int i, j, k;
        demorton3(lane % seg, i, j, k);
        double x0, x1, x2;
        voxel_camera(m, f, bx, by, bz, level, i, j, k, x0, x1, x2);
        upd = project_observe(m, f, depth, x0, x1, x2, obs);
    }
    if (!__ballot(upd)) return;
    float D = 0.f, S2 = 0.f;
    uint32_t W = 0;
    double dsum = 0.0;
    int dcnt = 0;
    if (upd) {
        const size_t at = (size_t)(info & kSlotMask) * seg + (lane % seg);
        D = m.D[level][at];
        W = m.W[level][at];
        S2 = m.S2[level][at];
        ts.lane_obs += 1;
        const double before = var_term(m, W, S2);
        const int cb = var_count(m, W);
        welford(obs, D, W, S2);
        dsum = var_term(m, W, S2) - before;
        dcnt = var_count(m, W) - cb;
    } else if (live && seg > 1) {
        // a segment whose block merges needs all of its voxels
        const size_t at = (size_t)(info & kSlotMask) * seg + (lane % seg);
        D = m.D[level][at];
        W = m.W[level][at];
        S2 = m.S2[level][at];
    }
    ts.lane_merges += (unsigned long long)finish_packed(m, live, id, info, level, seg, D, W, S2, upd, upd ? 1 : 0, dsum,
                                                      dcnt);
}

__global__ __launch_bounds__(256) void k_integrate_depth(DevMap m, DepthFrame f, const float* __restrict__ depth) {
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    const uint32_t n0 = m.ctr->vis_n[0], n1 = m.ctr->vis_n[1], n2 = m.ctr->vis_n[2], n3 = m.ctr->vis_n[3];
    const uint32_t g2 = (n2 + 7) / 8, g3 = (n3 + 63) / 64;
    const uint32_t ntask = n0 + n1 + g2 + g3;
    TaskStats ts;
    for (uint32_t t = wave; t < ntask; t += nwaves) {
        if (t < n0) integrate_fine_block(m, f, depth, m.vis[0][t], ts);
        else if (t < n0 + n1) integrate_level1_block(m, f, depth, m.vis[1][t - n0], ts);
        else if (t < n0 + n1 + g2) integrate_packed_blocks(m, f, depth, m.vis[2], n2, t - n0 - n1, 2, ts);
        else integrate_packed_blocks(m, f, depth, m.vis[3], n3, t - n0 - n1 - g2, 3, ts);
    }
    const unsigned long long lane_obs = wave_sum(ts.lane_obs), lane_merges = wave_sum(ts.lane_merges);
    if (lane_id() == 0) {
        stat_add(m, S_OBS, ts.obs + lane_obs);
        stat_add(m, S_OBS_FRESH, ts.fresh);
        stat_add(m, S_MERGE0, ts.merges[0]);
        stat_add(m, S_MERGE1, ts.merges[1]);
        stat_add(m, S_MERGE2, lane_merges);
    }
}

}  // namespace mrh

using namespace mrh;

extern "C" mrh_status mrh_integrate_depth(mrh_map* map, const float* depth_dev, int32_t width, int32_t height,
                                          const double K[4], const double T_ws[16]) {
    if (!map || !depth_dev || !K || !T_ws || width <= 0 || height <= 0) return MRH_ERR_INVALID_ARG;
    DepthFrame f;
    if (!pose_from(T_ws, f.P)) return set_error(map, MRH_ERR_INVALID_ARG, "non-finite pose");
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(K[i])) return set_error(map, MRH_ERR_INVALID_ARG, "non-finite intrinsics");
    if (K[0] == 0.0 || K[1] == 0.0) return set_error(map, MRH_ERR_INVALID_ARG, "zero focal length");
    f.fx = K[0];
    f.fy = K[1];
    f.cx = K[2];
    f.cy = K[3];
    f.ifx = 1.0 / f.fx;
    f.ify = 1.0 / f.fy;
    f.width = width;
    f.height = height;
    // side planes of the pixel frustum u in [-1/2, W - 1/2), v in [-1/2, H - 1/2) (camera frame),
    // and the largest ray length factor over the image for the range bound
    const double al = (-0.5 - f.cx) / f.fx, ar = ((double)width - 0.5 - f.cx) / f.fx;
    const double at = (-0.5 - f.cy) / f.fy, ab = ((double)height - 0.5 - f.cy) / f.fy;
    const double lo_x = al < ar ? al : ar, hi_x = al < ar ? ar : al, lo_y = at < ab ? at : ab, hi_y = at < ab ? ab : at;
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
    f.cull_range = lam * (map->cfg.max_depth + map->cfg.tau) * (1.0 + 1e-9) + 1e-6;

    const uint32_t tiles_x = (uint32_t)(width + 15) / 16, tiles = tiles_x * (uint32_t)((height + 15) / 16);
    const uint32_t cull_groups = 128;
    launch(map, K_ALLOC_DEPTH, [&] {
        hipLaunchKernelGGL(k_alloc_depth, dim3(tiles + cull_groups), dim3(256), 0, map->stream, map->dm, f, depth_dev,
                           tiles_x, tiles);
    });
    launch(map, K_INTEGRATE_DEPTH, [&] {
        hipLaunchKernelGGL(k_integrate_depth, dim3(1024), dim3(256), 0, map->stream, map->dm, f, depth_dev);
    });
    launch_finalize(map);
    return check_hip(map, hipGetLastError(), "integrate_depth");
}
