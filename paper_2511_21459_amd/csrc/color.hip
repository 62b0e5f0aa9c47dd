// Colour integration (Sec. 3: a voxel stores a colour), a standalone launch after a frame's depth
// update.
//
// For every block of the frame's update task space (the visible blocks queued by the cull, at their
// level when the frame started, and the frame's new blocks), every voxel takes the frame's
// projective decision again -- the same pixel and the same -tau gate as the update, so the same
// set of voxels -- and a voxel the frame updated averages the RGB value of its pixel into its
// colour, C <- C + (c - C) / W with the weight W after the update (Eq. 3 with w = 1).  A block the
// update merged one level coarser still holds its fine voxels (their slot is freed only for later
// frames) with the weights from before the frame: the colour is updated there with W + 1 and
// pooled into the coarse block as the weighted mean of the observed children, as the TSDF was.
// New blocks cannot merge in their first frame (no voxel reaches min_obs >= 2 observations).
#include <vector>

#include "mrh_depth.h"

namespace mrh {

// The update's decision for one voxel (camera-frame centre x), keeping the pixel index.
__device__ inline bool observe_pixel(const DevMap& m, const DepthFrame& f, double x0, double x1, double x2, int& p) {
    float lam, obs;
    p = pixel_fast(f, x0, x1, x2, lam);
    const bool exact = p == -2;
    if (exact) p = pixel_exact(f, x0, x1, x2);
    if (p < 0) return false;
    const float d = f.depth[p];
    if (!exact) {
        const int r = observe_fast(m, x2, lam, d, obs);
        if (r != 2) return r == 1;
    }
    return observe_exact(m, x0, x1, x2, (double)d, obs);
}

// A level-0 block (one wave; lane l owns the 2x2x2 group of Morton positions 8l .. 8l+7): the update's
// decisions for the group, the weights after the frame (W + 1 for an updated voxel of a block that
// merged, whose slot kept the values from before the frame), and the colours of the group, which
// are the 8 children of coarse voxel l when the block merged.
template <int ST>
__device__ inline void color_fine_block(const DevMap& m, const DepthFrame& f, const uint8_t* __restrict__ rgb, int32_t bx,
                                        int32_t by, int32_t bz, uint32_t info, uint32_t now, bool fresh, bool merged) {
    const int lane = lane_id();
    int I, J, K;
    demorton3(lane, I, J, K);
    int pix[8];
    float obs[8];
    const uint32_t upd = fine_decisions(m, f, f.depth, bx, by, bz, I, J, K, pix, obs);
    if (!__ballot(upd != 0) && !fresh) return;
    const size_t base = (size_t)(info & kSlotMask) * 512 + (size_t)lane * 8;
    uint32_t W[8];
    Store<ST>::getW8(m, base, W);
    float c[24];
    float4* cp = reinterpret_cast<float4*>(m.C[0] + 3 * base);  // 96 B per group, 16 B aligned
    if (fresh) {
        for (int k = 0; k < 24; ++k) c[k] = 0.f;
    } else {
        for (int k = 0; k < 6; ++k) {
            const float4 v = cp[k];
            c[4 * k] = v.x, c[4 * k + 1] = v.y, c[4 * k + 2] = v.z, c[4 * k + 3] = v.w;
        }
    }
    float sw = 0.f, s0 = 0.f, s1 = 0.f, s2 = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const bool u = (upd >> q) & 1;
        const uint32_t Wp = merged ? W[q] + (u ? 1u : 0u) : W[q];
        if (u) {
            const float inv = 1.0f / (float)Wp;
            for (int ch = 0; ch < 3; ++ch)
                c[3 * q + ch] = c[3 * q + ch] + ((float)rgb[3 * (size_t)pix[q] + ch] - c[3 * q + ch]) * inv;
        }
        const float w = (float)Wp;
        sw += w;
        s0 += w * c[3 * q];
        s1 += w * c[3 * q + 1];
        s2 += w * c[3 * q + 2];
    }
    if (merged) {
        const size_t at = (size_t)(now & kSlotMask) * 64 + (size_t)lane;
        const float inv = sw > 0.f ? 1.0f / sw : 0.f;
        float* Cc = m.C[1];
        Cc[3 * at] = s0 * inv;
        Cc[3 * at + 1] = s1 * inv;
        Cc[3 * at + 2] = s2 * inv;
    } else if (upd || fresh) {
        for (int k = 0; k < 6; ++k) cp[k] = make_float4(c[4 * k], c[4 * k + 1], c[4 * k + 2], c[4 * k + 3]);
    }
}

// One block (one wave): entry e as queued at the frame's start (or a new block of the frame).
template <int ST>
__device__ inline void color_block(const DevMap& m, const DepthFrame& f, const uint8_t* __restrict__ rgb, uint4 e,
                                   bool fresh) {
    const uint32_t id = e.x, info = e.y;
    if (info & kNoBlockBit) return;
    int32_t bx, by, bz;
    unpack_key(entry_key(e), bx, by, bz);
    const int lvl = (int)((info >> kLevelShift) & 3u), ms = 8 >> lvl, nv = ms * ms * ms;
    const size_t slot = info & kSlotMask;
    const uint32_t now = m.binfo[id];
    const bool merged = !fresh && !(now & kNoBlockBit) && (int)((now >> kLevelShift) & 3u) == lvl + 1;
    if (!fresh && block_hidden(m, f, bx, by, bz)) return;  // no voxel of it can be updated
    if (lvl == 0) {
        color_fine_block<ST>(m, f, rgb, bx, by, bz, info, now, fresh, merged);
        return;
    }
    const int lane = lane_id();
    float* C = m.C[lvl];
    for (int r = 0; r < nv; r += 64) {
        const int v = r + lane;
        const bool act = v < nv;
        bool upd = false;
        uint32_t Wp = 0;
        float c[3] = {0.f, 0.f, 0.f};
        if (act) {
            int i, j, k;
            demorton3(v, i, j, k);
            double x0, x1, x2;
            voxel_camera(m, f, bx, by, bz, lvl, i, j, k, x0, x1, x2);
            int p = -1;
            upd = observe_pixel(m, f, x0, x1, x2, p);
            const size_t at = slot * (size_t)nv + (size_t)v;
            const uint32_t W = Store<ST>::getW(m, lvl, at);
            Wp = merged ? W + (upd ? 1u : 0u) : W;
            if (!fresh)
                for (int ch = 0; ch < 3; ++ch) c[ch] = C[3 * at + ch];
            if (upd) {
                const float inv = 1.0f / (float)Wp;
                for (int ch = 0; ch < 3; ++ch) c[ch] = c[ch] + ((float)rgb[3 * (size_t)p + ch] - c[ch]) * inv;
            }
            if (!merged && (upd || fresh))
                for (int ch = 0; ch < 3; ++ch) C[3 * at + ch] = c[ch];
        }
        if (merged) {
            // the 8 children of coarse voxel v / 8 are 8 consecutive lanes (Morton order)
            float sw = (float)Wp, s0 = sw * c[0], s1 = sw * c[1], s2 = sw * c[2];
            sw = group8_sum(sw);
            s0 = group8_sum(s0);
            s1 = group8_sum(s1);
            s2 = group8_sum(s2);
            if (act && (v & 7) == 0) {
                const size_t at = (size_t)(now & kSlotMask) * (size_t)(nv / 8) + (size_t)(v >> 3);
                float* Cc = m.C[lvl + 1];
                const float inv = sw > 0.f ? 1.0f / sw : 0.f;
                Cc[3 * at] = s0 * inv;
                Cc[3 * at + 1] = s1 * inv;
                Cc[3 * at + 2] = s2 * inv;
            }
        }
    }
}

template <int ST>
__global__ __launch_bounds__(256) void k_integrate_color(const DevMap* __restrict__ pm, DepthFrame f,
                                                         const uint8_t* __restrict__ rgb) {
    const DevMap& m = *pm;
    const TaskCounts c = frame_task_counts(m, true, f.parity);
    const uint32_t n01 = c.n[0] + c.n_new, n012 = n01 + c.n[1], n0123 = n012 + c.n[2], ntask = n0123 + c.n[3];
    const uint32_t wave = uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t t = wave; t < ntask; t += nwaves) {
        uint4 e;
        bool fresh = false;
        if (t < c.n[0]) {
            e = m.vis[0][t];
        } else if (t < n01) {
            const uint32_t id = c.new_base + (t - c.n[0]);
            e = make_entry(id, m.binfo[id], m.bkey[id]);
            fresh = true;
        } else if (t < n012) {
            e = m.vis[1][t - n01];
        } else if (t < n0123) {
            e = m.vis[2][t - n012];
        } else {
            e = m.vis[3][t - n0123];
        }
        color_block<ST>(m, f, rgb, uniform(e), fresh);
    }
}

// Colours out, in the voxel order of mrh_extract_blocks (x fastest per block).
__global__ void k_extract_color(const DevMap* __restrict__ pm, uint32_t nb, const int32_t* __restrict__ pos,
                                const int64_t* __restrict__ offsets, float* out) {
    const DevMap& m = *pm;
    const int lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t id = wave; id < nb; id += nwaves) {
        const int32_t row = pos[id];
        const uint32_t info = m.binfo[id];
        if (row < 0 || (info & kNoBlockBit)) continue;
        const int lvl = (int)((info >> kLevelShift) & 3u), ms = 8 >> lvl, nv = ms * ms * ms;
        const size_t base = (size_t)(info & kSlotMask) * nv;
        for (int p = lane; p < nv; p += 64) {
            int i, j, k;
            demorton3(p, i, j, k);
            const int64_t o = offsets[row] + i + ms * (j + ms * k);
            for (int ch = 0; ch < 3; ++ch) out[3 * o + ch] = m.C[lvl][3 * (base + p) + ch];
        }
    }
}

}  // namespace mrh

using namespace mrh;

extern "C" mrh_status mrh_integrate_rgbd(mrh_map* map, const float* depth_dev, const uint8_t* rgb_dev, int32_t width,
                                         int32_t height, const double K[4], const double T_ws[16]) {
    if (!map || !rgb_dev) return MRH_ERR_INVALID_ARG;
    if (!map->cfg.color) return set_error(map, MRH_ERR_INVALID_ARG, "the map was created without colour");
    DepthFrame f;
    const mrh_status st = integrate_depth_frame(map, depth_dev, width, height, K, T_ws, &f);
    if (st != MRH_OK) return st;
    launch(map, K_COLOR, [&] {
        switch (map->cfg.storage) {
            case MRH_STORE_F16: hipLaunchKernelGGL(k_integrate_color<MRH_STORE_F16>, dim3(1024), dim3(256), 0, map->stream, map->dmd, f, rgb_dev); break;
            case MRH_STORE_BF16: hipLaunchKernelGGL(k_integrate_color<MRH_STORE_BF16>, dim3(1024), dim3(256), 0, map->stream, map->dmd, f, rgb_dev); break;
            default: hipLaunchKernelGGL(k_integrate_color<MRH_STORE_F32>, dim3(1024), dim3(256), 0, map->stream, map->dmd, f, rgb_dev);
        }
    });
    return check_hip(map, hipGetLastError(), "integrate_rgbd");
}

extern "C" mrh_status mrh_extract_color(mrh_map* map, float* rgb_dev, int64_t voxel_cap, int64_t* n_voxels) {
    if (!map || !n_voxels) return MRH_ERR_INVALID_ARG;
    if (!map->cfg.color) return set_error(map, MRH_ERR_INVALID_ARG, "the map was created without colour");
    DevCounters h;
    mrh_status st = check_hip(map, hipMemcpyAsync(&h, map->ctr, sizeof(h), hipMemcpyDeviceToHost, map->stream), "extract colour");
    if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "extract colour");
    if (st != MRH_OK) return st;
    const uint32_t nb = h.n_blocks < map->dm.max_blocks ? h.n_blocks : map->dm.max_blocks;
    std::vector<uint32_t> info(nb);
    if (nb) {
        st = check_hip(map, hipMemcpy(info.data(), map->dm.binfo, (size_t)nb * 4, hipMemcpyDeviceToHost), "extract colour");
        if (st != MRH_OK) return st;
    }
    // the rows and voxel offsets of mrh_extract_blocks
    std::vector<int32_t> pos(nb, -1);
    std::vector<int64_t> offs(1, 0);
    uint32_t nout = 0;
    for (uint32_t i = 0; i < nb; ++i) {
        if (info[i] & kGoneBit) continue;
        const int lvl = (int)((info[i] >> kLevelShift) & 3u);
        const int64_t nv = (info[i] & kNoBlockBit) ? 0 : (int64_t)side_of(lvl) * side_of(lvl) * side_of(lvl);
        pos[i] = (int32_t)nout++;
        offs.push_back(offs.back() + nv);
    }
    *n_voxels = offs[nout];
    if (!rgb_dev) return MRH_OK;
    if (voxel_cap < offs[nout]) return set_error(map, MRH_ERR_BUFFER_TOO_SMALL, "colour needs %lld voxels", (long long)offs[nout]);
    if (nout == 0) return MRH_OK;
    int64_t* doffs = nullptr;
    int32_t* dpos = nullptr;
    st = check_hip(map, hipMalloc((void**)&doffs, ((size_t)nout + 1) * 8), "extract colour");
    if (st == MRH_OK) st = check_hip(map, hipMalloc((void**)&dpos, (size_t)nb * 4), "extract colour");
    if (st == MRH_OK) st = check_hip(map, hipMemcpy(doffs, offs.data(), ((size_t)nout + 1) * 8, hipMemcpyHostToDevice), "extract colour");
    if (st == MRH_OK) st = check_hip(map, hipMemcpy(dpos, pos.data(), (size_t)nb * 4, hipMemcpyHostToDevice), "extract colour");
    if (st == MRH_OK) {
        const uint32_t grid = nb / 4 + 1 < 4096 ? nb / 4 + 1 : 4096;
        hipLaunchKernelGGL(k_extract_color, dim3(grid), dim3(256), 0, map->stream, map->dmd, nb, dpos, doffs, rgb_dev);
        st = check_hip(map, hipGetLastError(), "extract colour");
        if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "extract colour");
    }
    if (doffs) (void)hipFree(doffs);
    if (dpos) (void)hipFree(dpos);
    return st;
}
