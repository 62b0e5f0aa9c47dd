// RGB-D fusion work units (Sec. 3.1 "Cameras", Eq. 2; Eq. 3 and Eq. 5; Sec. 3.2.1 merging
// criterion), shared by the single-map kernels (depth.hip) and the batched kernels (batch.hip).
//
//   depth_alloc_tile   a 16 x 16 pixel tile (one workgroup, each wave a 16 x 4 strip): back-
//                      projection, band walk over the block lattice, wave-deduplicated insert; new
//                      blocks are queued for the update
//   depth_cull         one thread per block that existed at the frame's start: conservative frustum
//                      test, visible blocks queued per level
//   depth_update_task  one queued level-0 or level-1 block (a wave), or 8 level-2 / 64 level-3
//                      blocks per wave: per-voxel projection and update, block variance bookkeeping
//                      and the merge of a block whose mean variance fell below the threshold
#pragma once

#include "mrh_update.h"

namespace mrh {

struct DepthFrame {
    int32_t parity;  // the frame's parity (selects the double-buffered per-frame counts)
    Pose P;
    double fx, fy, cx, cy, ifx, ify;
    int32_t width, height;
    const float* depth;  // device z-depth image, row-major
    float fxf, fyf, cxf, cyf;  // intrinsics rounded to FP32 for the fast projection
    // conservative culling of whole blocks (camera frame): side-plane normals and a range bound
    double plane[4][3];
    double cull_range;
    // largest valid depth per 16 x 16 pixel tile (written by the allocation launch, -1 when the
    // tile holds no valid sample), tiles_x tiles per row
    float* tile_max;
    int32_t tiles_x, tiles_y;
};

// Host: frame sizes the kernels accept (pixel indices 32-bit, pixel coordinates exact in FP32).
bool depth_size_ok(int32_t width, int32_t height);

// Host: enqueue the allocation and update launches of one RGB-D frame (no colour check);
// *frame_out (may be NULL) receives the frame's descriptor.
mrh_status integrate_depth_frame(mrh_map* map, const float* depth_dev, int32_t width, int32_t height,
                                 const double K[4], const double T_ws[16], DepthFrame* frame_out);

// Host: fill a frame descriptor; false on a non-finite pose or intrinsics or a zero focal length.
bool make_depth_frame(const mrh_config& cfg, const float* depth, int32_t width, int32_t height, const double K[4],
                      const double T_ws[16], DepthFrame& f);

// Nearest pixel of the voxel centre x (camera frame) under the projection of Eq. 2: the FP64
// evaluation u = fx (x0 (1 / x2)) + cx, pixel floor(u + 1/2), and likewise for v.  Returns the
// row-major pixel index, or -1 when x is not in front of the camera or falls outside the image.
__device__ inline int pixel_exact(const DepthFrame& f, double x0, double x1, double x2) {
    if (!(x2 > 0.0)) return -1;
    const double iz = 1.0 / x2;
    const double uu = (f.fx * (x0 * iz)) + f.cx;
    const double vv = (f.fy * (x1 * iz)) + f.cy;
    const double fu = __builtin_floor(uu + 0.5), fv = __builtin_floor(vv + 0.5);
    if (!(fu >= 0.0 && fu <= (double)(f.width - 1) && fv >= 0.0 && fv <= (double)(f.height - 1))) return -1;
    return (int)fv * f.width + (int)fu;
}

// The same decision from the FP32 evaluation, taken only when it lies farther from a pixel boundary
// than its error can reach; returns -2 when it cannot decide.  Error budget of the FP32 u from FP64
// x: the roundings of x0, x2, fx, cx, the product and the sum (2^-24 relative each) and the hardware
// reciprocal (1 ulp) stay below 6e-7 (|u| + |cx|), under the margin 1e-6 (|u| + |cx| + 16).  `lam`
// receives |x| / x2 in FP32 for the range form.
__device__ inline int pixel_fast(const DepthFrame& f, double x0, double x1, double x2, float& lam) {
    lam = 0.f;
    if (!(x2 > 0.0)) return -1;
    const float xf0 = (float)x0, xf1 = (float)x1, xf2 = (float)x2;
    if (!(xf2 > 1e-6f)) return -2;
    const float izf = __builtin_amdgcn_rcpf(xf2);
    lam = __builtin_amdgcn_sqrtf((xf0 * xf0 + xf1 * xf1) + xf2 * xf2) * izf;
    const float uf = f.fxf * (xf0 * izf) + f.cxf;
    const float vf = f.fyf * (xf1 * izf) + f.cyf;
    const float su = uf + 0.5f, sv = vf + 0.5f;
    const float fu = __builtin_floorf(su), fv = __builtin_floorf(sv);
    const float du = __builtin_fminf(su - fu, fu + 1.0f - su), dv = __builtin_fminf(sv - fv, fv + 1.0f - sv);
    const float eu = 1e-6f * (__builtin_fabsf(uf) + __builtin_fabsf(f.cxf) + 16.0f);
    const float ev = 1e-6f * (__builtin_fabsf(vf) + __builtin_fabsf(f.cyf) + 16.0f);
    if (!(du > eu && dv > ev)) return -2;
    if (!(fu >= 0.0f && fu <= (float)(f.width - 1) && fv >= 0.0f && fv <= (float)(f.height - 1))) return -1;
    return (int)fv * f.width + (int)fu;
}

// Observation of Eq. 2 (gate at -tau, truncation at +tau) for the voxel centre x from the depth d
// of its pixel, in FP64: the canonical evaluation.  False when the voxel is not updated.
__device__ inline bool observe_exact(const DevMap& m, double x0, double x1, double x2, double d, float& obs) {
    if (!(__builtin_isfinite(d) && d > 0.0 && d <= m.max_depth)) return false;
    double raw;
    if (m.form == MRH_FORM_RANGE) {
        const double iz = 1.0 / x2;
        const double nx = __builtin_sqrt((x0 * x0 + x1 * x1) + x2 * x2);
        raw = nx * ((d * iz) - 1.0);
    } else {
        raw = d - x2;
    }
    if (raw < -m.tau) return false;
    obs = (float)(raw < m.tau ? raw : m.tau);
    return true;
}

// The same observation with the range form's scale |x| / x2 in FP32 (`lam` from pixel_fast).
// Returns 1 (update with obs), 0 (no update) or 2 (undecided: observe_exact must decide).  The
// validity test is the canonical one (max_depth_f is the largest float not above max_depth) and
// the z-difference form is evaluated exactly; the range-form value carries about 8 ulps (squares,
// sums, square root, reciprocal), so its -tau gate is taken only outside a 1e-5 tau band.
__device__ inline int observe_fast(const DevMap& m, double x2, float lam, float d, float& obs) {
    if (!(__builtin_isfinite(d) && d > 0.0f && d <= m.max_depth_f)) return 0;
    const double ddiff = (double)d - x2;
    if (m.form != MRH_FORM_RANGE) {
        if (ddiff < -m.tau) return 0;
        obs = (float)(ddiff < m.tau ? ddiff : m.tau);
        return 1;
    }
    const float raw = (float)ddiff * lam;
    if (__builtin_fabsf(raw + m.tau_f) <= 1e-5f * m.tau_f + 1e-6f * __builtin_fabsf(raw)) return 2;
    if (raw < -m.tau_f) return 0;
    obs = raw < m.tau_f ? raw : m.tau_f;
    return 1;
}

// One voxel: pixel decision, depth lookup, observation.
__device__ inline bool observe(const DevMap& m, const DepthFrame& f, const float* __restrict__ depth, double x0,
                               double x1, double x2, float& obs) {
    float lam;
    int p = pixel_fast(f, x0, x1, x2, lam);
    const bool exact = p == -2;
    if (exact) p = pixel_exact(f, x0, x1, x2);
    if (p < 0) return false;
    const float d = depth[p];
    if (!exact) {
        const int r = observe_fast(m, x2, lam, d, obs);
        if (r != 2) return r == 1;
    }
    return observe_exact(m, x0, x1, x2, (double)d, obs);
}

// Wave-uniform test (all lanes active): true when no voxel of block (bx, by, bz) can be updated by
// this frame.  With every block corner in front of the camera, each voxel centre projects inside the
// rectangle spanned by the projected corners (padded by a pixel against rounding) and lies at least
// as deep as the shallowest corner, zmin.  If zmin exceeds every valid depth of the tiles that the
// rectangle touches by more than tau, each voxel has x_z - d > tau for the depth d of its own pixel,
// so raw < -tau under both readings of Eq. 2 (the range reading scales x_z - d by |x| / x_z >= 1)
// and the gate rejects it; pixels outside the image or without a valid depth are never updated.
__device__ inline bool block_hidden(const DevMap& m, const DepthFrame& f, int32_t bx, int32_t by, int32_t bz) {
    const int lane = lane_id(), c = lane & 7;
    const double w0 = ((double)bx + (double)(c & 1)) * m.B - f.P.t[0];
    const double w1 = ((double)by + (double)((c >> 1) & 1)) * m.B - f.P.t[1];
    const double w2 = ((double)bz + (double)(c >> 2)) * m.B - f.P.t[2];
    const double x0 = (f.P.R[0][0] * w0 + f.P.R[1][0] * w1) + f.P.R[2][0] * w2;
    const double x1 = (f.P.R[0][1] * w0 + f.P.R[1][1] * w1) + f.P.R[2][1] * w2;
    const double x2 = (f.P.R[0][2] * w0 + f.P.R[1][2] * w1) + f.P.R[2][2] * w2;
    // every group of 8 lanes holds the 8 corners, so these reductions are wave-uniform
    double zmin = x2;
    zmin = group8_fmin(zmin);
    if (!(zmin > 1e-3)) return false;
    const double iz = 1.0 / x2;
    const double u = __builtin_fmin(__builtin_fmax(f.fx * (x0 * iz) + f.cx, -1e8), 1e8);
    const double v = __builtin_fmin(__builtin_fmax(f.fy * (x1 * iz) + f.cy, -1e8), 1e8);
    int u0 = (int)__builtin_floor(u) - 1, u1 = (int)__builtin_ceil(u) + 1;
    int v0 = (int)__builtin_floor(v) - 1, v1 = (int)__builtin_ceil(v) + 1;
    u0 = group8_min(u0);
    u1 = group8_max(u1);
    v0 = group8_min(v0);
    v1 = group8_max(v1);
    if (u1 < 0 || v1 < 0 || u0 > f.width - 1 || v0 > f.height - 1) return true;
    const int tu0 = max(u0, 0) >> 4, tu1 = min(u1, f.width - 1) >> 4;
    const int tv0 = max(v0, 0) >> 4, tv1 = min(v1, f.height - 1) >> 4;
    const int ntu = tu1 - tu0 + 1, nt = ntu * (tv1 - tv0 + 1);
    if (nt > 256) return false;
    float dmax = -1.0f;
    for (int k = lane; k < nt; k += 64) {
        const int ty = k / ntu;
        dmax = __builtin_fmaxf(dmax, f.tile_max[(tv0 + ty) * f.tiles_x + tu0 + (k - ty * ntu)]);
    }
    dmax = wave_max(dmax);
    return zmin > (double)dmax + m.tau * (1.0 + 1e-6) + 1e-9;
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

// Conservative frustum cull of the blocks that existed when the frame started, one thread per
// block: workgroup g of ng covers ids g * 256 + threadIdx, stepping by ng * 256.
__device__ inline void depth_cull(const DevMap& m, const DepthFrame& f, uint32_t g, uint32_t ng) {
    const uint32_t n = m.ctr->n_prev[f.parity];
    for (uint32_t base = g * blockDim.x; base < n; base += ng * blockDim.x) {
        const uint32_t id = base + threadIdx.x;
        int level = -1;
        uint32_t info = 0;
        unsigned long long key = 0;
        if (id < n) {
            info = m.binfo[id];
            if (!(info & kNoBlockBit)) {
                key = m.bkey[id];
                int32_t bx, by, bz;
                unpack_key(key, bx, by, bz);
                if ((info & kNewBit) || block_visible(m, f, bx, by, bz)) level = (int)((info >> kLevelShift) & 3u);
            }
        }
        queue_block_wg(m, level, id, info, key, f.parity);
    }
}

constexpr int kTileNew = 512;  // new blocks a tile registers with one allocation atomic

// One 16 x 16 pixel tile per workgroup (tile index `tile`, tiles_x tiles per row).  The keys a
// wave inserts are collected in LDS and registered with one atomic on the allocation word per
// workgroup; a key that finds the list full is registered by its wave directly.
__device__ inline void depth_alloc_tile(const DevMap& m, const DepthFrame& f, uint32_t tile, uint32_t tiles_x) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const float* __restrict__ depth = f.depth;
    const int u = (int)(tile % tiles_x) * 16 + (lane & 15);
    const int v = (int)(tile / tiles_x) * 16 + wave * 4 + (lane >> 4);
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
    __shared__ uint32_t cnt[3];
    __shared__ float tmx[4];
    __shared__ unsigned long long nkey[kTileNew];
    __shared__ uint32_t nslot[kTileNew];
    __shared__ uint32_t ncount;
    __shared__ unsigned long long nold;
    if (threadIdx.x == 0) cnt[0] = cnt[1] = cnt[2] = ncount = 0;
    const float wmax = wave_max(ok ? (float)d : -1.0f);
    if (lane == 0) tmx[wave] = wmax;
    __syncthreads();
    const unsigned long long vmask = __ballot(ok), dmask = __ballot(ok && !in_range);
    if (lane == 0) {
        atomicAdd(&cnt[0], (uint32_t)__popcll(vmask));
        atomicAdd(&cnt[1], (uint32_t)__popcll(dmask));
    }
    bool active = in_range;
    uint32_t ncand = 0;  // keys this wave's walks produce (wave-uniform)
    while (unsigned long long amask = __ballot(active)) {
        ncand += (uint32_t)__popcll(amask);
        const unsigned long long key = active ? pack_key(w.c0, w.c1, w.c2) : 0ull;
        uint32_t slot = 0;
        const bool is_new = claim_keys(m, active, key, &slot);
        const unsigned long long newmask = __ballot(is_new);
        bool spill = false;
        if (newmask) {
            const int first = __ffsll((long long)newmask) - 1;
            uint32_t at = 0;
            if (lane == first) at = atomicAdd(&ncount, (uint32_t)__popcll(newmask));
            at = (uint32_t)__shfl((int)at, first) + (uint32_t)rank_in_mask(newmask);
            if (is_new) {
                if (at < (uint32_t)kTileNew) {
                    nkey[at] = key;
                    nslot[at] = slot;
                } else {
                    spill = true;
                }
            }
            register_new(m, spill, key, slot);
        }
        if (active) active = w.next();
    }
    if (lane == 0 && ncand) atomicAdd(&cnt[2], ncand);
    __syncthreads();
    const uint32_t nnew = ncount < (uint32_t)kTileNew ? ncount : (uint32_t)kTileNew;
    if (threadIdx.x == 0 && nnew) nold = take_new_blocks(m, nnew);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nnew; i += blockDim.x)
        register_block(m, nkey[i], nslot[i], (uint32_t)nold + i, (uint32_t)(nold >> 32) + i);
    if (threadIdx.x == 0) {
        stat_add(m, S_VALID, cnt[0]);
        stat_add(m, S_DROPPED, cnt[1]);
        stat_add(m, S_CAND, cnt[2]);
        f.tile_max[tile] = __builtin_fmaxf(__builtin_fmaxf(tmx[0], tmx[1]), __builtin_fmaxf(tmx[2], tmx[3]));
    }
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

// The projective decisions of lane group (I, J, K) of level-0 block (bx, by, bz): the 2x2x2 voxels
// 2I + a, 2J + b, 2K + c at Morton positions q = a + 2 b + 4 c.  pix[q] receives the voxel's pixel
// (-1: none), obs[q] its observation, and the returned mask has bit q set when the frame updates the
// voxel.  Every launch that needs these decisions (the update, the colour launch) calls this one
// function, so they agree voxel for voxel.
__device__ inline uint32_t fine_decisions(const DevMap& m, const DepthFrame& f, const float* __restrict__ depth,
                                          int32_t bx, int32_t by, int32_t bz, int I, int J, int K, int pix[8],
                                          float obs[8]) {
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
    // pixels first (FP64 only where FP32 cannot decide), then all depth loads at once, then the
    // observations; x recomputed by voxel_camera equals these sums bit for bit (same products, same
    // order, no contraction)
    float lam[8];
    uint32_t exact = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int a = q & 1, b = (q >> 1) & 1, c = (q >> 2) & 1;
        const double x0 = (px[a][0] + py[b][0]) + pz[c][0];
        const double x1 = (px[a][1] + py[b][1]) + pz[c][1];
        const double x2 = (px[a][2] + py[b][2]) + pz[c][2];
        pix[q] = pixel_fast(f, x0, x1, x2, lam[q]);
        exact |= (pix[q] == -2 ? 1u : 0u) << q;
    }
    for (uint32_t amb = exact; amb;) {
        const int q = __builtin_ctz(amb);
        amb &= amb - 1;
        double x0, x1, x2;
        voxel_camera(m, f, bx, by, bz, 0, 2 * I + (q & 1), 2 * J + ((q >> 1) & 1), 2 * K + (q >> 2), x0, x1, x2);
        const int p = pixel_exact(f, x0, x1, x2);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k == q) pix[k] = p;
    }
    float dq[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) dq[q] = pix[q] >= 0 ? depth[pix[q]] : -1.f;
    uint32_t upd = 0, slow = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        obs[q] = 0.f;
        const double x2 = (px[q & 1][2] + py[(q >> 1) & 1][2]) + pz[q >> 2][2];
        const int r = (exact >> q) & 1 ? (dq[q] > 0.f ? 2 : 0) : observe_fast(m, x2, lam[q], dq[q], obs[q]);
        upd |= (r == 1 ? 1u : 0u) << q;
        slow |= (r == 2 ? 1u : 0u) << q;
    }
    // voxels the FP32 evaluation left undecided: the canonical evaluation from the same depth sample
    while (slow) {
        const int q = __builtin_ctz(slow);
        slow &= slow - 1;
        double x0, x1, x2;
        voxel_camera(m, f, bx, by, bz, 0, 2 * I + (q & 1), 2 * J + ((q >> 1) & 1), 2 * K + (q >> 2), x0, x1, x2);
        float o = 0.f, dsel = 0.f;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k == q) dsel = dq[k];
        if (observe_exact(m, x0, x1, x2, (double)dsel, o)) {
            upd |= 1u << q;
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k == q) obs[k] = o;
        }
    }
    return upd;
}

// Level-0 block: lane l owns the 2x2x2 group of Morton positions 8l .. 8l+7.
template <int ST>
__device__ inline TaskOut integrate_fine_block(const DevMap& m, const DepthFrame& f, const float* __restrict__ depth,
                                            const uint4 eq) {
    const int lane = lane_id();
    const uint4 e = uniform(eq);  // one block per wave
    const uint32_t id = e.x, info = e.y;
    if (info & kNoBlockBit) return TaskOut{};
    int32_t bx, by, bz;
    unpack_key(entry_key(e), bx, by, bz);
    const bool fresh = (info & kNewBit) != 0;
    const double bvs = m.bvsum[id];
    const uint32_t bvc = m.bvcnt[id];
    if (!fresh && block_hidden(m, f, bx, by, bz)) return TaskOut{};
    int I, J, K;
    demorton3(lane, I, J, K);
    int pix[8];
    float obs[8];
    const uint32_t upd = fine_decisions(m, f, depth, bx, by, bz, I, J, K, pix, obs);
    const int nupd = wave_sum((int)__popc(upd));
    if (nupd == 0 && !fresh) return TaskOut{};
    TaskOut out;
    out.obs = (uint32_t)nupd;
    out.fresh = fresh ? (uint32_t)nupd : 0u;

    const size_t base = (size_t)(info & kSlotMask) * 512 + (size_t)lane * 8;
    float D[8], S2[8];
    uint32_t W[8];
    bool have = false;
    if (fresh) {
        for (int q = 0; q < 8; ++q) D[q] = 0.f, S2[q] = 0.f, W[q] = 0u;
        have = true;
    } else if (upd) {
        Store<ST>::get8(m, base, D, W, S2);
        have = true;
    }
    double dsum = 0.0;
    int dcnt = 0;
    for (int q = 0; q < 8; ++q) {
        if (!(upd & (1u << q))) continue;
        const double before = var_term(m, W[q], S2[q]);
        const int cb = var_count(m, W[q]);
        welford(obs[q], D[q], W[q], S2[q]);
        Store<ST>::round(m, D[q], W[q], S2[q]);
        dsum += var_term(m, W[q], S2[q]) - before;
        dcnt += var_count(m, W[q]) - cb;
    }
    out.merge0 = (uint32_t)finish_fine<ST>(m, id, info, D, W, S2, have, upd != 0 || fresh, nupd, dsum, dcnt,
                                                        bvs, bvc, f.parity);
    return out;
}

// Level-1 block: lane l owns the voxel at Morton position l.
template <int ST>
__device__ inline TaskOut integrate_level1_block(const DevMap& m, const DepthFrame& f, const float* __restrict__ depth,
                                              const uint4 eq) {
    const int lane = lane_id();
    const uint4 e = uniform(eq);  // one block per wave
    const uint32_t id = e.x, info = e.y;
    int32_t bx, by, bz;
    unpack_key(entry_key(e), bx, by, bz);
    const double bvs = m.bvsum[id];
    const uint32_t bvc = m.bvcnt[id];
    if (block_hidden(m, f, bx, by, bz)) return TaskOut{};
    int i, j, k;
    demorton3(lane, i, j, k);
    double x0, x1, x2;
    voxel_camera(m, f, bx, by, bz, 1, i, j, k, x0, x1, x2);
    float obs = 0.f;
    const bool upd = observe(m, f, depth, x0, x1, x2, obs);
    const int nupd = __popcll(__ballot(upd));
    if (nupd == 0) return TaskOut{};
    TaskOut out;
    out.obs = (uint32_t)nupd;
    const size_t at = (size_t)(info & kSlotMask) * 64 + lane;
    float D, S2;
    uint32_t W;
    Store<ST>::get(m, 1, at, D, W, S2);
    double dsum = 0.0;
    int dcnt = 0;
    if (upd) {
        const double before = var_term(m, W, S2);
        const int cb = var_count(m, W);
        welford(obs, D, W, S2);
        Store<ST>::round(m, D, W, S2);
        dsum = var_term(m, W, S2) - before;
        dcnt = var_count(m, W) - cb;
    }
    out.merge1 = (uint32_t)finish_coarse<ST>(m, id, info, 1, D, W, S2, upd, nupd, dsum, dcnt, bvs, bvc,
                                                          f.parity);
    return out;
}

// 64 / seg blocks of `level` (2: seg = 8 voxels, 3: seg = 1 voxel) per wave.
template <int ST>
__device__ inline TaskOut integrate_packed_blocks(const DevMap& m, const DepthFrame& f, const float* __restrict__ depth,
                                               const uint4* list, uint32_t count, uint32_t group, int level) {
    const int lane = lane_id();
    const int seg = level == 2 ? 8 : 1;
    const uint32_t bi = group * (uint32_t)(64 / seg) + (uint32_t)(lane / seg);
    const bool live = bi < count;
    uint32_t id = 0, info = 0;
    bool upd = false;
    float obs = 0.f;
    if (live) {
        const uint4 e = list[bi];
        id = e.x;
        info = e.y;
        int32_t bx, by, bz;
        unpack_key(entry_key(e), bx, by, bz);
        int i, j, k;
        demorton3(lane % seg, i, j, k);
        double x0, x1, x2;
        voxel_camera(m, f, bx, by, bz, level, i, j, k, x0, x1, x2);
        upd = observe(m, f, depth, x0, x1, x2, obs);
    }
    if (!__ballot(upd)) return TaskOut{};
    float D = 0.f, S2 = 0.f;
    uint32_t W = 0;
    double dsum = 0.0;
    int dcnt = 0;
    if (upd) {
        Store<ST>::get(m, level, (size_t)(info & kSlotMask) * seg + (lane % seg), D, W, S2);
        const double before = var_term(m, W, S2);
        const int cb = var_count(m, W);
        welford(obs, D, W, S2);
        Store<ST>::round(m, D, W, S2);
        dsum = var_term(m, W, S2) - before;
        dcnt = var_count(m, W) - cb;
    } else if (live && seg > 1) {
        // a segment whose block merges needs all of its voxels
        Store<ST>::get(m, level, (size_t)(info & kSlotMask) * seg + (lane % seg), D, W, S2);
    }
    TaskOut out;
    out.obs = (uint32_t)wave_sum(upd ? 1 : 0);
    out.merge2 = (uint32_t)wave_sum(finish_packed<ST>(m, live, id, info, level, seg, D, W, S2, upd, upd ? 1 : 0, dsum,
                                                      dcnt));
    return out;
}

// One update task t of the frame's task space (see TaskCounts).
template <int ST>
__device__ inline TaskOut depth_update_task(const DevMap& m, const DepthFrame& f, uint32_t t, const TaskCounts& c) {
    const uint32_t n0 = c.n[0] + c.n_new;
    const uint32_t g2 = (c.n[2] + 7) / 8;
    if (t < c.n[0]) return integrate_fine_block<ST>(m, f, f.depth, m.vis[0][t]);
    if (t < n0) {
        const uint32_t id = c.new_base + (t - c.n[0]);
        return integrate_fine_block<ST>(m, f, f.depth, make_entry(id, m.binfo[id], m.bkey[id]));
    }
    if (t < n0 + c.n[1]) return integrate_level1_block<ST>(m, f, f.depth, m.vis[1][t - n0]);
    if (t < n0 + c.n[1] + g2) return integrate_packed_blocks<ST>(m, f, f.depth, m.vis[2], c.n[2], t - n0 - c.n[1], 2);
    return integrate_packed_blocks<ST>(m, f, f.depth, m.vis[3], c.n[3], t - n0 - c.n[1] - g2, 3);
}

}  // namespace mrh
