// Multi-resolution trilinear SDF query (Sec. 3.4) and its adjoint for points and a 6-DoF pose.
//
// One thread per point.  The point's block fixes the interpolation lattice (its level n); each of
// the 8 surrounding level-n lattice points takes the TSDF of the voxel, at whatever level its own
// block has, whose cell contains it; corners without a block or with W = 0 drop out and the
// remaining trilinear weights are renormalised.  Lattice indices and weights are FP64.
#include <cmath>

#include "mrh_store.h"

namespace mrh {

struct QueryParams {
    Pose P;
    int32_t identity;
    int32_t strict;
};

struct QueryResult {
    bool valid;
    double sdf;
    double grad[3];  // d sdf / d x (world)
};

// Block table row of `key` for a query corner: the home slot is read for all corners at once, and
// only a corner whose home slot holds another key walks the probe sequence.
__device__ inline uint32_t corner_info(const DevMap& m, unsigned long long key, unsigned long long home_key,
                                       uint32_t home_slot_id) {
    if (home_key == key) return m.hvals[home_slot_id];
    if (home_key == kEmptyKey) return kInvalidId;
    return find_block(m, key);
}

template <int ST>
__device__ inline QueryResult query_point(const DevMap& m, const double x[3], bool strict) {
    QueryResult q;
    q.valid = false;
    q.sdf = 0.0;
    q.grad[0] = q.grad[1] = q.grad[2] = 0.0;
    int64_t b[3];
    for (int k = 0; k < 3; ++k) {
        const double fb = __builtin_floor(x[k] * m.invB);
        if (!(__builtin_fabs(fb) <= (double)kKeyLimit)) return q;
        b[k] = (int64_t)fb;
    }
    const unsigned long long hkey = pack_key(b[0], b[1], b[2]);
    const uint32_t id = find_block(m, hkey);
    if (id == kInvalidId) return q;
    const uint32_t info = m.binfo[id];
    if (info & kNoBlockBit) return q;
    const int n = (int)((info >> kLevelShift) & 3u);
    const int shift = 3 - n;
    int64_t i0[3];
    double f[3];
    for (int k = 0; k < 3; ++k) {
        const double g = x[k] * m.inv_nu[n] - 0.5;
        const double fl = __builtin_floor(g);
        i0[k] = (int64_t)fl;
        f[k] = g - fl;
    }
    // the corners' blocks: along each axis the 2 lattice points lie in block lo or lo + 1
    int64_t blo[3];
    int cross[3];
    for (int k = 0; k < 3; ++k) {
        blo[k] = i0[k] >> shift;  // floor division by the block side 2^shift
        cross[k] = (int)(((i0[k] + 1) >> shift) - blo[k]);
    }
    // rows of the (up to 8) distinct blocks, addressed by (dx, dy, dz) in {0, 1}^3; all home
    // slots are read before any is examined
    unsigned long long bkeys[8], hk[8];
    uint32_t hs[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
        const bool need = (dx <= cross[0]) && (dy <= cross[1]) && (dz <= cross[2]);
        bkeys[c] = pack_key(blo[0] + dx, blo[1] + dy, blo[2] + dz);
        hs[c] = home_slot(bkeys[c], m.hmask);
        hk[c] = (!need || bkeys[c] == hkey) ? hkey : __hip_atomic_load(&m.hkeys[hs[c]], __ATOMIC_RELAXED,
                                                                          __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t binfo8[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
        const bool need = (dx <= cross[0]) && (dy <= cross[1]) && (dz <= cross[2]);
        uint32_t cid = kInvalidId;
        if (need) cid = bkeys[c] == hkey ? id : corner_info(m, bkeys[c], hk[c], hs[c]);
        binfo8[c] = cid == kInvalidId ? kNoBlockBit : (cid == id ? info : m.binfo[cid]);
    }
    // the 8 corner voxels: heap positions first, then all weight and TSDF reads
    double cw[8], cd[8];
    size_t at8[8];
    int lv8[8];
    uint32_t have = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int dl[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
        int64_t cell[3], cb[3];
        int sel = 0;
        for (int k = 0; k < 3; ++k) {
            cell[k] = i0[k] + dl[k];
            cb[k] = cell[k] >> shift;
            sel |= (int)(cb[k] - blo[k]) << k;
        }
        cw[c] = ((dl[0] ? f[0] : 1.0 - f[0]) * (dl[1] ? f[1] : 1.0 - f[1])) * (dl[2] ? f[2] : 1.0 - f[2]);
        const uint32_t binf = binfo8[sel];
        at8[c] = 0;
        lv8[c] = 0;
        if (binf & kNoBlockBit) continue;
        const int n2 = (int)((binf >> kLevelShift) & 3u);
        int idx[3];
        for (int k = 0; k < 3; ++k) {
            // lattice point (cell + 1/2) nu_n in half finest-voxel units, relative to its block
            const int64_t p2 = cell[k] * ((int64_t)2 << n) + ((int64_t)1 << n);
            idx[k] = (int)((p2 - 16 * cb[k]) >> (n2 + 1));
        }
        const int m2 = 8 >> n2;
        at8[c] = (size_t)(binf & kSlotMask) * (size_t)(m2 * m2 * m2) + (size_t)morton3(idx[0], idx[1], idx[2]);
        lv8[c] = n2;
        have |= 1u << c;
    }
    uint32_t W8[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        W8[c] = Store<ST>::getW(m, lv8[c], at8[c]);
        cd[c] = (double)Store<ST>::getD(m, lv8[c], at8[c]);
    }
    uint32_t valid_mask = 0;
    double wsum = 0.0, num = 0.0;
    bool any_pos = false;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (!(have & (1u << c)) || W8[c] == 0) {
            cd[c] = 0.0;
            continue;
        }
        valid_mask |= 1u << c;
        wsum += cw[c];
        num += cw[c] * cd[c];
        if (cw[c] > 0.0) any_pos = true;
    }
    if (strict ? valid_mask != 0xFFu : !any_pos) return q;
    q.valid = true;
    q.sdf = num / wsum;
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int c = 0; c < 8; ++c) {
            if (!(valid_mask & (1u << c))) continue;
            const int dl[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
            double dw = dl[a] ? 1.0 : -1.0;
            for (int bb = 0; bb < 3; ++bb)
                if (bb != a) dw *= dl[bb] ? f[bb] : 1.0 - f[bb];
            s += dw * (cd[c] - q.sdf);
        }
        q.grad[a] = s / wsum * m.inv_nu[n];
    }
    return q;
}

__device__ inline void world_point(const QueryParams& qp, const float* pts, int64_t i, double x[3]) {
    const double p[3] = {(double)pts[3 * i], (double)pts[3 * i + 1], (double)pts[3 * i + 2]};
    if (qp.identity) {
        x[0] = p[0], x[1] = p[1], x[2] = p[2];
    } else {
        pose_apply(qp.P, p, x);
    }
}

template <int ST>
__global__ __launch_bounds__(256) void k_query(const DevMap* __restrict__ pm, QueryParams qp, const float* __restrict__ pts,
                                               int64_t n, float* sdf, uint8_t* valid, float* grad) {
    const DevMap& m = *pm;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double x[3];
        world_point(qp, pts, i, x);
        const QueryResult q = query_point<ST>(m, x, qp.strict != 0);
        sdf[i] = (float)q.sdf;
        valid[i] = q.valid ? 1 : 0;
        if (grad) {
            grad[3 * i] = (float)q.grad[0];
            grad[3 * i + 1] = (float)q.grad[1];
            grad[3 * i + 2] = (float)q.grad[2];
        }
    }
}

// Backward: per point dL/dx = g_i * d sdf / dx; dL/dp = R^T dL/dx; pose terms (dL/dx, x cross
// dL/dx) summed per thread, then per workgroup in a fixed order into FP64 partials.
template <int ST>
__global__ __launch_bounds__(256) void k_query_backward(const DevMap* __restrict__ pm, QueryParams qp, const float* __restrict__ pts,
                                                        int64_t n, const float* __restrict__ gsdf, float* gpts,
                                                        double* partials) {
    const DevMap& m = *pm;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double x[3];
        world_point(qp, pts, i, x);
        const QueryResult q = query_point<ST>(m, x, qp.strict != 0);
        double g[3] = {0.0, 0.0, 0.0};
        if (q.valid) {
            const double gs = (double)gsdf[i];
            for (int k = 0; k < 3; ++k) g[k] = gs * q.grad[k];
        }
        for (int r = 0; r < 3; ++r) {
            const double v = qp.identity ? g[r] : (qp.P.R[0][r] * g[0] + qp.P.R[1][r] * g[1]) + qp.P.R[2][r] * g[2];
            gpts[3 * i + r] = (float)v;
        }
        acc[0] += g[0];
        acc[1] += g[1];
        acc[2] += g[2];
        acc[3] += x[1] * g[2] - x[2] * g[1];
        acc[4] += x[2] * g[0] - x[0] * g[2];
        acc[5] += x[0] * g[1] - x[1] * g[0];
    }
    __shared__ double red[4][6];
    for (int k = 0; k < 6; ++k) acc[k] = wave_sum(acc[k]);
    const int wave = threadIdx.x >> 6;
    if (lane_id() == 0)
        for (int k = 0; k < 6; ++k) red[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        partials[(size_t)blockIdx.x * 6 + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

// Final pose-gradient sum over the workgroup partials, in a fixed order (one workgroup of 256):
// strided per-thread sums, then a tree in LDS.
__global__ __launch_bounds__(256) void k_reduce_partials(const double* __restrict__ partials, int nparts, double* out) {
    __shared__ double red[6][256];
    double s[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nparts; b += 256)
        for (int k = 0; k < 6; ++k) s[k] += partials[(size_t)b * 6 + k];
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = s[k];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

static bool make_params(const double* T, int32_t strict, QueryParams& qp) {
    qp.strict = strict;
    if (!T) {
        qp.identity = 1;
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) qp.P.R[r][c] = r == c ? 1.0 : 0.0;
            qp.P.t[r] = 0.0;
        }
        return true;
    }
    qp.identity = 0;
    return pose_from(T, qp.P);
}

}  // namespace mrh

using namespace mrh;

extern "C" mrh_status mrh_query_sdf(mrh_map* map, const float* pts_dev, int64_t n, const double* T_wq, int32_t strict,
                                    float* sdf_dev, uint8_t* valid_dev, float* grad_dev) {
    if (!map || n < 0) return MRH_ERR_INVALID_ARG;
    if (n == 0) return MRH_OK;
    if (!pts_dev || !sdf_dev || !valid_dev) return MRH_ERR_INVALID_ARG;
    QueryParams qp;
    if (!make_params(T_wq, strict, qp)) return set_error(map, MRH_ERR_INVALID_ARG, "non-finite query pose");
    const int64_t blocks = (n + 255) / 256;
    const unsigned grid = (unsigned)(blocks < 16384 ? blocks : 16384);
    launch(map, K_QUERY, [&] {
        switch (map->cfg.storage) {
            case MRH_STORE_F16: hipLaunchKernelGGL(k_query<MRH_STORE_F16>, dim3(grid), dim3(256), 0, map->stream, map->dmd, qp, pts_dev, n, sdf_dev, valid_dev, grad_dev); break;
            case MRH_STORE_BF16: hipLaunchKernelGGL(k_query<MRH_STORE_BF16>, dim3(grid), dim3(256), 0, map->stream, map->dmd, qp, pts_dev, n, sdf_dev, valid_dev, grad_dev); break;
            default: hipLaunchKernelGGL(k_query<MRH_STORE_F32>, dim3(grid), dim3(256), 0, map->stream, map->dmd, qp, pts_dev, n, sdf_dev, valid_dev, grad_dev);
        }
    });
    return check_hip(map, hipGetLastError(), "query_sdf");
}

extern "C" mrh_status mrh_query_sdf_backward(mrh_map* map, const float* pts_dev, int64_t n, const double* T_wq,
                                             int32_t strict, const float* grad_sdf_dev, float* grad_pts_dev,
                                             double grad_pose_host[6]) {
    if (!map || n < 0 || !grad_pose_host) return MRH_ERR_INVALID_ARG;
    if (n > 0 && (!pts_dev || !grad_sdf_dev || !grad_pts_dev)) return MRH_ERR_INVALID_ARG;
    QueryParams qp;
    if (!make_params(T_wq, strict, qp)) return set_error(map, MRH_ERR_INVALID_ARG, "non-finite query pose");
    for (int k = 0; k < 6; ++k) grad_pose_host[k] = 0.0;
    if (n == 0) return MRH_OK;
    const int64_t blocks = (n + 255) / 256;
    const int grid = (int)(blocks < map->partials_cap ? blocks : map->partials_cap);
    launch(map, K_QUERY_BACKWARD, [&] {
        switch (map->cfg.storage) {
            case MRH_STORE_F16: hipLaunchKernelGGL(k_query_backward<MRH_STORE_F16>, dim3(grid), dim3(256), 0, map->stream, map->dmd, qp, pts_dev, n, grad_sdf_dev, grad_pts_dev, map->partials); break;
            case MRH_STORE_BF16: hipLaunchKernelGGL(k_query_backward<MRH_STORE_BF16>, dim3(grid), dim3(256), 0, map->stream, map->dmd, qp, pts_dev, n, grad_sdf_dev, grad_pts_dev, map->partials); break;
            default: hipLaunchKernelGGL(k_query_backward<MRH_STORE_F32>, dim3(grid), dim3(256), 0, map->stream, map->dmd, qp, pts_dev, n, grad_sdf_dev, grad_pts_dev, map->partials);
        }
    });
    launch(map, K_REDUCE, [&] {
        hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(256), 0, map->stream, map->partials, grid, map->pose_out);
    });
    mrh_status st = check_hip(map, hipGetLastError(), "query_sdf_backward");
    if (st != MRH_OK) return st;
    st = check_hip(map, hipMemcpyAsync(grad_pose_host, map->pose_out, 48, hipMemcpyDeviceToHost, map->stream),
                   "query_sdf_backward");
    if (st != MRH_OK) return st;
    return check_hip(map, hipStreamSynchronize(map->stream), "query_sdf_backward");
}
