// Batched fusion of many independent maps: one frame per map per call, at most five launches in
// total, each covering every map (of its kind) through device-side tables (the per-map work is exactly that of the
// single-map path, frame hand-offs included), captured once into a HIP graph and replayed while
// the frame sizes stay fixed.
//
//   k_batch_alloc     workgroup ranges per map: depth maps get their pixel tiles then their cull
//                     workgroups, LiDAR maps one workgroup per kAllocRaysPerGroup rays; a map's
//                     last workgroup also runs its allocation-side hand-off
//   k_batch_rays      LiDAR maps: one workgroup per kRaysPerGroup rays (their recorded (ray, block)
//                     pairs in parallel: traversal and accumulation)
//   k_batch_touch     LiDAR maps: the blocks the rays touched onto the map's update queues
//   k_batch_update    the update tasks of every map of one frame kind (RGB-D or LiDAR: one launch
//                     per kind present, so that each gets the registers of its own path), strided
//                     over the concatenated task space; workgroup i also runs the update-side
//                     hand-off of map i when map i is of that kind
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "mrh_depth.h"
#include "mrh_points.h"

namespace mrh {

mrh_status ensure_lidar(mrh_map* map, int64_t n);
bool depth_size_ok(int32_t width, int32_t height);
mrh_status attach_tiles(mrh_map* map, int32_t width, int32_t height, DepthFrame& f);

constexpr int kMaxBatch = 64;

struct BatchEntry {
    int32_t kind;
    uint32_t alloc_begin, alloc_end;  // workgroups of this map in the allocation launch
    uint32_t tiles, tiles_x;          // depth: pixel tiles (cull workgroups follow them)
    uint32_t ray_begin, ray_end;      // points: workgroups of this map in the ray launch
    DepthFrame df;
    ScanParams sp;
};

// The entry whose workgroup range holds workgroup b (all lanes of the wave active; n <= 64):
// lane i tests entry i, so the ranges are read in one round trip.
__host__ __device__ inline int32_t entry_parity(const BatchEntry& e) {
    return e.kind == MRH_FRAME_DEPTH ? e.df.parity : e.sp.parity;
}

__device__ inline int entry_of(const BatchEntry* __restrict__ e, int n, uint32_t b, bool rays) {
    const int lane = lane_id();
    bool hit = false;
    if (lane < n) {
        const uint32_t lo = rays ? e[lane].ray_begin : e[lane].alloc_begin;
        const uint32_t hi = rays ? e[lane].ray_end : e[lane].alloc_end;
        hit = b >= lo && b < hi;
    }
    const unsigned long long msk = __ballot(hit);
    return msk ? __ffsll((long long)msk) - 1 : -1;
}

__global__ __launch_bounds__(256) void k_batch_alloc(const DevMap* __restrict__ maps, const BatchEntry* __restrict__ ents,
                                                     int n) {
    const int i = entry_of(ents, n, blockIdx.x, false);
    if (i < 0) return;
    const BatchEntry& e = ents[i];
    const DevMap& m = maps[i];
    const uint32_t local = blockIdx.x - e.alloc_begin;
    if (local == e.alloc_end - e.alloc_begin - 1) alloc_duties(m, e.kind == MRH_FRAME_DEPTH ? e.df.parity : e.sp.parity);
    if (e.kind == MRH_FRAME_DEPTH) {
        if (local < e.tiles) depth_alloc_tile(m, e.df, local, e.tiles_x);
        else depth_cull(m, e.df, local - e.tiles, e.alloc_end - e.alloc_begin - e.tiles);
    } else {
        points_alloc_chunk(m, e.sp, local);
    }
}

template <int ST>
__global__ __launch_bounds__(256) void k_batch_rays(const DevMap* __restrict__ maps, const BatchEntry* __restrict__ ents,
                                                    int n) {
    __shared__ unsigned long long tab[kSatSlots];
    const int i = entry_of(ents, n, blockIdx.x, true);
    if (i < 0) return;  // uniform across the workgroup
    points_ray_chunk<ST, false>(maps[i], ents[i].sp, blockIdx.x - ents[i].ray_begin, tab);
}

// After the ray launch: each LiDAR map's touched blocks onto its update queues, kBatchTouchWgs
// workgroups per table entry (those of RGB-D entries return at once).
constexpr uint32_t kBatchTouchWgs = 64;

__global__ __launch_bounds__(256) void k_batch_touch(const DevMap* __restrict__ maps, const BatchEntry* __restrict__ ents,
                                                     int n) {
    const int i = (int)(blockIdx.x / kBatchTouchWgs);
    if (i >= n || ents[i].kind != MRH_FRAME_POINTS) return;  // uniform across the workgroup
    const DevMap& m = maps[i];
    const uint32_t nb = min(m.ctr->n_blocks, m.max_blocks);
    const uint32_t per = blockDim.x * (uint32_t)kTouchPerThread;
    for (uint32_t first = (blockIdx.x % kBatchTouchWgs) * per; first < nb; first += kBatchTouchWgs * per)
        queue_touched(m, first, min(per, nb - first), ents[i].sp.parity);
}

template <int ST, int KIND>
__global__ __launch_bounds__(256) void k_batch_update(const DevMap* __restrict__ maps, const BatchEntry* __restrict__ ents,
                                                      int n) {
    // the entry table is written by the host before the launch: read through the constant address
    // space, so that a frame's descriptor (pose, intrinsics) is loaded into scalar registers
    typedef __attribute__((address_space(4))) const BatchEntry CEntry;
    const CEntry* ce = (const CEntry*)ents;
    __shared__ TaskCounts cnt[kMaxBatch];
    __shared__ uint32_t pre[kMaxBatch + 1];
    __shared__ unsigned long long wst[kMaxBatch][6];
    if ((int)blockIdx.x < n && ents[blockIdx.x].kind == KIND)
        update_duties(maps[blockIdx.x], entry_parity(ents[blockIdx.x]));
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        if (ents[i].kind != KIND) cnt[i] = TaskCounts{{0u, 0u, 0u, 0u}, 0u, 0u};
        else cnt[i] = frame_task_counts(maps[i], KIND == MRH_FRAME_DEPTH, entry_parity(ents[i]));
    }
    for (int k = threadIdx.x; k < 6 * n; k += blockDim.x) wst[k / 6][k % 6] = 0ull;
    __syncthreads();
    if (threadIdx.x == 0) {
        pre[0] = 0;
        for (int i = 0; i < n; ++i) pre[i + 1] = pre[i] + update_task_count(cnt[i]);
    }
    __syncthreads();
    const uint32_t total = pre[n];
    const uint32_t wave = uniform((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    // strided over the concatenated task space (neighbouring tasks cost alike, so striding spreads
    // the expensive runs); a wave's statistics go to per-map LDS sums, flushed once per workgroup
    int cur = -1;
    TaskStats ts;
    auto flush = [&](int i) {
        if (lane_id() == 0) {
            atomicAdd(&wst[i][0], ts.obs);
            atomicAdd(&wst[i][1], ts.fresh);
            atomicAdd(&wst[i][2], ts.merge0);
            atomicAdd(&wst[i][3], ts.merge1);
            atomicAdd(&wst[i][4], ts.merge2);
            atomicAdd(&wst[i][5], KIND == MRH_FRAME_DEPTH ? ts.obs : ts.distinct);
        }
    };
    for (uint32_t t = wave; t < total; t += nwaves) {
        // the map of task t: the largest i with pre[i] <= t
        int lo = 0, hi = n;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= t) lo = mid;
            else hi = mid;
        }
        lo = (int)uniform((uint32_t)lo);
        if (lo != cur) {
            if (cur >= 0) flush(cur);
            ts = TaskStats();
            cur = lo;
        }
        const uint32_t local = t - pre[lo];
        TaskCounts c = cnt[lo];
        for (int k = 0; k < 4; ++k) c.n[k] = uniform(c.n[k]);
        c.new_base = uniform(c.new_base);
        c.n_new = uniform(c.n_new);
        if constexpr (KIND == MRH_FRAME_DEPTH) {
            const DepthFrame fr = *(const DepthFrame*)&ce[lo].df;
            ts.add(depth_update_task<ST>(maps[lo], fr, local, c));
        } else {
            ts.add_uniform(points_update_task<ST, false>(maps[lo], local, c, ((const BatchEntry*)&ce[lo])->sp.parity, nullptr));
        }
    }
    if (cur >= 0) flush(cur);
    __syncthreads();
    const int sid[6] = {S_OBS, S_OBS_FRESH, S_MERGE0, S_MERGE1, S_MERGE2, S_DISTINCT};
    for (int k = threadIdx.x; k < 6 * n; k += blockDim.x)
        if (wst[k / 6][k % 6]) stat_add(maps[k / 6], sid[k % 6], wst[k / 6][k % 6]);
}


}  // namespace mrh

using namespace mrh;

struct mrh_batch {
    std::vector<mrh_map*> maps;
    int n = 0;
    int storage = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    DevMap* d_maps = nullptr;
    BatchEntry* d_ents = nullptr;
    BatchEntry* h_ents[2] = {nullptr, nullptr};
    hipEvent_t copied[2] = {nullptr, nullptr};
    int buf = 0;
    std::vector<uint32_t> dm_seen;  // each map's descriptor version when d_maps was last uploaded
    int32_t update_wgs = 1024, cull_wgs = 32, use_graph = 1, update_waves = 4;
    hipGraphExec_t exec = nullptr;
    std::vector<int64_t> graph_sig;  // launch geometry the graph was captured with
};

namespace mrh {

static mrh_status batch_err(mrh_batch* b, mrh_status code, const char* what) {
    return set_error(b->maps.empty() ? nullptr : b->maps[0], code, "%s", what);
}

static void drop_graph(mrh_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->graph_sig.clear();
}

// Enqueue the batched launches on stream s for the launch geometry of the current table.
static void enqueue_step(mrh_batch* b, hipStream_t s, uint32_t alloc_wgs, uint32_t ray_wgs, int depth_maps,
                         int point_maps) {
    const int n = b->n;
    if (alloc_wgs) hipLaunchKernelGGL(k_batch_alloc, dim3(alloc_wgs), dim3(256), 0, s, b->d_maps, b->d_ents, n);
    if (ray_wgs) {
        switch (b->storage) {
            case MRH_STORE_F16: hipLaunchKernelGGL(k_batch_rays<MRH_STORE_F16>, dim3(ray_wgs), dim3(256), 0, s, b->d_maps, b->d_ents, n); break;
            case MRH_STORE_BF16: hipLaunchKernelGGL(k_batch_rays<MRH_STORE_BF16>, dim3(ray_wgs), dim3(256), 0, s, b->d_maps, b->d_ents, n); break;
            default: hipLaunchKernelGGL(k_batch_rays<MRH_STORE_F32>, dim3(ray_wgs), dim3(256), 0, s, b->d_maps, b->d_ents, n);
        }
        hipLaunchKernelGGL(k_batch_touch, dim3((unsigned)n * kBatchTouchWgs), dim3(256), 0, s, b->d_maps, b->d_ents, n);
    }
    // at least one workgroup per map: workgroup i carries map i's update-side hand-off
    const dim3 ug((unsigned)(b->update_wgs > n ? b->update_wgs : n)), ub((unsigned)(64 * b->update_waves));
    auto update = [&](auto kind) {
        constexpr int K = decltype(kind)::value;
        switch (b->storage) {
            case MRH_STORE_F16: hipLaunchKernelGGL((k_batch_update<MRH_STORE_F16, K>), ug, ub, 0, s, b->d_maps, b->d_ents, n); break;
            case MRH_STORE_BF16: hipLaunchKernelGGL((k_batch_update<MRH_STORE_BF16, K>), ug, ub, 0, s, b->d_maps, b->d_ents, n); break;
            default: hipLaunchKernelGGL((k_batch_update<MRH_STORE_F32, K>), ug, ub, 0, s, b->d_maps, b->d_ents, n);
        }
    };
    if (depth_maps) update(std::integral_constant<int, MRH_FRAME_DEPTH>());
    if (point_maps) update(std::integral_constant<int, MRH_FRAME_POINTS>());
}

}  // namespace mrh

extern "C" {

mrh_status mrh_batch_create(mrh_map* const* maps, int32_t n_maps, mrh_batch** out) {
    if (!maps || !out || n_maps < 1 || n_maps > kMaxBatch) return MRH_ERR_INVALID_ARG;
    *out = nullptr;
    for (int i = 0; i < n_maps; ++i) {
        // one stream for every map: the batch enqueues on it, and the autotuner's per-map resets
        // must be ordered with the batched launches
        if (!maps[i] || maps[i]->device != maps[0]->device || maps[i]->cfg.storage != maps[0]->cfg.storage ||
            maps[i]->stream != maps[0]->stream || maps[i]->cfg.color)
            return MRH_ERR_INVALID_ARG;
        for (int j = 0; j < i; ++j)
            if (maps[j] == maps[i]) return MRH_ERR_INVALID_ARG;
    }
    mrh_batch* b = new mrh_batch();
    b->maps.assign(maps, maps + n_maps);
    b->n = n_maps;
    b->storage = maps[0]->cfg.storage;
    b->stream = maps[0]->stream;
    b->dm_seen.assign(n_maps, ~0u);
    bool ok = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc((void**)&b->d_maps, sizeof(DevMap) * n_maps) == hipSuccess &&
              hipMalloc((void**)&b->d_ents, sizeof(BatchEntry) * n_maps) == hipSuccess;
    for (int k = 0; ok && k < 2; ++k)
        ok = hipHostMalloc((void**)&b->h_ents[k], sizeof(BatchEntry) * n_maps, hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&b->copied[k], hipEventDisableTiming) == hipSuccess;
    if (ok) {
        std::vector<DevMap> dm(n_maps);
        for (int i = 0; i < n_maps; ++i) dm[i] = maps[i]->dm;
        ok = hipMemcpy(b->d_maps, dm.data(), sizeof(DevMap) * n_maps, hipMemcpyHostToDevice) == hipSuccess;
    }
    if (!ok) {
        mrh_batch_destroy(b);
        return MRH_ERR_HIP;
    }
    *out = b;
    return MRH_OK;
}

void mrh_batch_destroy(mrh_batch* b) {
    if (!b) return;
    if (b->stream || b->maps.size()) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (int k = 0; k < 2; ++k) {
        if (b->h_ents[k]) (void)hipHostFree(b->h_ents[k]);
        if (b->copied[k]) (void)hipEventDestroy(b->copied[k]);
    }
    if (b->d_maps) (void)hipFree(b->d_maps);
    if (b->d_ents) (void)hipFree(b->d_ents);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    delete b;
}

mrh_status mrh_batch_set_launch(mrh_batch* b, const int32_t params[4]) {
    if (!b || !params || params[0] < 1 || params[0] > 65536 || params[1] < 1 || params[1] > 4096 ||
        (params[3] != 1 && params[3] != 2 && params[3] != 4))
        return MRH_ERR_INVALID_ARG;
    if (params[0] != b->update_wgs || params[1] != b->cull_wgs || params[3] != b->update_waves) drop_graph(b);
    b->update_wgs = params[0];
    b->cull_wgs = params[1];
    b->use_graph = params[2] != 0;
    b->update_waves = params[3];
    return MRH_OK;
}

mrh_status mrh_batch_get_launch(const mrh_batch* b, int32_t params[4]) {
    if (!b || !params) return MRH_ERR_INVALID_ARG;
    params[0] = b->update_wgs;
    params[1] = b->cull_wgs;
    params[2] = b->use_graph;
    params[3] = b->update_waves;
    return MRH_OK;
}

mrh_status mrh_batch_integrate(mrh_batch* b, const mrh_frame* frames) {
    if (!b || !frames) return MRH_ERR_INVALID_ARG;
    const int n = b->n;
    mrh_map* m0 = b->maps[0];
    // accumulators of LiDAR maps (first scan allocates them; the device table is refreshed)
    bool refresh = false;
    for (int i = 0; i < n; ++i) {
        const mrh_frame& f = frames[i];
        if (f.kind != MRH_FRAME_NONE && f.kind != MRH_FRAME_DEPTH && f.kind != MRH_FRAME_POINTS)
            return batch_err(b, MRH_ERR_INVALID_ARG, "batch: unknown frame kind");
        if (f.kind == MRH_FRAME_POINTS && f.n > 0) {
            const mrh_status st = ensure_lidar(b->maps[i], f.n);
            if (st != MRH_OK) return st;
        }
        if (b->maps[i]->dm_version != b->dm_seen[i]) refresh = true;
    }
    if (refresh) {
        std::vector<DevMap> dm(n);
        for (int i = 0; i < n; ++i) {
            dm[i] = b->maps[i]->dm;
            b->dm_seen[i] = b->maps[i]->dm_version;
        }
        if (hipStreamSynchronize(b->stream) != hipSuccess ||
            hipMemcpy(b->d_maps, dm.data(), sizeof(DevMap) * n, hipMemcpyHostToDevice) != hipSuccess)
            return batch_err(b, MRH_ERR_HIP, "batch: map table upload");
    }
    // descriptor table and launch geometry
    const int k = b->buf;
    b->buf ^= 1;
    if (hipEventSynchronize(b->copied[k]) != hipSuccess) return batch_err(b, MRH_ERR_HIP, "batch: event");
    BatchEntry* h = b->h_ents[k];
    std::memset(h, 0, sizeof(BatchEntry) * n);
    std::vector<int64_t> sig;
    sig.push_back(b->update_wgs);
    sig.push_back(b->cull_wgs);
    sig.push_back(b->update_waves);
    uint32_t alloc_wgs = 0, ray_wgs = 0;
    int depth_maps = 0, point_maps = 0;
    for (int i = 0; i < n; ++i) {
        const mrh_frame& f = frames[i];
        BatchEntry& e = h[i];
        e.kind = f.kind;
        e.alloc_begin = alloc_wgs;
        e.ray_begin = ray_wgs;
        if (f.kind == MRH_FRAME_DEPTH) {
            if (!f.data_dev || !depth_size_ok(f.width, f.height) ||
                !make_depth_frame(b->maps[i]->cfg, f.data_dev, f.width, f.height, f.K, f.T_ws, e.df))
                return batch_err(b, MRH_ERR_INVALID_ARG, "batch: bad depth frame");
            if (attach_tiles(b->maps[i], f.width, f.height, e.df) != MRH_OK)
                return batch_err(b, MRH_ERR_OOM, "batch: tile buffer");
            e.df.parity = (int32_t)(b->maps[i]->frames & 1u);
            e.tiles_x = (uint32_t)(f.width + 15) / 16;
            e.tiles = e.tiles_x * (uint32_t)((f.height + 15) / 16);
            alloc_wgs += e.tiles + (uint32_t)b->cull_wgs;
        } else if (f.kind == MRH_FRAME_POINTS) {
            if (f.n < 0 || (f.n > 0 && !f.data_dev) || !pose_from(f.T_ws, e.sp.P))
                return batch_err(b, MRH_ERR_INVALID_ARG, "batch: bad point frame");
            e.sp.xyz = f.data_dev;
            e.sp.n = f.n;
            e.sp.parity = (int32_t)(b->maps[i]->frames & 1u);
            // at least one workgroup: it carries the map's allocation-side hand-off
            alloc_wgs += f.n > 0 ? (uint32_t)((f.n + kAllocRaysPerGroup - 1) / kAllocRaysPerGroup) : 1u;
            ray_wgs += (uint32_t)((f.n + kRaysPerGroup - 1) / kRaysPerGroup);
        }
        e.alloc_end = alloc_wgs;
        e.ray_end = ray_wgs;
        depth_maps += f.kind == MRH_FRAME_DEPTH ? 1 : 0;
        point_maps += f.kind == MRH_FRAME_POINTS ? 1 : 0;
        sig.push_back(f.kind);
        sig.push_back((int64_t)e.alloc_end);
        sig.push_back((int64_t)e.ray_end);
    }
    if (hipMemcpyAsync(b->d_ents, h, sizeof(BatchEntry) * n, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipEventRecord(b->copied[k], b->stream) != hipSuccess)
        return batch_err(b, MRH_ERR_HIP, "batch: descriptor upload");

    // every map with a frame advances one frame (its parity flips) once the step is enqueued
    auto advance = [&] {
        for (int i = 0; i < n; ++i)
            if (frames[i].kind != MRH_FRAME_NONE) b->maps[i]->frames += 1;
    };
    if (!b->use_graph) {
        launch(m0, K_BATCH_GRAPH, [&] { enqueue_step(b, b->stream, alloc_wgs, ray_wgs, depth_maps, point_maps); });
        const mrh_status st = check_hip(m0, hipGetLastError(), "batch_integrate");
        if (st == MRH_OK) advance();
        return st;
    }
    if (!b->exec || b->graph_sig != sig) {
        drop_graph(b);
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return batch_err(b, MRH_ERR_HIP, "batch: begin capture");
        enqueue_step(b, b->capture_stream, alloc_wgs, ray_wgs, depth_maps, point_maps);
        const hipError_t ce = hipStreamEndCapture(b->capture_stream, &g);
        if (ce != hipSuccess || !g) return batch_err(b, MRH_ERR_HIP, "batch: end capture");
        const hipError_t ie = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            b->exec = nullptr;
            return batch_err(b, MRH_ERR_HIP, "batch: instantiate");
        }
        b->graph_sig = sig;
    }
    launch(m0, K_BATCH_GRAPH, [&] { (void)hipGraphLaunch(b->exec, b->stream); });
    const mrh_status st = check_hip(m0, hipGetLastError(), "batch_integrate");
    if (st == MRH_OK) advance();
    return st;
}

mrh_status mrh_batch_autotune(mrh_batch* b, const mrh_frame* frames, int32_t reps, int32_t best[4]) {
    if (!b || !frames || reps < 1 || !best) return MRH_ERR_INVALID_ARG;
    static const int32_t kUpdate[] = {256, 512, 1024, 2048, 4096};
    static const int32_t kCull[] = {16, 64};
    static const int32_t kWaves[] = {1, 2, 4};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MRH_ERR_HIP;
    float best_ms = 1e30f;
    int32_t keep[4] = {b->update_wgs, b->cull_wgs, b->use_graph, b->update_waves};
    mrh_status st = MRH_OK;
    for (int32_t u : kUpdate) {
        for (int32_t c : kCull) {
            for (int32_t wv : kWaves) {
                // the same total of waves per update launch for every workgroup size
                const int32_t p[4] = {u * 4 / wv, c, 1, wv};
                mrh_batch_set_launch(b, p);
                for (int i = 0; i < b->n && st == MRH_OK; ++i) st = mrh_map_reset(b->maps[i]);
                if (st == MRH_OK) st = mrh_batch_integrate(b, frames);  // capture outside the timing
                for (int i = 0; i < b->n && st == MRH_OK; ++i) st = mrh_map_reset(b->maps[i]);
                if (st != MRH_OK) break;
                (void)hipEventRecord(e0, b->stream);
                for (int r = 0; r < reps && st == MRH_OK; ++r) st = mrh_batch_integrate(b, frames);
                (void)hipEventRecord(e1, b->stream);
                if (st != MRH_OK || hipEventSynchronize(e1) != hipSuccess) break;
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best_ms) {
                    best_ms = ms;
                    keep[0] = p[0], keep[1] = c, keep[2] = 1, keep[3] = wv;
                }
            }
            if (st != MRH_OK) break;
        }
        if (st != MRH_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == MRH_OK) st = mrh_batch_set_launch(b, keep);
    for (int i = 0; i < b->n && st == MRH_OK; ++i) st = mrh_map_reset(b->maps[i]);
    if (st == MRH_OK) st = check_hip(b->maps[0], hipStreamSynchronize(b->stream), "autotune");
    for (int k = 0; k < 4; ++k) best[k] = keep[k];
    return st;
}

}  // extern "C"
