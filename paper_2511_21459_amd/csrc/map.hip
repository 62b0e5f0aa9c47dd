// Map lifetime, reset, statistics, extraction and error reporting.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "mrh_update.h"

namespace mrh {

mrh_status set_error(mrh_map* m, mrh_status code, const char* fmt, ...) {
    if (m) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(m->err, sizeof(m->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

mrh_status check_hip(mrh_map* m, hipError_t e, const char* what) {
    if (e == hipSuccess) return MRH_OK;
    return set_error(m, e == hipErrorOutOfMemory ? MRH_ERR_OOM : MRH_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Kernels read the map descriptor through a pointer: a ~900-byte by-value argument would not fit
// the scalar register file and would be spilled into vector lanes on every launch.
mrh_status upload_descriptor(mrh_map* m) {
    ++m->dm_version;
    mrh_status st = check_hip(m, hipMemcpyAsync(m->dmd, &m->dm, sizeof(DevMap), hipMemcpyHostToDevice, m->stream),
                              "descriptor upload");
    if (st == MRH_OK) st = check_hip(m, hipStreamSynchronize(m->stream), "descriptor upload");
    return st;
}

bool pose_from(const double* T, Pose& P) {
    if (!T) return false;
    for (int i = 0; i < 16; ++i)
        if (!std::isfinite(T[i])) return false;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) P.R[r][c] = T[4 * r + c];
        P.t[r] = T[4 * r + 3];
    }
    return true;
}

// Empty table, full free stacks, zero counters.
__global__ void k_reset(const DevMap* __restrict__ pm, uint32_t n_hash) {
    const DevMap& m = *pm;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    for (uint32_t i = tid; i < n_hash; i += stride) m.hkeys[i] = kEmptyKey;
    for (int n = 0; n < m.levels; ++n) {
        const uint32_t cap = (uint32_t)m.heap_cap[n];
        for (uint32_t i = tid; i < cap; i += stride) m.stack[n][i] = cap - 1 - i;  // pops give 0, 1, 2, ...
    }
    if (tid == 0) {
        DevCounters* c = m.ctr;
        c->n_blocks = 0;
        c->pops0 = 0;
        c->error_flags.v = 0;
        for (int p = 0; p < 2; ++p) {
            c->n_prev[p] = 0;
            c->pending0[p].v = 0;
            for (int n = 0; n < 4; ++n) c->vis_n[p][n].v = 0;
        }
        for (int n = 0; n < 4; ++n) {
            c->top[n].v = n < m.levels ? m.heap_cap[n] : 0;
            c->pending[n].v = 0;
        }
    }
    if (tid < 16 * kStripes) m.ctr->frame[tid >> 4][tid & 15] = 0;
}

// Copy blocks out: keys, levels and (optionally) voxels converted from Morton to x-fastest order.
template <int ST>
__global__ void k_extract(const DevMap* __restrict__ pm, uint32_t nb, const int32_t* __restrict__ pos,
                          const int64_t* __restrict__ offsets, int32_t* keys, uint8_t* levels, float* D, uint32_t* W,
                          float* S2) {
    const DevMap& m = *pm;
    const int lane = threadIdx.x & 63;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t id = wave; id < nb; id += nwaves) {
        const int32_t row = pos[id];
        if (row < 0) continue;  // streamed out
        const uint32_t info = m.binfo[id];
        const int lvl = (int)((info >> kLevelShift) & 3u);
        if (lane == 0) {
            if (keys) {
                int32_t x, y, z;
                unpack_key(m.bkey[id], x, y, z);
                keys[3 * row] = x;
                keys[3 * row + 1] = y;
                keys[3 * row + 2] = z;
            }
            if (levels) levels[row] = (info & kNoBlockBit) ? 0xFF : (uint8_t)lvl;
        }
        if ((info & kNoBlockBit) || !(D || W || S2)) continue;
        const int mside = 8 >> lvl, nv = mside * mside * mside;
        const size_t base = (size_t)(info & kSlotMask) * nv;
        const int64_t off = offsets[row];
        for (int p = lane; p < nv; p += 64) {
            int i, j, k;
            demorton3(p, i, j, k);
            const int64_t o = off + i + mside * (j + mside * k);
            float d, s2;
            uint32_t w;
            Store<ST>::get(m, lvl, base + p, d, w, s2);
            if (D) D[o] = d;
            if (W) W[o] = w;
            if (S2) S2[o] = s2;
        }
    }
}

}  // namespace mrh

using namespace mrh;

extern "C" {

int32_t mrh_abi_version(void) { return MRH_ABI_VERSION; }

uint32_t mrh_block_hash(int32_t x, int32_t y, int32_t z, uint64_t n_hash) {
    if (n_hash == 0) return 0;
    return (uint32_t)((uint64_t)spatial_hash(x, y, z) % n_hash);
}

const char* mrh_last_error(const mrh_map* map) { return map ? map->err : "null map"; }

static void free_all(mrh_map* m) {
    stream_free(m);
    DevMap& d = m->dm;
    void* ptrs[] = {d.hkeys, d.hvals, d.bkey, d.binfo, d.bvsum, d.bvcnt, m->ctr, m->partials, m->pose_out, m->dmd,
                    m->count_dev, m->mesh_order};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (d.btouch) (void)hipFree(d.btouch);
    for (int p = 0; p < 2; ++p)
        if (d.pend0[p]) (void)hipFree(d.pend0[p]);
    if (d.rslots) (void)hipFree(d.rslots);
    if (d.rcount) (void)hipFree(d.rcount);
    if (m->tile_max) (void)hipFree(m->tile_max);
    for (int n = 0; n < 4; ++n)
        if (d.vis[n]) (void)hipFree(d.vis[n]);
    for (int n = 0; n < 4; ++n) {
        void* lp[] = {d.stack[n], d.pend[n], d.D[n], d.W[n], d.S2[n], d.C[n], d.acc_sat[n], d.acc_band[n], d.acc_s1[n], d.acc_s2[n]};
        for (void* p : lp)
            if (p) (void)hipFree(p);
    }
}

mrh_status mrh_map_create(const mrh_config* cfg, void* stream, mrh_map** out) {
    if (!cfg || !out) return MRH_ERR_INVALID_ARG;
    *out = nullptr;
    const mrh_config& c = *cfg;
    const bool pow2 = c.hash_slots > 0 && (c.hash_slots & (c.hash_slots - 1)) == 0;
    if (!(c.voxel > 0.0) || !std::isfinite(c.voxel) || c.levels < 1 || c.levels > 4 || !(c.tau > 0.0) ||
        c.min_obs < 1 || !pow2 || c.max_blocks < 1 || c.hash_slots < 2 * c.max_blocks ||
        c.hash_slots > (int64_t(1) << 31) || c.max_blocks > (int64_t(1) << 30) || !(c.var_thr >= 0.0) ||
        c.storage < MRH_STORE_F32 || c.storage > MRH_STORE_BF16 || c.form < 0 || c.form > 1 || c.color < 0 ||
        c.color > 1 || (c.color && c.min_obs < 2))
        return MRH_ERR_INVALID_ARG;
    for (int n = 0; n < 4; ++n)
        if (c.heap_blocks[n] < 0 || c.heap_blocks[n] > (int64_t)kSlotMask + 1) return MRH_ERR_INVALID_ARG;

    mrh_map* m = new mrh_map();
    m->cfg = c;
    m->stream = (hipStream_t)stream;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return MRH_ERR_HIP;
    }
    DevMap& d = m->dm;
    d.hmask = (uint32_t)(c.hash_slots - 1);
    d.max_probe = c.max_probe > 0 ? c.max_probe : 4096;
    d.max_blocks = (uint32_t)c.max_blocks;
    d.levels = c.levels;
    d.B = 8.0 * c.voxel;
    d.invB = 1.0 / d.B;
    for (int n = 0; n < 4; ++n) {
        d.nu[n] = c.voxel * (double)(1 << n);
        d.inv_nu[n] = 1.0 / d.nu[n];
    }
    d.tau = c.tau;
    d.tau_f = (float)c.tau;
    d.inv_tau_f = (float)(1.0 / c.tau);
    d.tau2_f = (float)(c.tau * c.tau);
    {
        float mf = (float)c.max_depth;
        if ((double)mf > c.max_depth) mf = std::nextafter(mf, -INFINITY);
        d.max_depth_f = mf;
    }
    d.var_thr = c.var_thr;
    d.max_depth = c.max_depth;
    d.r2lo = c.min_range * c.min_range;
    d.r2hi = c.max_range * c.max_range;
    d.min_obs = c.min_obs;
    d.form = c.form;
    d.carve = c.carve;
    d.storage = c.storage;

    mrh_status st = MRH_OK;
    auto alloc = [&](void** p, size_t bytes, const char* what) {
        if (st != MRH_OK) return;
        st = check_hip(m, hipMalloc(p, bytes ? bytes : 16), what);
    };
    const size_t nh = (size_t)c.hash_slots, nb = (size_t)c.max_blocks;
    alloc((void**)&d.hkeys, nh * 8, "hash keys");
    alloc((void**)&d.hvals, nh * 4, "hash values");
    alloc((void**)&d.bkey, nb * 8, "block keys");
    alloc((void**)&d.binfo, nb * 4, "block info");
    alloc((void**)&d.bvsum, nb * 8, "block variance sums");
    alloc((void**)&d.bvcnt, nb * 4, "block variance counts");
    alloc((void**)&m->ctr, sizeof(DevCounters), "counters");
    for (int n = 0; n < c.levels; ++n) alloc((void**)&d.vis[n], nb * 16, "visible-block lists");
    for (int n = 0; n < c.levels; ++n) {
        const int64_t cap = c.heap_blocks[n] > 0 ? c.heap_blocks[n] : c.max_blocks;
        d.heap_cap[n] = (int32_t)cap;
        const size_t nv = (size_t)cap * (size_t)(side_of(n) * side_of(n) * side_of(n));
        alloc((void**)&d.stack[n], (size_t)cap * 4, "free stack");
        if (n >= 1) alloc((void**)&d.pend[n], (size_t)cap * 4, "pending frees");
        if (n == 0)
            for (int p = 0; p < 2; ++p) alloc((void**)&d.pend0[p], (size_t)cap * 4, "pending frees");
        const size_t pb = (size_t)plane_bytes(c.storage);
        alloc((void**)&d.D[n], nv * pb, "TSDF heap");
        alloc((void**)&d.W[n], nv * pb, "weight heap");
        alloc((void**)&d.S2[n], nv * pb, "variance heap");
        if (c.color) alloc((void**)&d.C[n], nv * 12, "colour heap");
    }
    m->partials_cap = 1024;
    alloc((void**)&m->partials, (size_t)m->partials_cap * 6 * 8, "reduction partials");
    alloc((void**)&m->pose_out, 6 * 8, "pose gradient");
    alloc((void**)&m->count_dev, 8, "extraction counter");
    alloc((void**)&m->dmd, sizeof(DevMap), "map descriptor");
    d.ctr = m->ctr;
    if (st == MRH_OK) st = upload_descriptor(m);
    if (st != MRH_OK) {
        free_all(m);
        delete m;
        return st;
    }
    st = mrh_map_reset(m);
    if (st == MRH_OK) st = check_hip(m, hipStreamSynchronize(m->stream), "create");
    if (st != MRH_OK) {
        free_all(m);
        delete m;
        return st;
    }
    *out = m;
    return MRH_OK;
}

void mrh_map_destroy(mrh_map* map) {
    if (!map) return;
    (void)hipStreamSynchronize(map->stream);
    for (auto& r : map->prof) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : map->event_pool) (void)hipEventDestroy(e);
    free_all(map);
    delete map;
}

mrh_status mrh_map_reset(mrh_map* map) {
    if (!map) return MRH_ERR_INVALID_ARG;
    map->frames = map->frames_at_sync = 0;
    for (int s = 0; s < 16; ++s) map->stats_at_sync[s] = 0;
    stream_clear(map);
    const uint32_t n_hash = map->dm.hmask + 1;
    launch(map, K_RESET, [&] { hipLaunchKernelGGL(k_reset, dim3(1024), dim3(256), 0, map->stream, map->dmd, n_hash); });
    return check_hip(map, hipGetLastError(), "reset");
}

static void fill_stats(const unsigned long long* s, unsigned long long frames, uint32_t nblocks, uint32_t flags,
                       mrh_stats* out) {
    std::memset(out, 0, sizeof(*out));
    out->frames = (int64_t)frames;
    out->valid_points = (int64_t)s[S_VALID];
    out->dropped_points = (int64_t)s[S_DROPPED];
    out->new_blocks = (int64_t)s[S_NEW];
    out->observations = (int64_t)s[S_OBS];
    for (int n = 0; n < 4; ++n) out->merges[n] = (int64_t)s[S_MERGE0 + n];
    out->failed_inserts = (int64_t)s[S_FAILED];
    out->fresh_observations = (int64_t)s[S_OBS_FRESH];
    out->distinct_voxels = (int64_t)s[S_DISTINCT];
    out->candidate_keys = (int64_t)s[S_CAND];
    out->queued_blocks = (int64_t)s[S_QUEUED];
    out->blocks = (int64_t)nblocks;
    out->error_flags = flags;
}

mrh_status mrh_sync(mrh_map* map, mrh_stats* last, mrh_stats* totals) {
    if (!map) return MRH_ERR_INVALID_ARG;
    DevCounters h;
    mrh_status st = check_hip(map, hipMemcpyAsync(&h, map->ctr, sizeof(h), hipMemcpyDeviceToHost, map->stream), "sync");
    if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "sync");
    if (st != MRH_OK) return st;
    const uint32_t nb = h.n_blocks < map->dm.max_blocks ? h.n_blocks : map->dm.max_blocks;
    unsigned long long tot[16], since[16];
    for (int s = 0; s < 16; ++s) {
        tot[s] = 0;
        for (int k = 0; k < kStripes; ++k) tot[s] += h.frame[k][s];
        since[s] = tot[s] - map->stats_at_sync[s];
        map->stats_at_sync[s] = tot[s];
    }
    const uint32_t frames_since = map->frames - map->frames_at_sync;
    map->frames_at_sync = map->frames;
    const uint32_t live = nb - (uint32_t)(map->gone < nb ? map->gone : nb);
    if (last) fill_stats(since, frames_since, live, h.error_flags.v, last);
    if (totals) fill_stats(tot, map->frames, live, h.error_flags.v, totals);
    if (h.error_flags.v) {
        const uint32_t zero = 0;
        st = check_hip(map, hipMemcpyAsync(&map->ctr->error_flags.v, &zero, 4, hipMemcpyHostToDevice, map->stream),
                       "clear errors");
        if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "clear errors");
        if (st != MRH_OK) return st;
        if (h.error_flags.v & kErrTableFull)
            return set_error(map, MRH_ERR_TABLE_FULL, "hash table full (probe limit %d)", map->dm.max_probe);
        if (h.error_flags.v & kErrHeapFull) return set_error(map, MRH_ERR_HEAP_FULL, "a level heap ran out of blocks");
        return set_error(map, MRH_ERR_BLOCK_LIMIT, "more than %u blocks", map->dm.max_blocks);
    }
    return MRH_OK;
}

mrh_status mrh_extract_blocks(mrh_map* map, int32_t* keys_dev, uint8_t* levels_dev, int64_t* offsets_dev,
                              float* D_dev, uint32_t* W_dev, float* S2_dev, int64_t block_cap, int64_t voxel_cap,
                              int64_t* n_blocks, int64_t* n_voxels) {
    if (!map) return MRH_ERR_INVALID_ARG;
    DevCounters h;
    mrh_status st = check_hip(map, hipMemcpyAsync(&h, map->ctr, sizeof(h), hipMemcpyDeviceToHost, map->stream),
                              "extract");
    if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "extract");
    if (st != MRH_OK) return st;
    const uint32_t nb = h.n_blocks < map->dm.max_blocks ? h.n_blocks : map->dm.max_blocks;
    std::vector<uint32_t> info(nb);
    if (nb) {
        st = check_hip(map, hipMemcpy(info.data(), map->dm.binfo, (size_t)nb * 4, hipMemcpyDeviceToHost), "extract");
        if (st != MRH_OK) return st;
    }
    // rows of blocks streamed out to the host store are skipped; pos[id] is a row's output index
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
    if (n_blocks) *n_blocks = nout;
    if (n_voxels) *n_voxels = offs[nout];
    const bool want_blocks = keys_dev || levels_dev || offsets_dev;
    const bool want_vox = D_dev || W_dev || S2_dev;
    if (!want_blocks && !want_vox) return MRH_OK;
    if (block_cap < (int64_t)nout || (want_vox && voxel_cap < offs[nout]))
        return set_error(map, MRH_ERR_BUFFER_TOO_SMALL, "extract needs %u blocks / %lld voxels", nout,
                         (long long)offs[nout]);
    if (nout == 0) {
        if (offsets_dev) return check_hip(map, hipMemcpy(offsets_dev, offs.data(), 8, hipMemcpyHostToDevice), "extract");
        return MRH_OK;
    }
    // block voxel offsets per output row (the caller's buffer when given) and row positions per id
    int64_t* doffs = offsets_dev;
    int32_t* dpos = nullptr;
    if (!doffs) st = check_hip(map, hipMalloc((void**)&doffs, ((size_t)nout + 1) * 8), "extract offsets");
    if (st == MRH_OK) st = check_hip(map, hipMalloc((void**)&dpos, (size_t)nb * 4), "extract rows");
    if (st == MRH_OK) st = check_hip(map, hipMemcpy(doffs, offs.data(), ((size_t)nout + 1) * 8, hipMemcpyHostToDevice), "extract");
    if (st == MRH_OK) st = check_hip(map, hipMemcpy(dpos, pos.data(), (size_t)nb * 4, hipMemcpyHostToDevice), "extract");
    if (st == MRH_OK) {
        const uint32_t grid = nb / 4 + 1 < 4096 ? nb / 4 + 1 : 4096;
        switch (map->cfg.storage) {
            case MRH_STORE_F16: hipLaunchKernelGGL(k_extract<MRH_STORE_F16>, dim3(grid), dim3(256), 0, map->stream, map->dmd, nb, dpos, doffs, keys_dev, levels_dev, D_dev, W_dev, S2_dev); break;
            case MRH_STORE_BF16: hipLaunchKernelGGL(k_extract<MRH_STORE_BF16>, dim3(grid), dim3(256), 0, map->stream, map->dmd, nb, dpos, doffs, keys_dev, levels_dev, D_dev, W_dev, S2_dev); break;
            default: hipLaunchKernelGGL(k_extract<MRH_STORE_F32>, dim3(grid), dim3(256), 0, map->stream, map->dmd, nb, dpos, doffs, keys_dev, levels_dev, D_dev, W_dev, S2_dev);
        }
        st = check_hip(map, hipGetLastError(), "extract");
        if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "extract");
    }
    if (!offsets_dev && doffs) (void)hipFree(doffs);
    if (dpos) (void)hipFree(dpos);
    return st;
}

mrh_status mrh_profile_enable(mrh_map* map, int32_t on) {
    if (!map) return MRH_ERR_INVALID_ARG;
    map->profiling = on != 0;
    return MRH_OK;
}

mrh_status mrh_profile_collect(mrh_map* map, double* ms, int64_t* launches, int32_t n_kernels) {
    if (!map || n_kernels < 0 || (n_kernels > 0 && (!ms || !launches))) return MRH_ERR_INVALID_ARG;
    mrh_status st = check_hip(map, hipStreamSynchronize(map->stream), "profile");
    if (st != MRH_OK) return st;
    for (int k = 0; k < n_kernels; ++k) ms[k] = 0.0, launches[k] = 0;
    for (auto& r : map->prof) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.start, r.stop) == hipSuccess && r.kernel < n_kernels) {
            ms[r.kernel] += (double)t;
            launches[r.kernel] += 1;
        }
        map->event_pool.push_back(r.start);
        map->event_pool.push_back(r.stop);
    }
    map->prof.clear();
    return MRH_OK;
}

}  // extern "C"

namespace mrh {
hipEvent_t take_event(mrh_map* m) {
    if (!m->event_pool.empty()) {
        hipEvent_t e = m->event_pool.back();
        m->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

}  // namespace mrh
