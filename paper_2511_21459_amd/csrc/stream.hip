// Capacity-driven streaming of voxel blocks between the GPU heaps and host memory (Sec. 3.3).
//
// Streaming is deferred until the voxel heaps are filled to a threshold (the fill of the fullest
// level's heap); then every block that lies outside the current sensor region -- the camera
// frustum for RGB-D, a ball around the sensor for LiDAR -- leaves the GPU for the map's host store.
// Stored blocks that lie inside a region are brought back before that region is fused again.
// A block's region test uses its bounding sphere (centre of the block, radius half the block
// diagonal): it lies inside when the sphere meets the frustum (the conservative test of the
// update's cull) or the ball.
//
// Leaving the GPU: the block's three planes are copied out in the storage format (so a round trip
// is bit exact, variance sums included), its hash entry becomes a tombstone (lookups step over it,
// inserts never reuse it), its heap slot goes back on its level's free stack, and its table row is
// marked gone (no kernel reads a gone row).  Block ids are not reused: the block table bounds the
// number of keys ever inserted, the heaps bound the voxel memory.  All of it runs between frames on
// the map's stream, where the free stacks are in their settled state (a frame's level-0 pops are
// taken off by its own update launch; slots freed by its merges wait on the pending lists, which
// are left alone).
#include <sys/mman.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <unordered_map>
#include <vector>

#include "mrh_depth.h"

namespace mrh {

constexpr unsigned long long kTombKey = ~0ull - 1ull;  // never a packed key (those use 63 bits)

struct Region {
    int32_t kind;      // MRH_FRAME_DEPTH or MRH_FRAME_POINTS
    DepthFrame f;      // DEPTH: pose, side planes and range bound of the frustum
    double o[3];       // POINTS: sensor origin
    double radius;     // POINTS: ball radius
};

// Does the sphere of centre c and radius rb reach into the region?  Every test only grows with
// rb, so a sphere that misses the region contains no smaller sphere that reaches it.
__host__ __device__ inline bool region_meets(const Region& r, const double c[3], double rb) {
    if (r.kind == MRH_FRAME_POINTS) {
        const double d0 = c[0] - r.o[0], d1 = c[1] - r.o[1], d2 = c[2] - r.o[2];
        return __builtin_sqrt((d0 * d0 + d1 * d1) + d2 * d2) - rb <= r.radius;
    }
    const DepthFrame& f = r.f;
    const double d0 = c[0] - f.P.t[0], d1 = c[1] - f.P.t[1], d2 = c[2] - f.P.t[2];
    double x[3];
    for (int q = 0; q < 3; ++q) x[q] = (f.P.R[0][q] * d0 + f.P.R[1][q] * d1) + f.P.R[2][q] * d2;
    if (x[2] < -rb) return false;
    if (__builtin_sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) - rb > f.cull_range) return false;
    for (int p = 0; p < 4; ++p)
        if (f.plane[p][0] * x[0] + f.plane[p][1] * x[1] + f.plane[p][2] * x[2] < -rb) return false;
    return true;
}

// Bounding sphere of block (bx, by, bz) against the region (host and device evaluate the same
// expression).
__host__ __device__ inline bool region_holds(const Region& r, double B, int32_t bx, int32_t by, int32_t bz) {
    const double hb = 0.5 * B;
    const double c[3] = {(double)bx * B + hb, (double)by * B + hb, (double)bz * B + hb};
    return region_meets(r, c, B * 0.8660254037844387 * (1.0 + 1e-9) + 1e-9);
}

// Blocks outside the region, appended to per-level id lists (one atomic per level per wave).
__global__ __launch_bounds__(256) void k_stream_select(const DevMap* __restrict__ pm, Region r, uint32_t nb,
                                                       uint32_t* ids, uint32_t stride, uint32_t* counts) {
    const DevMap& m = *pm;
    const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    int level = -1;
    if (id < nb) {
        const uint32_t info = m.binfo[id];
        if (!(info & kNoBlockBit)) {
            int32_t bx, by, bz;
            unpack_key(m.bkey[id], bx, by, bz);
            if (!region_holds(r, m.B, bx, by, bz)) level = (int)((info >> kLevelShift) & 3u);
        }
    }
    for (int lv = 0; lv < 4; ++lv) {
        const unsigned long long bal = __ballot(level == lv);
        if (!bal) continue;
        const int first = __ffsll((long long)bal) - 1;
        uint32_t base = 0;
        if (lane_id() == first) base = atomicAdd(&counts[lv], (uint32_t)__popcll(bal));
        base = (uint32_t)__shfl((int)base, first);
        if (level == lv) ids[(size_t)lv * stride + base + (uint32_t)rank_in_mask(bal)] = id;
    }
}

// The three planes of a block between a heap slot and a contiguous buffer, in elements of the
// storage format (T: 32-bit for FP32, 16-bit otherwise); to_heap selects the direction.
template <typename T>
__device__ inline void copy_planes(const DevMap& m, int level, uint32_t slot, T* buf, bool to_heap) {
    const int nv = 1 << (3 * (3 - level));
    T* planes[3] = {static_cast<T*>(m.D[level]), static_cast<T*>(m.W[level]), static_cast<T*>(m.S2[level])};
    for (int p = 0; p < 3; ++p)
        for (int v = lane_id(); v < nv; v += 64) {
            T& h = planes[p][(size_t)slot * nv + v];
            if (to_heap) h = buf[p * nv + v];
            else buf[p * nv + v] = h;
        }
}

// Copy one level's selected blocks out (one wave per block: the three planes in the storage
// format, the key and the variance sums), then take them off the GPU.
__global__ __launch_bounds__(256) void k_stream_out(const DevMap* __restrict__ pm, int level, const uint32_t* __restrict__ ids,
                                                    uint32_t n, uint8_t* payload, unsigned long long* keys,
                                                    double* vsum, uint32_t* vcnt) {
    const DevMap& m = *pm;
    const uint32_t e = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (e >= n) return;
    const int lane = lane_id();
    const uint32_t id = ids[e];
    const uint32_t info = m.binfo[id];
    const uint32_t slot = info & kSlotMask;
    const int pb = plane_bytes(m.storage);
    const size_t bytes = (size_t)3 * (size_t)(1 << (3 * (3 - level))) * (size_t)pb;
    if (pb == 4) copy_planes(m, level, slot, reinterpret_cast<uint32_t*>(payload + e * bytes), false);
    else copy_planes(m, level, slot, reinterpret_cast<uint16_t*>(payload + e * bytes), false);
    if (lane == 0) {
        const unsigned long long key = m.bkey[id];
        keys[e] = key;
        vsum[e] = m.bvsum[id];
        vcnt[e] = m.bvcnt[id];
        const uint32_t h = probe_find(m, key, nullptr);
        if (h != kInvalidId) m.hkeys[h] = kTombKey;
        const int32_t at = atomicAdd(&m.ctr->top[level].v, 1);
        m.stack[level][at] = slot;
        m.binfo[id] = kNoBlockBit | kGoneBit;
    }
}

// Bring blocks back (one wave per block): insert the key (a key present already is left alone and
// reported), take a block id and a heap slot, write the planes and the variance sums (recomputed
// from the voxels when `sums` is 0).
template <int ST>
__global__ __launch_bounds__(256) void k_stream_in(const DevMap* __restrict__ pm, int level, uint32_t n,
                                                   const unsigned long long* __restrict__ keys,
                                                   const uint8_t* __restrict__ payload, const double* __restrict__ vsum,
                                                   const uint32_t* __restrict__ vcnt, int sums, uint32_t* result) {
    const DevMap& m = *pm;
    const uint32_t e = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (e >= n) return;
    const int lane = lane_id();
    const unsigned long long key = keys[e];
    uint32_t id = kInvalidId, slot = 0;
    if (lane == 0) {
        uint32_t stop = kInvalidId;
        uint32_t outcome = 0;  // 1 restored, 2 key present, 3 table full, 4 block limit, 5 heap full
        if (probe_find(m, key, &stop) != kInvalidId) {
            outcome = 2;
        } else {
            uint32_t h = 0;
            const int ins = stop == kInvalidId ? INS_FULL : probe_insert(m, key, stop, &h);
            if (ins == INS_FOUND) {
                outcome = 2;
            } else if (ins == INS_FULL) {
                outcome = 3;
                atomicOr(&m.ctr->error_flags.v, kErrTableFull);
            } else {
                id = (uint32_t)atomicAdd(reinterpret_cast<unsigned long long*>(&m.ctr->n_blocks), 1ull);
                const int32_t t = atomicSub(&m.ctr->top[level].v, 1);
                if (id >= m.max_blocks) {
                    m.hvals[h] = kInvalidId;
                    atomicOr(&m.ctr->error_flags.v, kErrBlockLimit);
                    if (t > 0) atomicAdd(&m.ctr->top[level].v, 1);
                    outcome = 4;
                    id = kInvalidId;
                } else if (t <= 0) {
                    atomicAdd(&m.ctr->top[level].v, 1);
                    atomicOr(&m.ctr->error_flags.v, kErrHeapFull);
                    m.bkey[id] = key;
                    m.binfo[id] = kNoBlockBit;
                    m.hvals[h] = id;
                    outcome = 5;
                    id = kInvalidId;
                } else {
                    slot = m.stack[level][t - 1];
                    m.bkey[id] = key;
                    m.hvals[h] = id;
                    if (m.btouch) m.btouch[id] = 0ull;
                    outcome = 1;
                }
            }
        }
        result[e] = outcome;
    }
    id = (uint32_t)__shfl((int)id, 0);
    slot = (uint32_t)__shfl((int)slot, 0);
    if (id == kInvalidId) return;
    const int nv = 1 << (3 * (3 - level));
    const int pb = plane_bytes(m.storage);
    const size_t bytes = (size_t)3 * (size_t)nv * (size_t)pb;
    uint8_t* in = const_cast<uint8_t*>(payload) + e * bytes;
    if (pb == 4) copy_planes(m, level, slot, reinterpret_cast<uint32_t*>(in), true);
    else copy_planes(m, level, slot, reinterpret_cast<uint16_t*>(in), true);
    double s = 0.0;
    uint32_t c = 0;
    if (sums) {
        s = vsum[e];
        c = vcnt[e];
    } else {
        double ps = 0.0;
        int pc = 0;
        for (int v = lane; v < nv; v += 64) {
            float D, S2;
            uint32_t W;
            Store<ST>::get(m, level, (size_t)slot * nv + v, D, W, S2);
            ps += var_term(m, W, S2);
            pc += var_count(m, W);
        }
        s = wave_sum(ps);
        c = (uint32_t)wave_sum(pc);
    }
    if (lane == 0) {
        m.bvsum[id] = s;
        m.bvcnt[id] = c;
        m.binfo[id] = slot | ((uint32_t)level << kLevelShift);
    }
}

// One stored block: its level, variance sums and the index of its planes in its level's slab.
struct HostBlock {
    int level;
    uint32_t at;    // index of its planes in its level's slab
    uint32_t bpos;  // position of its key in its bucket's key list
    uint32_t vcnt;
    double vsum;
};

// The stored planes of one level (D plane, W plane, S2 plane of a block, Morton order, storage
// format; a fixed size per level), in chunks of about 4 MiB with a free list, so that storing a
// block costs a copy rather than an allocation and the store grows without moving what it holds.
// Chunks are anonymous mappings populated when they are made (before the blocks leave the GPU),
// so the copies into them take no page faults.
struct Slab {
    static constexpr size_t kChunkBytes = (size_t)4 << 20;
    struct Chunk {
        uint8_t* p = nullptr;
        size_t len = 0;
        explicit Chunk(size_t n) : len(n) {
            void* q = mmap(nullptr, n, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_POPULATE, -1, 0);
            if (q == MAP_FAILED) throw std::bad_alloc();
            p = static_cast<uint8_t*>(q);
        }
        ~Chunk() { munmap(p, len); }
        Chunk(const Chunk&) = delete;
        Chunk& operator=(const Chunk&) = delete;
    };
    std::vector<std::unique_ptr<Chunk>> chunks;
    std::vector<uint32_t> free;
    uint32_t fresh = 0;  // blocks handed out from the chunks so far, free or not
    uint32_t per = 0;    // blocks per chunk
    size_t bytes = 0;    // per block
    void set_bytes(size_t b) {
        if (b == bytes) return;
        clear();
        bytes = b;
        per = (uint32_t)((kChunkBytes + b - 1) / b);
    }
    uint8_t* at(uint32_t i) const { return chunks[i / per]->p + (size_t)(i % per) * bytes; }
    uint32_t put(const uint8_t* src) {
        uint32_t i;
        if (!free.empty()) {
            i = free.back();
            free.pop_back();
        } else {
            if (fresh == chunks.size() * (size_t)per) chunks.push_back(std::make_unique<Chunk>((size_t)per * bytes));
            i = fresh++;
        }
        std::memcpy(at(i), src, bytes);
        return i;
    }
    // room for n more blocks without allocating in put(); false when the host is out of memory
    bool reserve(uint32_t n) {
        try {
            while ((size_t)free.size() + chunks.size() * (size_t)per - fresh < n)
                chunks.push_back(std::make_unique<Chunk>((size_t)per * bytes));
            free.reserve(free.size() + n);
        } catch (const std::bad_alloc&) {
            return false;
        }
        return true;
    }
    const uint8_t* get(uint32_t i) const { return at(i); }
    void release(uint32_t i) { free.push_back(i); }
    void clear() {
        chunks.clear();
        free.clear();
        fresh = 0;
    }
};

bool make_region(const mrh_map* map, const mrh_region* rg, Region& r) {
    std::memset(&r, 0, sizeof(r));
    r.kind = rg->kind;
    if (rg->kind == MRH_FRAME_POINTS) {
        Pose P;
        if (!pose_from(rg->T_ws, P) || !std::isfinite(rg->radius) || rg->radius < 0.0) return false;
        for (int k = 0; k < 3; ++k) r.o[k] = P.t[k];
        r.radius = rg->radius;
        return true;
    }
    if (rg->kind != MRH_FRAME_DEPTH || !depth_size_ok(rg->width, rg->height)) return false;
    return make_depth_frame(map->cfg, nullptr, rg->width, rg->height, rg->K, rg->T_ws, r.f);
}

// Fill of the voxel memory: each level's heap is its own share of it, so the fullest heap decides
// (slots not on a free stack count as used, frees still pending among them).
double heap_usage(const mrh_map* map, const DevCounters& h) {
    double worst = 0.0;
    for (int n = 0; n < map->cfg.levels; ++n) {
        const double cap = (double)map->dm.heap_cap[n];
        const double freeb = h.top[n].v > 0 ? (double)h.top[n].v : 0.0;
        if (cap > 0.0) worst = std::max(worst, (cap - freeb) / cap);
    }
    return worst;
}

// Host conversions of the storage formats, the same arithmetic as the device codecs (decoding
// multiplies in FP32 in the same order; encoding rounds to nearest even).  Stored blocks are
// decoded only for inspection; blocks loaded from outside are encoded with an exact division in
// place of the device's reciprocal for the variance, which can differ from a device store by one
// 16-bit ulp.
// voxel p of a block of nv voxels held as three planes in `buf`
inline void host_decode(int st, const uint8_t* buf, int nv, int p, float tau_f, float tau2_f, float& D, uint32_t& W,
                        float& S2) {
    if (st == MRH_STORE_F32) {
        std::memcpy(&D, buf + 4 * (size_t)p, 4);
        std::memcpy(&W, buf + 4 * ((size_t)nv + p), 4);
        std::memcpy(&S2, buf + 4 * (2 * (size_t)nv + p), 4);
        return;
    }
    uint16_t d, w, v;
    std::memcpy(&d, buf + 2 * (size_t)p, 2);
    std::memcpy(&w, buf + 2 * ((size_t)nv + p), 2);
    std::memcpy(&v, buf + 2 * (2 * (size_t)nv + p), 2);
    D = (st == MRH_STORE_F16 ? h_f16(d) : h_bf16(d)) * tau_f;
    W = st == MRH_STORE_F16 ? (uint32_t)w : (uint32_t)h_f16(w);
    S2 = h_f16(v) * (float)W * tau2_f;
}

inline void host_encode(int st, uint8_t* buf, int nv, int p, float tau_f, float inv_tau_f, float tau2_f, float D,
                        uint32_t W, float S2) {
    (void)tau_f;
    if (st == MRH_STORE_F32) {
        std::memcpy(buf + 4 * (size_t)p, &D, 4);
        std::memcpy(buf + 4 * ((size_t)nv + p), &W, 4);
        std::memcpy(buf + 4 * (2 * (size_t)nv + p), &S2, 4);
        return;
    }
    const float x = D * inv_tau_f;
    const uint16_t d = st == MRH_STORE_F16 ? h_to_f16(x) : h_to_bf16(x);
    const uint16_t w = st == MRH_STORE_F16 ? (uint16_t)(W < 65535u ? W : 65535u) : h_to_f16((float)(W < 65504u ? W : 65504u));
    const uint32_t wd = st == MRH_STORE_F16 ? (uint32_t)w : (uint32_t)h_f16(w);
    const uint16_t v = h_to_f16(wd > 0 ? S2 / ((float)wd * tau2_f) : 0.f);
    std::memcpy(buf + 2 * (size_t)p, &d, 2);
    std::memcpy(buf + 2 * ((size_t)nv + p), &w, 2);
    std::memcpy(buf + 2 * (2 * (size_t)nv + p), &v, 2);
}

// device staging buffers, grown on demand
template <typename T>
mrh_status grow(mrh_map* map, T** p, size_t& cap, size_t need, const char* what) {
    if (need <= cap) return MRH_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    cap = 0;
    const mrh_status st = check_hip(map, hipMalloc((void**)p, need * sizeof(T)), what);
    if (st == MRH_OK) cap = need;
    return st;
}

}  // namespace mrh

using namespace mrh;

// Host store and staging of a map (created on first use).
// The host store is indexed by buckets of kBucketSide^3 blocks, so that bringing a region back
// tests the buckets' bounding spheres first and only the blocks of the buckets that reach it.
constexpr int kBucketShift = 5;
constexpr int kBucketSide = 1 << kBucketShift;

inline unsigned long long bucket_of(unsigned long long key) {
    int32_t x, y, z;
    unpack_key(key, x, y, z);
    return pack_key(x >> kBucketShift, y >> kBucketShift, z >> kBucketShift);
}

struct mrh_stream_state {
    std::unordered_map<unsigned long long, HostBlock> store;
    Slab slabs[4];
    std::unordered_map<unsigned long long, std::vector<unsigned long long>> buckets;  // bucket -> keys
    uint32_t* ids = nullptr;
    size_t ids_cap = 0;
    uint32_t* counts = nullptr;
    uint8_t* payload = nullptr;
    size_t payload_cap = 0;
    unsigned long long* keys = nullptr;
    size_t keys_cap = 0;
    double* vsum = nullptr;
    size_t vsum_cap = 0;
    uint32_t* vcnt = nullptr;
    size_t vcnt_cap = 0;
    uint32_t* result = nullptr;
    size_t result_cap = 0;
    uint8_t* stage = nullptr;  // pinned host staging of the payloads copied in and out
    size_t stage_cap = 0;
};

namespace mrh {
mrh_stream_state* stream_state(mrh_map* map) {
    if (!map->stream_st) map->stream_st = new mrh_stream_state();
    return map->stream_st;
}

void stream_free(mrh_map* map) {
    mrh_stream_state* s = map->stream_st;
    if (!s) return;
    void* ptrs[] = {s->ids, s->counts, s->payload, s->keys, s->vsum, s->vcnt, s->result};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (s->stage) (void)hipHostFree(s->stage);
    delete s;
    map->stream_st = nullptr;
}

void stream_clear(mrh_map* map) {
    if (map->stream_st) {
        map->stream_st->store.clear();
        map->stream_st->buckets.clear();
        for (Slab& sl : map->stream_st->slabs) sl.clear();
    }
    map->gone = 0;
}

static mrh_status read_counters(mrh_map* map, DevCounters& h) {
    mrh_status st = check_hip(map, hipMemcpyAsync(&h, map->ctr, sizeof(h), hipMemcpyDeviceToHost, map->stream), "stream");
    if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "stream");
    return st;
}

// The pinned staging buffer, grown to at least `bytes` (its contents are not kept).
static mrh_status grow_stage(mrh_map* map, mrh_stream_state* S, size_t bytes) {
    if (bytes <= S->stage_cap) return MRH_OK;
    if (S->stage) {
        mrh_status st = check_hip(map, hipHostFree(S->stage), "stream staging");
        S->stage = nullptr;
        S->stage_cap = 0;
        if (st != MRH_OK) return st;
    }
    const size_t cap = bytes + bytes / 4;
    mrh_status st = check_hip(map, hipHostMalloc((void**)&S->stage, cap, hipHostMallocDefault), "stream staging");
    if (st == MRH_OK) S->stage_cap = cap;
    else S->stage = nullptr;
    return st;
}

// Upload blocks (keys, levels, plane words, optional sums) and run the insert kernel per level.
static mrh_status stream_insert(mrh_map* map, const std::vector<unsigned long long>& keys, const std::vector<int>& levels,
                                const std::vector<const uint8_t*>& words, const std::vector<double>& vsum,
                                const std::vector<uint32_t>& vcnt, int sums, std::vector<uint32_t>& outcome) {
    mrh_stream_state* S = stream_state(map);
    const size_t n = keys.size();
    outcome.assign(n, 0);
    if (n == 0) return MRH_OK;
    const int pb = plane_bytes(map->cfg.storage);
    for (int lv = 0; lv < map->cfg.levels; ++lv) {
        std::vector<size_t> sel;
        for (size_t i = 0; i < n; ++i)
            if (levels[i] == lv) sel.push_back(i);
        if (sel.empty()) continue;
        const size_t cnt = sel.size();
        const size_t wpb = (size_t)3 * (size_t)(side_of(lv) * side_of(lv) * side_of(lv)) * (size_t)pb;  // bytes
        mrh_status st = grow(map, &S->payload, S->payload_cap, cnt * wpb, "stream payload");
        if (st == MRH_OK) st = grow(map, &S->keys, S->keys_cap, cnt, "stream keys");
        if (st == MRH_OK) st = grow(map, &S->vsum, S->vsum_cap, cnt, "stream sums");
        if (st == MRH_OK) st = grow(map, &S->vcnt, S->vcnt_cap, cnt, "stream counts");
        if (st == MRH_OK) st = grow(map, &S->result, S->result_cap, cnt, "stream results");
        if (st == MRH_OK) st = grow_stage(map, S, cnt * wpb);
        if (st != MRH_OK) return st;
        std::vector<unsigned long long> hk(cnt);
        std::vector<double> hs(cnt, 0.0);
        std::vector<uint32_t> hc(cnt, 0u);
        for (size_t q = 0; q < cnt; ++q) {
            const size_t i = sel[q];
            std::memcpy(S->stage + q * wpb, words[i], wpb);
            hk[q] = keys[i];
            if (sums) hs[q] = vsum[i], hc[q] = vcnt[i];
        }
        st = check_hip(map, hipMemcpyAsync(S->payload, S->stage, cnt * wpb, hipMemcpyHostToDevice, map->stream), "stream in");
        if (st == MRH_OK) st = check_hip(map, hipMemcpyAsync(S->keys, hk.data(), cnt * 8, hipMemcpyHostToDevice, map->stream), "stream in");
        if (st == MRH_OK) st = check_hip(map, hipMemcpyAsync(S->vsum, hs.data(), cnt * 8, hipMemcpyHostToDevice, map->stream), "stream in");
        if (st == MRH_OK) st = check_hip(map, hipMemcpyAsync(S->vcnt, hc.data(), cnt * 4, hipMemcpyHostToDevice, map->stream), "stream in");
        if (st != MRH_OK) return st;
        const unsigned grid = (unsigned)((cnt + 3) / 4);
        switch (map->cfg.storage) {
            case MRH_STORE_F16: hipLaunchKernelGGL(k_stream_in<MRH_STORE_F16>, dim3(grid), dim3(256), 0, map->stream, map->dmd, lv, (uint32_t)cnt, S->keys, S->payload, S->vsum, S->vcnt, sums, S->result); break;
            case MRH_STORE_BF16: hipLaunchKernelGGL(k_stream_in<MRH_STORE_BF16>, dim3(grid), dim3(256), 0, map->stream, map->dmd, lv, (uint32_t)cnt, S->keys, S->payload, S->vsum, S->vcnt, sums, S->result); break;
            default: hipLaunchKernelGGL(k_stream_in<MRH_STORE_F32>, dim3(grid), dim3(256), 0, map->stream, map->dmd, lv, (uint32_t)cnt, S->keys, S->payload, S->vsum, S->vcnt, sums, S->result);
        }
        st = check_hip(map, hipGetLastError(), "stream in");
        std::vector<uint32_t> res(cnt);
        if (st == MRH_OK) st = check_hip(map, hipMemcpyAsync(res.data(), S->result, cnt * 4, hipMemcpyDeviceToHost, map->stream), "stream in");
        if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "stream in");
        if (st != MRH_OK) return st;
        for (size_t q = 0; q < cnt; ++q) outcome[sel[q]] = res[q];
    }
    // blocks that came back are not new to the next frame: its new-block id range starts after them
    DevCounters h;
    mrh_status st = read_counters(map, h);
    if (st != MRH_OK) return st;
    const uint32_t nb = h.n_blocks < map->dm.max_blocks ? h.n_blocks : map->dm.max_blocks;
    return check_hip(map, hipMemcpyAsync(&map->ctr->n_prev[map->frames & 1u], &nb, 4, hipMemcpyHostToDevice, map->stream),
                     "stream in");
}
}  // namespace mrh

extern "C" {

mrh_status mrh_heap_usage(mrh_map* map, double* frac) {
    if (!map || !frac) return MRH_ERR_INVALID_ARG;
    DevCounters h;
    const mrh_status st = read_counters(map, h);
    if (st != MRH_OK) return st;
    *frac = heap_usage(map, h);
    return MRH_OK;
}

mrh_status mrh_stream_out(mrh_map* map, const mrh_region* region, double threshold, int64_t* n_out) {
    if (!map || !region || !n_out || !(threshold >= 0.0)) return MRH_ERR_INVALID_ARG;
    if (map->cfg.color) return set_error(map, MRH_ERR_INVALID_ARG, "maps with colour are not streamed");
    *n_out = 0;
    Region r;
    if (!make_region(map, region, r)) return set_error(map, MRH_ERR_INVALID_ARG, "invalid streaming region");
    DevCounters h;
    mrh_status st = read_counters(map, h);
    if (st != MRH_OK) return st;
    if (heap_usage(map, h) < threshold) return MRH_OK;
    const uint32_t nb = h.n_blocks < map->dm.max_blocks ? h.n_blocks : map->dm.max_blocks;
    if (nb == 0) return MRH_OK;
    mrh_stream_state* S = stream_state(map);
    st = grow(map, &S->ids, S->ids_cap, (size_t)4 * nb, "stream ids");
    if (st == MRH_OK && !S->counts) st = check_hip(map, hipMalloc((void**)&S->counts, 16), "stream counts");
    if (st == MRH_OK) st = check_hip(map, hipMemsetAsync(S->counts, 0, 16, map->stream), "stream");
    if (st != MRH_OK) return st;
    hipLaunchKernelGGL(k_stream_select, dim3((nb + 255) / 256), dim3(256), 0, map->stream, map->dmd, r, nb, S->ids, nb, S->counts);
    uint32_t cnt[4] = {0, 0, 0, 0};
    st = check_hip(map, hipGetLastError(), "stream select");
    if (st == MRH_OK) st = check_hip(map, hipMemcpyAsync(cnt, S->counts, 16, hipMemcpyDeviceToHost, map->stream), "stream");
    if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "stream");
    if (st != MRH_OK) return st;
    try {
        S->store.reserve(S->store.size() + (size_t)cnt[0] + cnt[1] + cnt[2] + cnt[3]);
    } catch (const std::bad_alloc&) {
        return set_error(map, MRH_ERR_OOM, "host store: out of memory");
    }
    const int pb = plane_bytes(map->cfg.storage);
    for (int lv = 0; lv < map->cfg.levels; ++lv) {
        const uint32_t n = cnt[lv];
        if (!n) continue;
        const size_t wpb = (size_t)3 * (size_t)(side_of(lv) * side_of(lv) * side_of(lv)) * (size_t)pb;  // bytes
        st = grow(map, &S->payload, S->payload_cap, (size_t)n * wpb, "stream payload");
        if (st == MRH_OK) st = grow(map, &S->keys, S->keys_cap, n, "stream keys");
        if (st == MRH_OK) st = grow(map, &S->vsum, S->vsum_cap, n, "stream sums");
        if (st == MRH_OK) st = grow(map, &S->vcnt, S->vcnt_cap, n, "stream counts");
        if (st == MRH_OK) st = grow_stage(map, S, (size_t)n * wpb);
        if (st != MRH_OK) return st;
        // host room first: the launch below takes the blocks off the GPU
        Slab& sl = S->slabs[lv];
        sl.set_bytes(wpb);
        if (!sl.reserve(n)) return set_error(map, MRH_ERR_OOM, "host store: out of memory for %u blocks", n);
        hipLaunchKernelGGL(k_stream_out, dim3((n + 3) / 4), dim3(256), 0, map->stream, map->dmd, lv,
                           S->ids + (size_t)lv * nb, n, S->payload, S->keys, S->vsum, S->vcnt);
        std::vector<unsigned long long> hk(n);
        std::vector<double> hs(n);
        std::vector<uint32_t> hc(n);
        st = check_hip(map, hipGetLastError(), "stream out");
        if (st == MRH_OK) st = check_hip(map, hipMemcpyAsync(S->stage, S->payload, (size_t)n * wpb, hipMemcpyDeviceToHost, map->stream), "stream out");
        if (st == MRH_OK) st = check_hip(map, hipMemcpyAsync(hk.data(), S->keys, (size_t)n * 8, hipMemcpyDeviceToHost, map->stream), "stream out");
        if (st == MRH_OK) st = check_hip(map, hipMemcpyAsync(hs.data(), S->vsum, (size_t)n * 8, hipMemcpyDeviceToHost, map->stream), "stream out");
        if (st == MRH_OK) st = check_hip(map, hipMemcpyAsync(hc.data(), S->vcnt, (size_t)n * 4, hipMemcpyDeviceToHost, map->stream), "stream out");
        if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "stream out");
        if (st != MRH_OK) return st;
        for (uint32_t q = 0; q < n; ++q) {
            auto ins = S->store.try_emplace(hk[q]);
            HostBlock& hb = ins.first->second;
            if (!ins.second) {
                S->slabs[hb.level].release(hb.at);  // a stored copy the GPU block replaces
            } else {
                std::vector<unsigned long long>& bv = S->buckets[bucket_of(hk[q])];
                hb.bpos = (uint32_t)bv.size();
                bv.push_back(hk[q]);
            }
            hb.level = lv;
            hb.at = sl.put(S->stage + (size_t)q * wpb);
            hb.vsum = hs[q];
            hb.vcnt = hc[q];
        }
        map->gone += n;
        *n_out += n;
    }
    return MRH_OK;
}

mrh_status mrh_stream_in(mrh_map* map, const mrh_region* region, int64_t* n_in) {
    if (!map || !region || !n_in) return MRH_ERR_INVALID_ARG;
    if (map->cfg.color) return set_error(map, MRH_ERR_INVALID_ARG, "maps with colour are not streamed");
    *n_in = 0;
    Region r;
    if (!make_region(map, region, r)) return set_error(map, MRH_ERR_INVALID_ARG, "invalid streaming region");
    mrh_stream_state* S = stream_state(map);
    std::vector<unsigned long long> keys;
    std::vector<int> levels;
    std::vector<const uint8_t*> words;
    std::vector<double> vsum;
    std::vector<uint32_t> vcnt;
    const double B = map->dm.B, bb = B * kBucketSide;
    const double brad = bb * 0.8660254037844387 * (1.0 + 1e-9) + 1e-9;
    for (const auto& bk : S->buckets) {
        int32_t cx, cy, cz;
        unpack_key(bk.first, cx, cy, cz);
        const double c[3] = {((double)cx + 0.5) * bb, ((double)cy + 0.5) * bb, ((double)cz + 0.5) * bb};
        if (!region_meets(r, c, brad)) continue;
        for (unsigned long long key : bk.second) {
            int32_t x, y, z;
            unpack_key(key, x, y, z);
            if (!region_holds(r, B, x, y, z)) continue;
            const HostBlock& hb = S->store.at(key);
            keys.push_back(key);
            levels.push_back(hb.level);
            words.push_back(S->slabs[hb.level].get(hb.at));
            vsum.push_back(hb.vsum);
            vcnt.push_back(hb.vcnt);
        }
    }
    if (keys.empty()) return MRH_OK;
    // the free slots must hold every block brought back
    DevCounters h;
    mrh_status st = read_counters(map, h);
    if (st != MRH_OK) return st;
    int64_t need[4] = {0, 0, 0, 0};
    for (int lv : levels) need[lv]++;
    for (int lv = 0; lv < map->cfg.levels; ++lv)
        if (need[lv] > (int64_t)h.top[lv].v)
            return set_error(map, MRH_ERR_HEAP_FULL, "level %d heap has %d free blocks, %lld to bring back", lv,
                             h.top[lv].v, (long long)need[lv]);
    if ((int64_t)h.n_blocks + (int64_t)keys.size() > (int64_t)map->dm.max_blocks)
        return set_error(map, MRH_ERR_BLOCK_LIMIT, "block table full");
    std::vector<uint32_t> outcome;
    st = stream_insert(map, keys, levels, words, vsum, vcnt, 1, outcome);
    if (st != MRH_OK) return st;
    for (size_t i = 0; i < keys.size(); ++i) {
        // restored blocks leave the store; a key present on the GPU keeps its stored copy
        if (outcome[i] == 1) {
            auto it = S->store.find(keys[i]);
            const HostBlock hb = it->second;
            S->store.erase(it);
            S->slabs[hb.level].release(hb.at);
            // take the key out of its bucket: the bucket's last key moves into its place
            auto b = S->buckets.find(bucket_of(keys[i]));
            std::vector<unsigned long long>& bv = b->second;
            const unsigned long long last = bv.back();
            bv.pop_back();
            if (last != keys[i]) {
                bv[hb.bpos] = last;
                S->store.find(last)->second.bpos = hb.bpos;
            }
            if (bv.empty()) S->buckets.erase(b);
            ++*n_in;
        }
    }
    return MRH_OK;
}

mrh_status mrh_store_extract(mrh_map* map, int32_t* keys, uint8_t* levels, int64_t* offsets, float* D, uint32_t* W,
                             float* S2, int64_t block_cap, int64_t voxel_cap, int64_t* n_blocks, int64_t* n_voxels) {
    if (!map) return MRH_ERR_INVALID_ARG;
    std::vector<std::pair<unsigned long long, const HostBlock*>> blocks;
    if (map->stream_st)
        for (const auto& kv : map->stream_st->store) blocks.emplace_back(kv.first, &kv.second);
    std::sort(blocks.begin(), blocks.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    int64_t nv = 0;
    for (const auto& b : blocks) nv += (int64_t)side_of(b.second->level) * side_of(b.second->level) * side_of(b.second->level);
    if (n_blocks) *n_blocks = (int64_t)blocks.size();
    if (n_voxels) *n_voxels = nv;
    const bool want_vox = D || W || S2;
    if (!(keys || levels || offsets || want_vox)) return MRH_OK;
    if (block_cap < (int64_t)blocks.size() || (want_vox && voxel_cap < nv))
        return set_error(map, MRH_ERR_BUFFER_TOO_SMALL, "store holds %zu blocks / %lld voxels", blocks.size(), (long long)nv);
    const int st = map->cfg.storage;
    const float tau_f = map->dm.tau_f, tau2_f = map->dm.tau2_f;
    int64_t off = 0;
    if (offsets) offsets[0] = 0;
    for (size_t i = 0; i < blocks.size(); ++i) {
        const HostBlock& hb = *blocks[i].second;
        int32_t x, y, z;
        unpack_key(blocks[i].first, x, y, z);
        if (keys) keys[3 * i] = x, keys[3 * i + 1] = y, keys[3 * i + 2] = z;
        if (levels) levels[i] = (uint8_t)hb.level;
        const int ms = side_of(hb.level), nvb = ms * ms * ms;
        for (int p = 0; p < nvb && want_vox; ++p) {
            int a, b, c;
            demorton3(p, a, b, c);
            const int64_t o = off + a + ms * (b + ms * c);
            float d, s2;
            uint32_t w;
            host_decode(st, map->stream_st->slabs[hb.level].get(hb.at), nvb, p, tau_f, tau2_f, d, w, s2);
            if (D) D[o] = d;
            if (W) W[o] = w;
            if (S2) S2[o] = s2;
        }
        off += nvb;
        if (offsets) offsets[i + 1] = off;
    }
    return MRH_OK;
}

mrh_status mrh_load_blocks(mrh_map* map, int64_t n, const int32_t* keys, const uint8_t* levels, const float* D,
                           const uint32_t* W, const float* S2, int64_t* n_loaded) {
    if (!map || n < 0 || !n_loaded || (n > 0 && (!keys || !levels || !D || !W || !S2))) return MRH_ERR_INVALID_ARG;
    if (map->cfg.color) return set_error(map, MRH_ERR_INVALID_ARG, "maps with colour are not streamed");
    *n_loaded = 0;
    if (n == 0) return MRH_OK;
    const int st = map->cfg.storage, pb = plane_bytes(st);
    const float tau_f = map->dm.tau_f, inv_tau_f = map->dm.inv_tau_f, tau2_f = map->dm.tau2_f;
    std::vector<unsigned long long> hk((size_t)n);
    std::vector<int> hl((size_t)n);
    std::vector<std::vector<uint8_t>> bufs((size_t)n);
    std::vector<const uint8_t*> ptrs((size_t)n);
    int64_t need[4] = {0, 0, 0, 0};
    int64_t off = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int lv = levels[i];
        if (lv >= map->cfg.levels) return set_error(map, MRH_ERR_INVALID_ARG, "block %lld: level %d", (long long)i, lv);
        for (int k = 0; k < 3; ++k)
            if (keys[3 * i + k] < -(int32_t)kKeyLimit || keys[3 * i + k] > (int32_t)kKeyLimit)
                return set_error(map, MRH_ERR_INVALID_ARG, "block %lld: key out of range", (long long)i);
        hk[(size_t)i] = pack_key(keys[3 * i], keys[3 * i + 1], keys[3 * i + 2]);
        hl[(size_t)i] = lv;
        need[lv]++;
        const int ms = side_of(lv), nvb = ms * ms * ms;
        bufs[(size_t)i].assign((size_t)3 * nvb * pb, 0);
        for (int p = 0; p < nvb; ++p) {
            int a, b, c;
            demorton3(p, a, b, c);
            const int64_t o = off + a + ms * (b + ms * c);
            host_encode(st, bufs[(size_t)i].data(), nvb, p, tau_f, inv_tau_f, tau2_f, D[o], W[o], S2[o]);
        }
        ptrs[(size_t)i] = bufs[(size_t)i].data();
        off += nvb;
    }
    DevCounters h;
    mrh_status s = read_counters(map, h);
    if (s != MRH_OK) return s;
    for (int lv = 0; lv < map->cfg.levels; ++lv)
        if (need[lv] > (int64_t)h.top[lv].v)
            return set_error(map, MRH_ERR_HEAP_FULL, "level %d heap has %d free blocks, %lld to load", lv, h.top[lv].v,
                             (long long)need[lv]);
    if ((int64_t)h.n_blocks + n > (int64_t)map->dm.max_blocks) return set_error(map, MRH_ERR_BLOCK_LIMIT, "block table full");
    std::vector<double> vs((size_t)n, 0.0);
    std::vector<uint32_t> vc((size_t)n, 0u);
    std::vector<uint32_t> outcome;
    s = stream_insert(map, hk, hl, ptrs, vs, vc, 0, outcome);
    if (s != MRH_OK) return s;
    for (uint32_t o : outcome) *n_loaded += o == 1;
    return MRH_OK;
}

mrh_status mrh_store_info(mrh_map* map, int64_t* n_blocks, int64_t* n_voxels, int64_t* bytes) {
    if (!map) return MRH_ERR_INVALID_ARG;
    int64_t nb = 0, nv = 0, by = 0;
    if (map->stream_st)
        for (const auto& kv : map->stream_st->store) {
            ++nb;
            nv += (int64_t)side_of(kv.second.level) * side_of(kv.second.level) * side_of(kv.second.level);
            by += (int64_t)map->stream_st->slabs[kv.second.level].bytes + 24;
        }
    if (n_blocks) *n_blocks = nb;
    if (n_voxels) *n_voxels = nv;
    if (bytes) *bytes = by;
    return MRH_OK;
}

}  // extern "C"
