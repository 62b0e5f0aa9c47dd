// Internal layout and device helpers of the mrhash library (gfx950).
//
// Map layout in HBM (all arrays allocated once at map creation):
//   hash table   hkeys[u64 n_hash] packed block keys (EMPTY = all ones), hvals[u32 n_hash] block id
//   block table  bkey[u64 max_blocks], binfo[u32] = heap slot | level << 27 | NEW | NOBLOCK,
//                bvsum[f64] = sum over voxels with W >= min_obs of S2 / W, bvcnt[u32] = their count
//   heaps        per level n: D, W, S2 planes of heap_blocks[n] blocks x (8 >> n)^3 voxels, voxels
//                of a block in Morton (Z) order so the 2x2x2 children of a coarse voxel are
//                contiguous; a free stack of slot indices and a pending-free list per level
//   counters     DevCounters (block count, stack tops, stats, latched error flags)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "mrhash.h"

namespace mrh {

constexpr unsigned long long kEmptyKey = ~0ull;
constexpr uint32_t kInvalidId = 0xFFFFFFFFu;
constexpr int64_t kKeyLimit = (int64_t(1) << 20) - 2;  // |block coordinate| bound for segment ends

constexpr uint32_t kSlotMask = (1u << 27) - 1;
constexpr int kLevelShift = 27;
constexpr uint32_t kNewBit = 1u << 29;
constexpr uint32_t kGoneBit = 1u << 30;     // block streamed out to the host store (always with NOBLOCK)
constexpr uint32_t kNoBlockBit = 1u << 31;

constexpr uint32_t kErrTableFull = 1u, kErrHeapFull = 2u, kErrBlockLimit = 4u;

// per-frame statistics slots (u64)
enum Stat { S_VALID = 0, S_DROPPED, S_NEW, S_OBS, S_MERGE0, S_MERGE1, S_MERGE2, S_MERGE3, S_FAILED, S_OBS_FRESH,
            S_DISTINCT, S_CAND, S_QUEUED, S_COUNT };

// Per-frame statistics are accumulated in kStripes cache-line-sized stripes (a workgroup adds to
// the stripe of its index) so that atomics from different workgroups rarely meet on one line; the
// end-of-frame kernel sums the stripes.
constexpr int kStripes = 32;

// A counter alone on a 128-byte line.  Device-scope atomics are performed beyond the per-XCD L2s,
// so plain loads of a line that other waves update atomically keep missing; counters that are
// updated atomically each get their own line, apart from the ones every wave reads.
template <typename T>
struct alignas(128) Line {
    T v;
};

// A frame runs as an allocation launch and an update launch (LiDAR: allocation, rays, update);
// there is no separate end-of-frame launch.  The hand-offs between frames cross kernel boundaries
// only: per-frame counts are double-buffered by frame parity p (the host alternates it), each
// launch reads the buffer of its own frame and clears or fills the other one; slots freed at
// level n >= 1 are returned to their stacks by the next allocation launch (which never pops those
// levels), level-0 slots by one workgroup of the next update launch (which never pops level 0).
struct alignas(128) DevCounters {
    // allocation word: one 64-bit atomic adds k to both halves for k new blocks
    uint32_t n_blocks;   // block ids handed out (keys inserted), low half
    uint32_t pops0;      // level-0 slots taken by this frame's new blocks, high half
    uint32_t n_prev[2];  // per parity: min(n_blocks, max_blocks) when the frame started (ids >= are new)
    Line<uint32_t> error_flags;
    Line<int32_t> top[4];
    Line<uint32_t> pending[4];   // slots freed at level n >= 1 this frame (entry 0 unused)
    Line<uint32_t> pending0[2];  // slots freed at level 0, per parity
    Line<uint32_t> vis_n[2][4];  // per parity: blocks queued for the update, per level
    unsigned long long frame[kStripes][16];  // statistics since the reset, in stripes
};

// Everything a kernel needs to find the map; passed by value as a kernel argument.
struct DevMap {
    unsigned long long* hkeys;
    uint32_t* hvals;
    uint32_t hmask;
    int32_t max_probe;
    unsigned long long* bkey;
    uint32_t* binfo;
    double* bvsum;
    uint32_t* bvcnt;
    uint32_t max_blocks;
    int32_t levels;
    DevCounters* ctr;
    uint32_t* stack[4];
    uint32_t* pend[4];      // level n >= 1 frees (entry 0 unused)
    uint32_t* pend0[2];     // level-0 frees, per parity
    int32_t heap_cap[4];
    void* D[4];   // per level, plane of the storage format (see mrh_store.h)
    void* W[4];
    void* S2[4];
    float* C[4];  // per level, colour RGB float32 x 3 per voxel (maps created with colour; else null)
    // LiDAR per-frame accumulators, parallel to the heaps (zero between frames):
    // saturated (+tau) observation counts, band observation counts, and the exact integer sums of
    // the band observations' fixed-point values q = rint(d 2^24) and of q^2
    uint32_t* acc_sat[4];
    uint32_t* acc_band[4];
    unsigned long long* acc_s1[4];
    unsigned long long* acc_s2[4];
    // per block: the lane groups rays touched this frame, bit g = the voxels lane g of the update
    // owns (level 0: Morton positions 8g .. 8g+7, level 1: position g; levels 2, 3: bit 0)
    unsigned long long* btouch;
    // LiDAR: the hash slots of the block keys each ray's walk visits, in walk order (rcap_k per ray,
    // written by the allocation launch; kInvalidId for a key the full table could not take), and
    // their count per ray (may exceed rcap_k)
    uint32_t* rslots;
    uint32_t* rcount;
    int32_t rcap_k;
    uint4* vis[4];     // per level: the blocks the update visits this frame, (id, info, key lo, key hi)
    double B, invB;
    double nu[4], inv_nu[4];
    double tau, var_thr;
    double max_depth, r2lo, r2hi;
    float tau_f, inv_tau_f, tau2_f;
    float max_depth_f;  // largest float <= max_depth: (double)d <= max_depth  <=>  d <= max_depth_f
    int32_t min_obs, form, carve, storage;
};

// An update-queue entry carries the block's table row, so an update task needs no second lookup.
__device__ inline uint4 make_entry(uint32_t id, uint32_t info, unsigned long long key) {
    return make_uint4(id, info, (uint32_t)key, (uint32_t)(key >> 32));
}

__device__ inline unsigned long long entry_key(const uint4& e) {
    return (unsigned long long)e.z | ((unsigned long long)e.w << 32);
}

// Values the caller knows to be equal on every active lane, moved to scalar registers (a wave waits
// for a loaded value here, so loaded values that are needed late are better left alone).
__device__ inline uint32_t uniform(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ inline uint4 uniform(const uint4& e) { return make_uint4(uniform(e.x), uniform(e.y), uniform(e.z), uniform(e.w)); }

// world <- sensor rigid transform, FP64
struct Pose {
    double R[3][3];
    double t[3];
};

// ---------------------------------------------------------------------------------------------
// keys and the spatial hash (Eq. 4)
// ---------------------------------------------------------------------------------------------

__host__ __device__ inline unsigned long long pack_key(int64_t x, int64_t y, int64_t z) {
    const unsigned long long b = 1ull << 20;
    return ((unsigned long long)(x + (int64_t)b) & 0x1FFFFFull) |
           (((unsigned long long)(y + (int64_t)b) & 0x1FFFFFull) << 21) |
           (((unsigned long long)(z + (int64_t)b) & 0x1FFFFFull) << 42);
}

__host__ __device__ inline void unpack_key(unsigned long long k, int32_t& x, int32_t& y, int32_t& z) {
    x = (int32_t)(k & 0x1FFFFFull) - (1 << 20);
    y = (int32_t)((k >> 21) & 0x1FFFFFull) - (1 << 20);
    z = (int32_t)((k >> 42) & 0x1FFFFFull) - (1 << 20);
}

// Eq. 4: (x p1 xor y p2 xor z p3) in 32-bit unsigned arithmetic; the table size is a power of two
// so "mod n_hash" is a mask of the low bits.
__host__ __device__ inline uint32_t spatial_hash(int32_t x, int32_t y, int32_t z) {
    return ((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349669u) ^ ((uint32_t)z * 83492791u);
}

__device__ inline uint32_t home_slot(unsigned long long key, uint32_t mask) {
    int32_t x, y, z;
    unpack_key(key, x, y, z);
    return spatial_hash(x, y, z) & mask;
}

// Read-only probe.  Returns the slot holding `key`, or kInvalidId; *stop gets the first EMPTY
// slot met (where an insert would start) or kInvalidId when the probe limit was reached.
__device__ inline uint32_t probe_find(const DevMap& m, unsigned long long key, uint32_t* stop) {
    uint32_t h = home_slot(key, m.hmask);
    for (int p = 0; p < m.max_probe; ++p) {
        const unsigned long long k = __hip_atomic_load(&m.hkeys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == key) return h;
        if (k == kEmptyKey) {
            if (stop) *stop = h;
            return kInvalidId;
        }
        h = (h + 1) & m.hmask;
    }
    if (stop) *stop = kInvalidId;
    return kInvalidId;
}

// Block id of `key`, or kInvalidId when absent (or inserted without a block id).
__device__ inline uint32_t find_block(const DevMap& m, unsigned long long key) {
    const uint32_t h = probe_find(m, key, nullptr);
    return h == kInvalidId ? kInvalidId : m.hvals[h];
}

enum InsertResult { INS_FOUND = 0, INS_NEW = 1, INS_FULL = 2 };

// Lock-free linear-probing insert from slot `start` (the first EMPTY slot a read-only probe met).
// Keys are only ever written by this CAS, so the returned old value decides every race.  The CAS
// at `start` is issued without re-reading the slot (the probe saw it empty; the CAS's old value
// says whether it still was), which saves a round trip on every new key.  *slot receives the slot
// holding the key (inserted or found).
__device__ inline int probe_insert(const DevMap& m, unsigned long long key, uint32_t start, uint32_t* slot) {
    uint32_t h = start;
    for (int p = 0; p < m.max_probe; ++p) {
        const unsigned long long k =
            p == 0 ? kEmptyKey : __hip_atomic_load(&m.hkeys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == key) {
            *slot = h;
            return INS_FOUND;
        }
        if (k == kEmptyKey) {
            const unsigned long long old = atomicCAS(&m.hkeys[h], kEmptyKey, key);
            if (old == kEmptyKey || old == key) {
                *slot = h;
                return old == key ? INS_FOUND : INS_NEW;
            }
        }
        h = (h + 1) & m.hmask;
    }
    return INS_FULL;
}

// ---------------------------------------------------------------------------------------------
// wave helpers (wave64)
// ---------------------------------------------------------------------------------------------

__device__ inline int lane_id() { return __lane_id(); }

__device__ inline int rank_in_mask(unsigned long long mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

__device__ inline unsigned long long shfl_u64(unsigned long long v, int src) {
    const uint32_t lo = __shfl((int)(uint32_t)v, src), hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
}

// Cross-lane moves by DPP (gfx9): each lane reads a lane of its own 16-lane row, in the VALU, with
// no LDS round trip.  XOR1 / XOR2 read lane i ^ 1 / i ^ 2 (quad permutations), HALF_MIRROR lane
// 7 - i of its group of 8, ROW_MIRROR lane 15 - i of its row.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppRowMirror = 0x140;

template <int CTRL>
__device__ inline int dpp(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ inline uint32_t dpp(uint32_t v) {
    return (uint32_t)dpp<CTRL>((int)v);
}
template <int CTRL>
__device__ inline float dpp(float v) {
    return __builtin_bit_cast(float, dpp<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ inline unsigned long long dpp(unsigned long long v) {
    const uint32_t lo = dpp<CTRL>((uint32_t)v), hi = dpp<CTRL>((uint32_t)(v >> 32));
    return ((unsigned long long)hi << 32) | lo;
}
template <int CTRL>
__device__ inline double dpp(double v) {
    return __builtin_bit_cast(double, dpp<CTRL>(__builtin_bit_cast(unsigned long long, v)));
}

// Sum over each group of 8 consecutive lanes, on every lane of the group, associated as
// ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7)) whatever the lane (after the pairs and the quads
// every lane of a quad holds the same value, so the mirror lane 7 - i brings the other quad's sum).
template <typename T>
__device__ inline T group8_sum(T v) {
    v += dpp<kDppXor1>(v);
    v += dpp<kDppXor2>(v);
    return v + dpp<kDppHalfMirror>(v);
}
// The same for min / max (exact, so the order does not matter).
template <typename T>
__device__ inline T group8_min(T v) {
    v = min(v, dpp<kDppXor1>(v));
    v = min(v, dpp<kDppXor2>(v));
    return min(v, dpp<kDppHalfMirror>(v));
}
template <typename T>
__device__ inline T group8_max(T v) {
    v = max(v, dpp<kDppXor1>(v));
    v = max(v, dpp<kDppXor2>(v));
    return max(v, dpp<kDppHalfMirror>(v));
}
__device__ inline double group8_fmin(double v) {
    v = __builtin_fmin(v, dpp<kDppXor1>(v));
    v = __builtin_fmin(v, dpp<kDppXor2>(v));
    return __builtin_fmin(v, dpp<kDppHalfMirror>(v));
}

// Sum over each 16-lane row (group8_sum, then the row's other half by the row mirror).
template <typename T>
__device__ inline T row16_sum(T v) {
    v = group8_sum(v);
    return v + dpp<kDppRowMirror>(v);
}

template <typename T>
__device__ inline T lane_value(T v, int lane);
template <>
__device__ inline int lane_value(int v, int lane) {
    return __builtin_amdgcn_readlane(v, lane);
}
template <>
__device__ inline float lane_value(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}
template <>
__device__ inline unsigned long long lane_value(unsigned long long v, int lane) {
    return ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane) << 32) |
           (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
}
template <>
__device__ inline double lane_value(double v, int lane) {
    return __builtin_bit_cast(double, lane_value(__builtin_bit_cast(unsigned long long, v), lane));
}

// Sums over the wave (all 64 lanes active), returned wave-uniform: the four row sums, then
// (r0 + r1) + (r2 + r3).
template <typename T>
__device__ inline T wave_sum_rows(T v) {
    v = row16_sum(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}
__device__ inline double wave_sum(double v) { return wave_sum_rows(v); }
__device__ inline int wave_sum(int v) { return wave_sum_rows(v); }
__device__ inline unsigned long long wave_sum(unsigned long long v) { return wave_sum_rows(v); }

__device__ inline float wave_max(float v) {
    v = __builtin_fmaxf(v, dpp<kDppXor1>(v));
    v = __builtin_fmaxf(v, dpp<kDppXor2>(v));
    v = __builtin_fmaxf(v, dpp<kDppHalfMirror>(v));
    v = __builtin_fmaxf(v, dpp<kDppRowMirror>(v));
    return __builtin_fmaxf(__builtin_fmaxf(lane_value(v, 0), lane_value(v, 16)),
                           __builtin_fmaxf(lane_value(v, 32), lane_value(v, 48)));
}

// add to a per-frame statistic (striped by workgroup)
__device__ inline void stat_add(const DevMap& m, int s, unsigned long long v) {
    if (v) atomicAdd(&m.ctr->frame[(blockIdx.x + 7u * blockIdx.y) % kStripes][s], v);
}

// Morton (Z-order) position of voxel (i, j, k) inside a block of side 8 >> level, x lowest bit.
__host__ __device__ inline int morton3(int i, int j, int k) {
    int p = 0;
    for (int b = 0; b < 3; ++b) p |= (((i >> b) & 1) << (3 * b)) | (((j >> b) & 1) << (3 * b + 1)) | (((k >> b) & 1) << (3 * b + 2));
    return p;
}

__host__ __device__ inline void demorton3(int p, int& i, int& j, int& k) {
    i = j = k = 0;
    for (int b = 0; b < 3; ++b) {
        i |= ((p >> (3 * b)) & 1) << b;
        j |= ((p >> (3 * b + 1)) & 1) << b;
        k |= ((p >> (3 * b + 2)) & 1) << b;
    }
}

// ---------------------------------------------------------------------------------------------
// canonical FP64 geometry shared by the kernels of this library (the library is built with
// -ffp-contract=off: every expression is evaluated exactly as written)
// ---------------------------------------------------------------------------------------------

__device__ inline void pose_apply(const Pose& P, const double p[3], double out[3]) {
    for (int r = 0; r < 3; ++r) out[r] = ((P.R[r][0] * p[0] + P.R[r][1] * p[1]) + P.R[r][2] * p[2]) + P.t[r];
}

__device__ inline void unit_direction(const double p[3], const double o[3], double n[3]) {
    const double v0 = p[0] - o[0], v1 = p[1] - o[1], v2 = p[2] - o[2];
    const double inv = 1.0 / __builtin_sqrt((v0 * v0 + v1 * v1) + v2 * v2);
    n[0] = v0 * inv;
    n[1] = v1 * inv;
    n[2] = v2 * inv;
}

__device__ inline bool segment_in_range(const double a[3], const double e[3], double invB) {
    for (int k = 0; k < 3; ++k) {
        const double fa = __builtin_floor(a[k] * invB), fe = __builtin_floor(e[k] * invB);
        if (!(__builtin_fabs(fa) <= (double)kKeyLimit && __builtin_fabs(fe) <= (double)kKeyLimit)) return false;
    }
    return true;
}

// Amanatides-Woo walk over unit cells of a lattice scaled by inv_cell: half-open cells, start in
// the cell of a, step across the nearest boundary (lowest axis on ties), stop past e.  Boundary
// parameters are recomputed from the cell index at every step.
// One axis of a walk: position A (in cell units), cell c, step direction, inverse extent and the
// parameter of the next boundary.
__device__ inline void walk_axis(double a, double e, double inv_cell, double& A, int64_t& c, int& st, double& iD,
                                 double& t, int64_t& guard) {
    A = a * inv_cell;
    const double E = e * inv_cell;
    c = (int64_t)__builtin_floor(A);
    const double dv = E - A;
    const int64_t fe = (int64_t)__builtin_floor(E);
    guard += fe > c ? fe - c : c - fe;
    if (dv > 0.0) {
        st = 1;
        iD = 1.0 / dv;
        t = ((double)(c + 1) - A) * iD;
    } else if (dv < 0.0) {
        st = -1;
        iD = 1.0 / dv;
        t = ((double)c - A) * iD;
    } else {
        st = 0;
        iD = 0.0;
        t = __builtin_inf();
    }
}

// Amanatides-Woo walk over unit cells of a lattice scaled by inv_cell: half-open cells, start in
// the cell of a, step across the nearest boundary (lowest axis on ties), stop past e.  Boundary
// parameters are recomputed from the cell index at every step.  Kept in scalars (no indexed
// arrays) so the walk state lives in registers.
struct Walk {
    double A0, A1, A2, iD0, iD1, iD2, t0, t1, t2;
    int64_t c0, c1, c2;
    int s0, s1, s2;
    int64_t guard;

    __device__ inline void init(const double a[3], const double e[3], double inv_cell) {
        guard = 3;
        walk_axis(a[0], e[0], inv_cell, A0, c0, s0, iD0, t0, guard);
        walk_axis(a[1], e[1], inv_cell, A1, c1, s1, iD1, t1, guard);
        walk_axis(a[2], e[2], inv_cell, A2, c2, s2, iD2, t2, guard);
    }
    // advance to the next cell; false once the walk is over
    __device__ inline bool next() {
        if (guard <= 0) return false;
        --guard;
        double tm = t0;
        int k = 0;
        if (t1 < tm) tm = t1, k = 1;
        if (t2 < tm) tm = t2, k = 2;
        if (!(tm <= 1.0)) return false;
        if (k == 0) {
            c0 += s0;
            t0 = ((double)(c0 + (s0 > 0 ? 1 : 0)) - A0) * iD0;
        } else if (k == 1) {
            c1 += s1;
            t1 = ((double)(c1 + (s1 > 0 ? 1 : 0)) - A1) * iD1;
        } else {
            c2 += s2;
            t2 = ((double)(c2 + (s2 > 0 ? 1 : 0)) - A2) * iD2;
        }
        return true;
    }
};

// ---------------------------------------------------------------------------------------------
// host-side helpers shared by the entry points
// ---------------------------------------------------------------------------------------------

inline int side_of(int level) { return 8 >> level; }

// kernel ids reported by mrh_profile_collect (same order as MRH_KERNEL_* in the public header)
enum KernelId { K_RESET = MRH_KERNEL_RESET, K_ALLOC_DEPTH = MRH_KERNEL_ALLOC_DEPTH, K_INTEGRATE_DEPTH = MRH_KERNEL_INTEGRATE_DEPTH,
                K_FINALIZE = MRH_KERNEL_FINALIZE, K_ALLOC_POINTS = MRH_KERNEL_ALLOC_POINTS, K_RAYS = MRH_KERNEL_RAYS,
                K_APPLY_POINTS = MRH_KERNEL_APPLY_POINTS, K_QUERY = MRH_KERNEL_QUERY, K_QUERY_BACKWARD = MRH_KERNEL_QUERY_BACKWARD,
                K_REDUCE = MRH_KERNEL_REDUCE, K_BATCH_ALLOC = MRH_KERNEL_BATCH_ALLOC, K_BATCH_RAYS = MRH_KERNEL_BATCH_RAYS,
                K_BATCH_UPDATE = MRH_KERNEL_BATCH_UPDATE, K_BATCH_FINALIZE = MRH_KERNEL_BATCH_FINALIZE,
                K_BATCH_GRAPH = MRH_KERNEL_BATCH_GRAPH, K_MESH = MRH_KERNEL_MESH, K_COLOR = MRH_KERNEL_COLOR };

// one profiled launch: kernel id and its bracketing events on the map's stream
struct ProfRec {
    int kernel;
    hipEvent_t start, stop;
};

}  // namespace mrh

struct mrh_stream_state;  // host store and staging of the streaming calls

struct mrh_map {
    mrh_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    mrh::DevMap dm{};
    mrh::DevMap* dmd = nullptr;  // device copy of dm, passed to every kernel by pointer
    mrh::DevCounters* ctr = nullptr;
    double* partials = nullptr;  // query-backward per-workgroup FP64 partial sums
    double* pose_out = nullptr;  // 6 doubles, final reduction
    unsigned long long* count_dev = nullptr;  // one device counter for the extraction calls
    uint32_t* mesh_order = nullptr;  // the mesh launch's block ids by level (4 regions) and 4 counts
    size_t mesh_order_cap = 0;
    int32_t partials_cap = 0;
    bool lidar_ready = false;    // accumulators allocated
    int64_t rcap_n = 0;          // rays the per-ray block-key buffers hold
    uint32_t frames = 0;         // frames enqueued since the last reset (parity of the next = frames & 1)
    uint32_t frames_at_sync = 0;
    unsigned long long stats_at_sync[16] = {0};
    uint32_t dm_version = 0;     // bumped whenever the device copy of dm is rewritten
    float* tile_max = nullptr;   // per 16 x 16 pixel tile of the current depth frame: largest valid depth
    size_t tile_cap = 0;
    bool profiling = false;      // bracket every launch with events (mrh_profile_enable)
    std::vector<mrh::ProfRec> prof;
    std::vector<hipEvent_t> event_pool;
    mrh_stream_state* stream_st = nullptr;
    uint64_t gone = 0;           // blocks streamed out since the last reset (their ids stay used)
    char err[512] = {0};
};

namespace mrh {
mrh_status set_error(mrh_map* m, mrh_status code, const char* fmt, ...);
mrh_status check_hip(mrh_map* m, hipError_t e, const char* what);
bool pose_from(const double* T, Pose& P);
mrh_status upload_descriptor(mrh_map* m);
void stream_free(mrh_map* m);   // release the host store and the streaming staging buffers
void stream_clear(mrh_map* m);  // empty the host store (map reset)

// Launch through `fn` (a callable that enqueues one kernel on m->stream), bracketed by events
// when profiling is on.
hipEvent_t take_event(mrh_map* m);
template <typename F>
inline void launch(mrh_map* m, int kernel, F&& fn) {
    if (!m->profiling) {
        fn();
        return;
    }
    hipEvent_t a = take_event(m), b = take_event(m);
    (void)hipEventRecord(a, m->stream);
    fn();
    (void)hipEventRecord(b, m->stream);
    m->prof.push_back({kernel, a, b});
}
}  // namespace mrh
