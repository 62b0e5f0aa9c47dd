// LiDAR fusion work units (Sec. 3.1 "3D Point Cloud", Eq. 1; Eq. 3 and Eq. 5; Sec. 3.2.1),
// shared by the single-map kernels (points.hip) and the batched kernels (batch.hip).
//
//   points_alloc_chunk  32 rays: validity, segment [o, p + tau n] (carving) or the band
//                       [p - tau n, p + tau n], walk over the block lattice, wave-deduplicated
//                       insert, and the record of the hash slots of each ray's blocks in walk order
//   points_ray_chunk    8 rays: their recorded (ray, block) pairs in parallel; inside each block a
//                       walk over the block's own voxel lattice; each crossed voxel gets
//                       clip((p - x) . n, -tau, tau).
//                       Saturated observations (+tau) only bump an integer count; the others add
//                       their fixed-point value q = rint(d 2^24) and its square q^2 to exact integer
//                       sums, so the accumulation is order-independent and needs no read of the
//                       voxel's state; the update forms the sums of (d - D) and (d - D)^2 from them.
//                       A block's first touch in the scan queues it on its level's list.
//   points_update_task  one queued level-0 or level-1 block (a wave), or 8 level-2 / 64 level-3
//                       blocks per wave: each voxel's scan statistics merge into its state (W' =
//                       W + n, D' = D + s1 / W', S2' = S2 + s2 - s1^2 / W', the batch form of Eq. 3
//                       and Eq. 5), then the block variance bookkeeping and the merging criterion
#pragma once

#include "mrh_update.h"

namespace mrh {

constexpr double kS1Scale = 16777216.0;         // 2^24 per metre: q = rint(d 2^24), |q| <= tau 2^24
constexpr double kS2Scale = 281474976710656.0;  // 2^48 per square metre: the sum of q^2

struct ScanParams {
    int32_t parity;  // the frame's parity (selects the double-buffered per-frame counts)
    Pose P;
    const float* xyz;  // device points, sensor frame, [n][3]
    int64_t n;
};

__device__ inline bool point_segment(const DevMap& m, const ScanParams& sp, int64_t i, double a[3], double e[3],
                                     double p[3], double n[3]) {
    const float* __restrict__ xyz = sp.xyz;
    const double ps[3] = {(double)xyz[3 * i], (double)xyz[3 * i + 1], (double)xyz[3 * i + 2]};
    if (!(__builtin_isfinite(ps[0]) && __builtin_isfinite(ps[1]) && __builtin_isfinite(ps[2]))) return false;
    const double r2 = (ps[0] * ps[0] + ps[1] * ps[1]) + ps[2] * ps[2];
    if (!(r2 >= m.r2lo && r2 <= m.r2hi)) return false;
    pose_apply(sp.P, ps, p);
    unit_direction(p, sp.P.t, n);
    for (int k = 0; k < 3; ++k) {
        a[k] = m.carve ? sp.P.t[k] : p[k] - m.tau * n[k];
        e[k] = p[k] + m.tau * n[k];
    }
    return true;
}

// Rays per wave of the allocation launch (each ray's block walk is a serial chain of lookups, so
// waves carry few rays and many waves are in flight), and per 256-thread workgroup.
constexpr int kAllocRaysPerWave = 8;
constexpr int kAllocRaysPerGroup = 4 * kAllocRaysPerWave;

// Allocation for rays chunk * kAllocRaysPerGroup ..: the block walk of each ray, the wave-
// deduplicated insert of the keys, and the record of the hash slot of each ray's keys in walk order.  A ray's walk
// is a chain of lookups, so it advances kAllocRound blocks at a time: the ray's lane runs that many
// DDA steps (arithmetic only) and leaves the keys in LDS, and then every lane of the wave claims one
// key (ray = lane / kAllocRound, step = lane % kAllocRound): one round of probes and inserts for the
// 64 keys instead of one per step.
constexpr int kAllocRound = 64 / kAllocRaysPerWave;

__device__ inline void points_alloc_chunk(const DevMap& m, const ScanParams& sp, uint32_t chunk) {
    __shared__ unsigned long long skeys[4][64];  // per wave: kAllocRaysPerWave rays x kAllocRound keys
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6);
    const bool mine = lane < kAllocRaysPerWave;
    const int64_t r0 = (int64_t)chunk * kAllocRaysPerGroup + (int64_t)wv * kAllocRaysPerWave;
    const int64_t i = r0 + lane;
    double a[3], e[3], p[3], nn[3];
    const bool ok = mine && i < sp.n && point_segment(m, sp, i, a, e, p, nn);
    const unsigned long long vmask = __ballot(ok);
    const bool in_range = ok && segment_in_range(a, e, m.invB);
    const unsigned long long dmask = __ballot(ok && !in_range);
    if (lane == 0) {
        stat_add(m, S_VALID, (unsigned long long)__popcll(vmask));
        stat_add(m, S_DROPPED, (unsigned long long)__popcll(dmask));
    }
    Walk w;
    if (in_range) w.init(a, e, m.invB);
    bool active = in_range;
    uint32_t steps = 0;
    // the ray and walk step whose key this lane claims in each round
    const int ray = lane / kAllocRound, k = lane % kAllocRound;
    const int64_t ri = r0 + ray;
    uint32_t* rs = m.rslots + (size_t)(ri < sp.n ? ri : 0) * (size_t)m.rcap_k;
    while (__ballot(active)) {
        uint32_t cnt = 0;
        if (mine) {
            for (int s = 0; s < kAllocRound; ++s) {
                unsigned long long key = 0ull;
                if (active) {
                    key = pack_key(w.c0, w.c1, w.c2);
                    ++cnt;
                    active = w.next();
                }
                skeys[wv][lane * kAllocRound + s] = key;
            }
        }
        // LDS operations of one wave complete in order; the fences keep the compiler from moving
        // the read above the other lanes' writes
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const unsigned long long key = skeys[wv][lane];
        const uint32_t rcnt = (uint32_t)__shfl((int)cnt, ray), rsteps = (uint32_t)__shfl((int)steps, ray);
        const bool has = (uint32_t)k < rcnt;
        uint32_t slot = kInvalidId;
        const bool is_new = claim_keys(m, has, key, &slot);
        register_new(m, is_new, key, slot);
        if (has && rsteps + (uint32_t)k < (uint32_t)m.rcap_k) rs[rsteps + (uint32_t)k] = slot;
        steps += cnt;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (mine && i < sp.n) m.rcount[i] = steps;
    const int ncand = wave_sum(mine ? (int)steps : 0);
    if (lane == 0 && ncand) stat_add(m, S_CAND, (unsigned long long)ncand);
}

// Saturated (+tau) observations of voxels near the sensor origin are first counted in a
// workgroup-private LDS table: every ray of a scan starts at the origin, so near it thousands of
// rays cross the same voxels and direct global atomics on those addresses serialise.  The table is
// flushed with one global atomic per distinct voxel once the workgroup's rays are done.  The counts
// are integers, so the result equals adding them one at a time.  An entry is (key + 1) << 32 | count
// with key = level << 30 | heap position; keys are never removed while rays run.
constexpr int kSatBits = 9;
constexpr int kSatSlots = 1 << kSatBits;
constexpr double kSatNear2 = 1024.0;  // voxels within 32 voxel edges of the origin use the table

__device__ inline void sat_table_clear(unsigned long long* tab) {
    for (int k = threadIdx.x; k < kSatSlots; k += blockDim.x) tab[k] = 0ull;
    __syncthreads();
}

// Count one saturated observation in the table; false when the voxel must go to global memory
// (heap position too large for a key, or no free entry within 8 probes).
__device__ inline bool sat_table_add(unsigned long long* tab, int level, size_t at) {
    if (at >= (size_t)((1u << 30) - 1u)) return false;
    const uint32_t key = (((uint32_t)level << 30) | (uint32_t)at) + 1u;
    uint32_t h = (key * 2654435761u) >> (32 - kSatBits);
    for (int p = 0; p < 8; ++p) {
        const uint32_t k = (uint32_t)(__hip_atomic_load(&tab[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) >> 32);
        if (k == key) {
            atomicAdd(&tab[h], 1ull);
            return true;
        }
        if (k == 0u) {
            const unsigned long long old = atomicCAS(&tab[h], 0ull, ((unsigned long long)key << 32) | 1ull);
            if (old == 0ull) return true;
            if ((uint32_t)(old >> 32) == key) {
                atomicAdd(&tab[h], 1ull);
                return true;
            }
        }
        h = (h + 1) & (kSatSlots - 1);
    }
    return false;
}

// All threads of the workgroup: add the table's counts to the global accumulators.
__device__ inline void sat_table_flush(const DevMap& m, unsigned long long* tab) {
    __syncthreads();
    for (int k = threadIdx.x; k < kSatSlots; k += blockDim.x) {
        const unsigned long long e = tab[k];
        if (e) {
            const uint32_t code = (uint32_t)(e >> 32) - 1u;
            atomicAdd(&m.acc_sat[code >> 30][code & ((1u << 30) - 1u)], (uint32_t)e);
        }
    }
}

// Accumulate one observation d of the voxel at heap position `at` of `level`; `near` routes a
// saturated one through the workgroup table.  A band observation adds 1, q and q^2 (q its
// fixed-point value): exact integers, fire-and-forget atomics with no dependent load.
__device__ inline void accumulate(const DevMap& m, int level, size_t at, double d, bool near, unsigned long long* tab) {
    if (d >= m.tau) {
        if (!(near && sat_table_add(tab, level, at))) atomicAdd(&m.acc_sat[level][at], 1u);
        return;
    }
    const long long q = (long long)__builtin_rint(d * kS1Scale);
    atomicAdd(&m.acc_band[level][at], 1u);
    atomicAdd(&m.acc_s1[level][at], (unsigned long long)q);
    atomicAdd(&m.acc_s2[level][at], (unsigned long long)(q * q));
}

// The block walk restricted to one block: the segment is clipped to the block's box, the walk
// starts in the (clamped) cell of the clipped entry point and steps on the block's own lattice of
// side^3 voxels until it leaves the block or passes the clipped exit parameter.
struct BoxWalk {
    double A0, A1, A2, iD0, iD1, iD2, t0, t1, t2, tout;
    int c0, c1, c2, s0, s1, s2, side;

    __device__ static inline void axis(double a, double e, double ob, double inv_nu, int side, double& A, double& D,
                                       double& iD, int& st, double& tin, double& tout) {
        A = (a - ob) * inv_nu;
        const double El = (e - ob) * inv_nu;
        D = El - A;
        if (D != 0.0) {
            iD = 1.0 / D;
            const double nearb = D > 0.0 ? 0.0 : (double)side;
            const double farb = D > 0.0 ? (double)side : 0.0;
            const double ta = (nearb - A) * iD;
            const double tb = (farb - A) * iD;
            if (ta > tin) tin = ta;
            if (tb < tout) tout = tb;
            st = D > 0.0 ? 1 : -1;
        } else {
            iD = 0.0;
            st = 0;
        }
    }
    __device__ static inline void start(double A, double D, double iD, int st, double tin, int side, int& c, double& t) {
        double fl = __builtin_floor(A + tin * D);
        if (fl < 0.0) fl = 0.0;
        if (fl > (double)(side - 1)) fl = (double)(side - 1);
        c = (int)fl;
        t = st != 0 ? ((double)(c + (st > 0 ? 1 : 0)) - A) * iD : __builtin_inf();
    }
    __device__ inline void init(const double a[3], const double e[3], const int64_t b[3], double B, double inv_nu,
                                int side_) {
        side = side_;
        double D0, D1, D2, tin = 0.0;
        tout = 1.0;
        axis(a[0], e[0], (double)b[0] * B, inv_nu, side, A0, D0, iD0, s0, tin, tout);
        axis(a[1], e[1], (double)b[1] * B, inv_nu, side, A1, D1, iD1, s1, tin, tout);
        axis(a[2], e[2], (double)b[2] * B, inv_nu, side, A2, D2, iD2, s2, tin, tout);
        start(A0, D0, iD0, s0, tin, side, c0, t0);
        start(A1, D1, iD1, s1, tin, side, c1, t1);
        start(A2, D2, iD2, s2, tin, side, c2, t2);
    }
    __device__ inline bool next() {
        double tm = t0;
        int k = 0;
        if (t1 < tm) tm = t1, k = 1;
        if (t2 < tm) tm = t2, k = 2;
        if (!(tm <= tout)) return false;
        if (k == 0) {
            c0 += s0;
            if (c0 < 0 || c0 >= side) return false;
            t0 = ((double)(c0 + (s0 > 0 ? 1 : 0)) - A0) * iD0;
        } else if (k == 1) {
            c1 += s1;
            if (c1 < 0 || c1 >= side) return false;
            t1 = ((double)(c1 + (s1 > 0 ? 1 : 0)) - A1) * iD1;
        } else {
            c2 += s2;
            if (c2 < 0 || c2 >= side) return false;
            t2 = ((double)(c2 + (s2 > 0 ? 1 : 0)) - A2) * iD2;
        }
        return true;
    }
};

// The observations of one ray (segment a..e, surface point p, direction nn) inside the block
// `key` (block id `id`, kInvalidId when it has none) that its walk visits: the block walk restricted
// to the block's own voxel lattice.
template <int ST, bool QUEUE>
__device__ inline void ray_block(const DevMap& m, const ScanParams& sp, const double a[3], const double e[3],
                                 const double p[3], const double nn[3], unsigned long long key, uint32_t id,
                                 unsigned long long* tab) {
    int32_t bx, by, bz;
    unpack_key(key, bx, by, bz);
    const int64_t b[3] = {bx, by, bz};
    const uint32_t info = id == kInvalidId ? kNoBlockBit : m.binfo[id];
    const int level = (int)((info >> kLevelShift) & 3u);
    const bool has = !(info & kNoBlockBit);
    unsigned long long groups = 0ull;  // the update's lane groups this ray touches in the block
    if (has) {
        const int side = 8 >> level;
        const size_t base = (size_t)(info & kSlotMask) * (size_t)(side * side * side);
        const double nu = m.nu[level];
        BoxWalk bw;
        bw.init(a, e, b, m.B, m.inv_nu[level], side);
        for (int s = 0;; ++s) {
            // observation of the voxel centre (Eq. 1)
            const double x0 = (double)b[0] * m.B + ((double)bw.c0 + 0.5) * nu;
            const double x1 = (double)b[1] * m.B + ((double)bw.c1 + 0.5) * nu;
            const double x2 = (double)b[2] * m.B + ((double)bw.c2 + 0.5) * nu;
            const double sd = ((p[0] - x0) * nn[0] + (p[1] - x1) * nn[1]) + (p[2] - x2) * nn[2];
            const double d = sd < -m.tau ? -m.tau : (sd > m.tau ? m.tau : sd);
            bool near = false;
            if (d >= m.tau) {
                const double r0 = x0 - sp.P.t[0], r1 = x1 - sp.P.t[1], r2 = x2 - sp.P.t[2];
                const double il = m.inv_nu[level];
                near = ((r0 * r0 + r1 * r1) + r2 * r2) * (il * il) < kSatNear2;
            }
            const uint32_t mo = morton3(bw.c0, bw.c1, bw.c2);
            groups |= 1ull << (level == 0 ? mo >> 3 : (level == 1 ? mo : 0u));
            accumulate(m, level, base + (size_t)mo, d, near, tab);
            if (s == 3 * side || !bw.next()) break;
        }
    }
    // mark the groups.  With QUEUE, the ray that sets the block's first bit this scan queues it for
    // the update (exactly one: the walk observes at least one voxel, so groups != 0); without, the
    // OR returns nothing and queue_touched queues the touched blocks after the launch.
    if (QUEUE) {
        bool first = false;
        if (has) {
            const unsigned long long cur = m.btouch[id];
            if ((cur & groups) != groups) first = atomicOr(&m.btouch[id], groups) == 0ull;
        }
        if (__ballot(first)) queue_block(m, first ? level : -1, id, info, key, sp.parity);
    } else if (has) {
        // most rays through a block find their groups already marked: reading first keeps the
        // same-address atomics (thousands per block near the sensor) off the memory side
        if ((m.btouch[id] & groups) != groups) atomicOr(&m.btouch[id], groups);
    }
}

// The blocks the scan's rays touched (non-zero touch mask), queued per level for the update: block
// ids first .. first + count - 1 of this workgroup's range, positions taken in LDS and one atomic
// per level per workgroup (every thread of the workgroup calls).
constexpr int kTouchPerThread = 8;

__device__ inline void queue_touched(const DevMap& m, uint32_t first, uint32_t count, int par) {
    __shared__ uint32_t lcnt[4], lbase[4];
    if (threadIdx.x < 4) lcnt[threadIdx.x] = 0;
    __syncthreads();
    int lvl[kTouchPerThread];
    uint32_t pos[kTouchPerThread];
    for (int r = 0; r < kTouchPerThread; ++r) {
        const uint32_t k = (uint32_t)r * blockDim.x + threadIdx.x;  // consecutive threads, consecutive ids
        lvl[r] = -1;
        pos[r] = 0;
        if (k < count && m.btouch[first + k] != 0ull) {
            lvl[r] = (int)((m.binfo[first + k] >> kLevelShift) & 3u);
            pos[r] = atomicAdd(&lcnt[lvl[r]], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < 4 && lcnt[threadIdx.x]) lbase[threadIdx.x] = atomicAdd(&m.ctr->vis_n[par][threadIdx.x].v, lcnt[threadIdx.x]);
    __syncthreads();
    for (int r = 0; r < kTouchPerThread; ++r) {
        if (lvl[r] < 0) continue;
        const uint32_t id = first + (uint32_t)r * blockDim.x + threadIdx.x;
        m.vis[lvl[r]][lbase[lvl[r]] + pos[r]] = make_entry(id, m.binfo[id], m.bkey[id]);
    }
}

// Rays per wave of the ray launch, and per 256-thread workgroup.
constexpr int kRaysPerWave = 2;
constexpr int kRaysPerGroup = 4 * kRaysPerWave;

// Traversal and accumulation for rays chunk * kRaysPerGroup .. (all threads of the workgroup; tab
// is the workgroup's LDS table of kSatSlots entries).  A ray's block walk is a serial chain of
// lookups, so the (ray, block) pairs that the allocation launch recorded are processed in parallel
// instead: each wave takes its kRaysPerWave rays' pairs 64 at a time, lane l the l-th pair of the
// batch.  The blocks of a ray beyond the recorded rcap_k are walked afterwards by the ray's lane.
template <int ST, bool QUEUE>
__device__ inline void points_ray_chunk(const DevMap& m, const ScanParams& sp, uint32_t chunk, unsigned long long* tab) {
    sat_table_clear(tab);
    const int lane = lane_id();
    const int64_t r0 = (int64_t)chunk * kRaysPerGroup + (int64_t)(threadIdx.x >> 6) * kRaysPerWave;
    const int64_t own = r0 + lane;
    const uint32_t K = (uint32_t)m.rcap_k;
    const uint32_t cnt = (lane < kRaysPerWave && own < sp.n) ? m.rcount[own] : 0u;
    const uint32_t c = cnt < K ? cnt : K;
    uint32_t incl = c;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= o) incl += v;
    }
    const uint32_t total = (uint32_t)__shfl((int)incl, 63);
    const uint32_t excl = incl - c;
    double a[3], e[3], p[3], nn[3];
    // each ray's segment, once, by its own lane; the lanes of its (ray, block) pairs read it from LDS
    __shared__ double seg[4][kRaysPerWave][12];
    const int wv = (int)(threadIdx.x >> 6);
    if (c > 0) {
        point_segment(m, sp, own, a, e, p, nn);  // valid: the ray has recorded blocks
        for (int k = 0; k < 3; ++k) {
            seg[wv][lane][k] = a[k];
            seg[wv][lane][3 + k] = e[k];
            seg[wv][lane][6 + k] = p[k];
            seg[wv][lane][9 + k] = nn[k];
        }
    }
    // LDS operations of one wave complete in order; the fences keep the compiler from moving the
    // reads above the writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (uint32_t base = 0; base < total; base += 64) {
        const uint32_t q = base + (uint32_t)lane;
        // owner: the largest lane j with excl_j <= q (excl is non-decreasing over the lanes)
        int j = 0;
        for (int step = 32; step > 0; step >>= 1) {
            const uint32_t ej = (uint32_t)__shfl((int)excl, j + step);
            if (ej <= q) j += step;
        }
        const uint32_t ej = (uint32_t)__shfl((int)excl, j);
        if (q < total) {
            const int64_t i = r0 + j;
            double sa[3], se[3], sp3[3], sn[3];
            for (int k = 0; k < 3; ++k) {
                sa[k] = seg[wv][j][k];
                se[k] = seg[wv][j][3 + k];
                sp3[k] = seg[wv][j][6 + k];
                sn[k] = seg[wv][j][9 + k];
            }
            const uint32_t slot = m.rslots[(size_t)i * K + (q - ej)];
            const bool ok = slot != kInvalidId;
            const unsigned long long key = ok ? m.hkeys[slot] : 0ull;
            const uint32_t id = ok ? m.hvals[slot] : kInvalidId;
            ray_block<ST, QUEUE>(m, sp, sa, se, sp3, sn, key, id, tab);
        }
    }
    if (cnt > K) {
        point_segment(m, sp, own, a, e, p, nn);
        // the walk state waits in LDS while a block is traversed (registers would hold both)
        __shared__ Walk wsave[4][kRaysPerWave];  // lanes below kRaysPerWave own the rays
        Walk w;
        w.init(a, e, m.invB);
        bool more = true;
        for (uint32_t s = 0; s < K && more; ++s) more = w.next();
        while (more) {
            const unsigned long long key = pack_key(w.c0, w.c1, w.c2);
            wsave[wv][lane] = w;
            __asm__ volatile("" ::: "memory");
            ray_block<ST, QUEUE>(m, sp, a, e, p, nn, key, find_block(m, key), tab);
            __asm__ volatile("" ::: "memory");
            w = wsave[wv][lane];
            more = w.next();
        }
    }
    sat_table_flush(m, tab);
}

// Batch form of Eq. 3 and Eq. 5 for the scan's observations of one voxel: nsat at +tau, and nband
// in the band with sums s1q of q and s2q of q^2 (q = rint(d 2^24)).  With T and Q those sums in
// metres, the band's sums of (d - D) and (d - D)^2 are T - n D and Q - 2 D T + n D^2.
__device__ inline void apply_stats(const DevMap& m, uint32_t nsat, uint32_t nband, unsigned long long s1q,
                                   unsigned long long s2q, float& D, uint32_t& W, float& S2) {
    const uint32_t nobs = nsat + nband;
    const double Dp = (double)D;
    const double ts = m.tau - Dp;
    const double nb = (double)nband;
    const double T = (double)(long long)s1q / kS1Scale, Q = (double)s2q / kS2Scale;
    const double b2 = (Q - 2.0 * Dp * T) + nb * (Dp * Dp);
    const double s1 = (double)nsat * ts + (T - nb * Dp);
    const double s2 = (double)nsat * (ts * ts) + (b2 > 0.0 ? b2 : 0.0);
    const double Wn = (double)W + (double)nobs;
    const double S2n = (double)S2 + s2 - s1 * s1 / Wn;
    D = (float)(Dp + s1 / Wn);
    S2 = (float)(S2n > 0.0 ? S2n : 0.0);
    W = W + nobs;
}

// Read and clear one voxel's scan accumulators.
__device__ inline void take_accumulators(const DevMap& m, int level, size_t at, uint32_t& ns, uint32_t& nb,
                                         unsigned long long& s1, unsigned long long& s2) {
    ns = m.acc_sat[level][at];
    nb = m.acc_band[level][at];
    s1 = s2 = 0ull;
    if (ns) m.acc_sat[level][at] = 0u;
    if (nb) {
        s1 = m.acc_s1[level][at];
        s2 = m.acc_s2[level][at];
        m.acc_band[level][at] = 0u;
        m.acc_s1[level][at] = 0ull;
        m.acc_s2[level][at] = 0ull;
    }
}

template <int ST, bool DEFER>
__device__ inline TaskOut apply_fine(const DevMap& m, const uint4 eq, int par, DeferList* dl) {
    const int lane = lane_id();
    const uint4 e = uniform(eq);  // one block per wave
    const uint32_t id = e.x, info = e.y;
    const double bvs = m.bvsum[id];
    const uint32_t bvc = m.bvcnt[id];
    const bool fresh = (info & kNewBit) != 0;
    const size_t base = (size_t)(info & kSlotMask) * 512 + (size_t)lane * 8;
    // lanes whose group no ray touched have zero accumulators: they read nothing
    const unsigned long long touched = m.btouch[id];
    uint32_t ns[8] = {0, 0, 0, 0, 0, 0, 0, 0}, nb[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if ((touched >> lane) & 1ull) {
        const uint4* a = reinterpret_cast<const uint4*>(m.acc_sat[0] + base);
        const uint4* b = reinterpret_cast<const uint4*>(m.acc_band[0] + base);
        const uint4 a0 = a[0], a1 = a[1], b0 = b[0], b1 = b[1];
        ns[0] = a0.x, ns[1] = a0.y, ns[2] = a0.z, ns[3] = a0.w, ns[4] = a1.x, ns[5] = a1.y, ns[6] = a1.z, ns[7] = a1.w;
        nb[0] = b0.x, nb[1] = b0.y, nb[2] = b0.z, nb[3] = b0.w, nb[4] = b1.x, nb[5] = b1.y, nb[6] = b1.z, nb[7] = b1.w;
    }
    uint32_t upd = 0;
    int nobs = 0;
    for (int q = 0; q < 8; ++q) {
        if (ns[q] + nb[q]) upd |= 1u << q;
        nobs += (int)(ns[q] + nb[q]);
    }
    bool any_band = false;
    for (int q = 0; q < 8; ++q) any_band |= nb[q] != 0;
    const int wobs = wave_sum(nobs);
    TaskOut out;
    out.obs = (uint32_t)wobs;
    out.fresh = fresh ? (uint32_t)wobs : 0u;
    out.distinct = (uint32_t)wave_sum((int)__popc(upd));
    if (lane == 0) m.btouch[id] = 0ull;
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
    if (upd) {
        const ulonglong2* s1p = reinterpret_cast<const ulonglong2*>(m.acc_s1[0] + base);
        const ulonglong2* s2p = reinterpret_cast<const ulonglong2*>(m.acc_s2[0] + base);
        for (int h = 0; h < 2; ++h) {
        unsigned long long s1[4], s2[4];
        if (any_band) {
            const ulonglong2 u0 = s1p[2 * h], u1 = s1p[2 * h + 1], v0 = s2p[2 * h], v1 = s2p[2 * h + 1];
            s1[0] = u0.x, s1[1] = u0.y, s1[2] = u1.x, s1[3] = u1.y, s2[0] = v0.x, s2[1] = v0.y, s2[2] = v1.x, s2[3] = v1.y;
        } else {
            for (int k = 0; k < 4; ++k) s1[k] = s2[k] = 0ull;
        }
        for (int qq = 0; qq < 4; ++qq) {
            const int q = 4 * h + qq;
            if (!(upd & (1u << q))) continue;
            const double before = var_term(m, W[q], S2[q]);
            const int cb = var_count(m, W[q]);
            apply_stats(m, ns[q], nb[q], s1[qq], s2[qq], D[q], W[q], S2[q]);
            Store<ST>::round(m, D[q], W[q], S2[q]);
            dsum += var_term(m, W[q], S2[q]) - before;
            dcnt += var_count(m, W[q]) - cb;
        }
        }
        // leave the accumulators at zero for the next scan
        uint4* a = reinterpret_cast<uint4*>(m.acc_sat[0] + base);
        uint4* b = reinterpret_cast<uint4*>(m.acc_band[0] + base);
        a[0] = a[1] = make_uint4(0, 0, 0, 0);
        if (any_band) {
            b[0] = b[1] = make_uint4(0, 0, 0, 0);
            ulonglong2* s1p = reinterpret_cast<ulonglong2*>(m.acc_s1[0] + base);
            ulonglong2* s2p = reinterpret_cast<ulonglong2*>(m.acc_s2[0] + base);
            for (int h = 0; h < 4; ++h) s1p[h] = s2p[h] = make_ulonglong2(0ull, 0ull);
        }
    }
    out.merge0 = (uint32_t)finish_fine<ST, DEFER>(m, id, info, D, W, S2, have, upd != 0 || fresh, wobs, dsum, dcnt,
                                                        bvs, bvc, par, dl);
    return out;
}

// Level-1 block: lane l owns the voxel at Morton position l.
template <int ST, bool DEFER>
__device__ inline TaskOut apply_level1(const DevMap& m, const uint4 eq, int par, DeferList* dl) {
    const int lane = lane_id();
    const uint4 e = uniform(eq);  // one block per wave
    const uint32_t id = e.x, info = e.y;
    const double bvs = m.bvsum[id];
    const uint32_t bvc = m.bvcnt[id];
    const size_t at = (size_t)(info & kSlotMask) * 64 + lane;
    uint32_t ns = 0, nb = 0;
    unsigned long long s1 = 0ull, s2 = 0ull;
    if ((m.btouch[id] >> lane) & 1ull) take_accumulators(m, 1, at, ns, nb, s1, s2);
    if (lane == 0) m.btouch[id] = 0ull;
    const bool upd = ns + nb > 0;
    const int wobs = wave_sum((int)(ns + nb));
    TaskOut out;
    out.obs = (uint32_t)wobs;
    out.distinct = (uint32_t)wave_sum(upd ? 1 : 0);
    float D, S2;
    uint32_t W;
    Store<ST>::get(m, 1, at, D, W, S2);
    double dsum = 0.0;
    int dcnt = 0;
    if (upd) {
        const double before = var_term(m, W, S2);
        const int cb = var_count(m, W);
        apply_stats(m, ns, nb, s1, s2, D, W, S2);
        Store<ST>::round(m, D, W, S2);
        dsum = var_term(m, W, S2) - before;
        dcnt = var_count(m, W) - cb;
    }
    out.merge1 = (uint32_t)finish_coarse<ST, DEFER>(m, id, info, 1, D, W, S2, upd, wobs, dsum, dcnt, bvs, bvc, par, dl);
    return out;
}

// 64 / seg blocks of `level` (2: seg = 8 voxels, 3: seg = 1 voxel) per wave.
template <int ST>
__device__ inline TaskOut apply_packed(const DevMap& m, const uint4* list, uint32_t count, uint32_t group, int level) {
    const int lane = lane_id();
    const int seg = level == 2 ? 8 : 1;
    const uint32_t bi = group * (uint32_t)(64 / seg) + (uint32_t)(lane / seg);
    const bool live = bi < count;
    uint32_t id = 0, info = 0, ns = 0, nb = 0;
    unsigned long long s1 = 0ull, s2 = 0ull;
    float D = 0.f, S2 = 0.f;
    uint32_t W = 0;
    if (live) {
        const uint4 e = list[bi];
        id = e.x;
        info = e.y;
        const size_t at = (size_t)(info & kSlotMask) * seg + (lane % seg);
        take_accumulators(m, level, at, ns, nb, s1, s2);
        if (lane % seg == 0) m.btouch[id] = 0ull;
        Store<ST>::get(m, level, at, D, W, S2);
    }
    const bool upd = ns + nb > 0;
    double dsum = 0.0;
    int dcnt = 0;
    if (upd) {
        const double before = var_term(m, W, S2);
        const int cb = var_count(m, W);
        apply_stats(m, ns, nb, s1, s2, D, W, S2);
        Store<ST>::round(m, D, W, S2);
        dsum = var_term(m, W, S2) - before;
        dcnt = var_count(m, W) - cb;
    }
    TaskOut out;
    out.obs = (uint32_t)wave_sum((int)(ns + nb));
    out.distinct = (uint32_t)wave_sum(upd ? 1 : 0);
    out.merge2 = (uint32_t)wave_sum(finish_packed<ST>(m, live, id, info, level, seg, D, W, S2, upd, upd ? 1 : 0, dsum, dcnt));
    return out;
}

// One update task t of a scan whose queues hold n0..n3 blocks per level.
// DEFER: merges of level-0 / level-1 blocks are recorded in *dl and done in batches (run_deferred);
// the single-map update does this (a scan's merges all hit one map's stack tops and pending
// counts), the batched update does not (its merges are spread over the maps' counters).
template <int ST, bool DEFER>
__device__ inline TaskOut points_update_task(const DevMap& m, uint32_t t, const TaskCounts& c, int par, DeferList* dl) {
    const uint32_t* n = c.n;  // LiDAR frames queue their new blocks like the others (n_new = 0)
    const uint32_t g2 = (n[2] + 7) / 8;
    if (t < n[0]) return apply_fine<ST, DEFER>(m, m.vis[0][t], par, dl);
    if (t < n[0] + n[1]) return apply_level1<ST, DEFER>(m, m.vis[1][t - n[0]], par, dl);
    if (t < n[0] + n[1] + g2) return apply_packed<ST>(m, m.vis[2], n[2], t - n[0] - n[1], 2);
    return apply_packed<ST>(m, m.vis[3], n[3], t - n[0] - n[1] - g2, 3);
}

}  // namespace mrh
