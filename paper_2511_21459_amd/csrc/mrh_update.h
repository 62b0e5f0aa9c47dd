// Per-block voxel-state helpers shared by the RGB-D and LiDAR update kernels: the running mean /
// Welford update (Eq. 3, Eq. 5) in FP32 registers, the block mean-variance bookkeeping (Eq. 6
// averaged over a block) and the merging criterion of Sec. 3.2.1 with 2x2x2 pooling, for every
// storage format (template parameter ST, see mrh_store.h).  The variance bookkeeping always uses
// the values as stored (after the format's rounding) so that it stays consistent across frames.
//
// Work split: one wave per block.  A level-0 block (8^3 voxels, Morton order) gives lane l the
// 8 contiguous voxels 8l .. 8l+7, which are the children of coarse voxel l; a level n >= 1 block
// (at most 64 voxels) gives lane l the voxel at Morton position l.
#pragma once

#include "mrh_store.h"

namespace mrh {

// Eq. 3 with w_k = 1 and Eq. 5 (Welford) in FP32; 1 / W from the hardware reciprocal (1 ulp).
__device__ inline void welford(float obs, float& D, uint32_t& W, float& S2) {
    const uint32_t Wn = W + 1;
    const float Dold = D;
    const float Dnew = Dold + (obs - Dold) * __builtin_amdgcn_rcpf((float)Wn);
    S2 = S2 + (obs - Dold) * (obs - Dnew);
    D = Dnew;
    W = Wn;
}

// A voxel's term of the block mean variance: sigma^2 = S2 / W (Eq. 6) for voxels with W >= min_obs,
// evaluated in FP32 (a fixed function of the stored S2 and W, so that the incremental block sums
// stay consistent) and summed in FP64.
__device__ inline double var_term(const DevMap& m, uint32_t W, float S2) {
    return W >= (uint32_t)m.min_obs ? (double)(S2 * __builtin_amdgcn_rcpf((float)W)) : 0.0;
}

__device__ inline int var_count(const DevMap& m, uint32_t W) { return W >= (uint32_t)m.min_obs ? 1 : 0; }

// Pop one slot from a level's free stack (single lane).  Returns -1 when the heap is exhausted.
__device__ inline int64_t pop_slot(const DevMap& m, int level) {
    const int32_t top = atomicSub(&m.ctr->top[level].v, 1);
    if (top <= 0) {
        atomicAdd(&m.ctr->top[level].v, 1);
        atomicOr(&m.ctr->error_flags.v, kErrHeapFull);
        return -1;
    }
    return (int64_t)m.stack[level][top - 1];
}

// Slots freed by a merge wait in a pending list until a later launch that does not pop their
// level returns them (a stack that is popped in the same launch is never pushed).  par is the
// frame's parity.
__device__ inline void push_pending(const DevMap& m, int level, uint32_t slot, int par) {
    if (level == 0) {
        const uint32_t p = atomicAdd(&m.ctr->pending0[par].v, 1u);
        m.pend0[par][p] = slot;
    } else {
        const uint32_t p = atomicAdd(&m.ctr->pending[level].v, 1u);
        m.pend[level][p] = slot;
    }
}

// Wave-level forms of the two above for the lanes in `want` / `push` (one atomic for the wave, since
// same-address device atomics serialise chip-wide).  The popped slots are those the same number of
// single pops would return (stack[top-1], stack[top-2], ..); lanes beyond the free count get -1 and
// the heap-full flag is raised.  Callable with some lanes inactive.
__device__ inline int64_t pop_slots_wave(const DevMap& m, int level, bool want) {
    const unsigned long long mask = __ballot(want);
    if (!mask) return -1;
    const int n = __popcll(mask), first = __ffsll((long long)mask) - 1;
    int32_t top = 0;
    if (lane_id() == first) {
        top = atomicSub(&m.ctr->top[level].v, n);
        const int32_t avail = top <= 0 ? 0 : (top < n ? top : n);
        if (avail < n) {
            atomicAdd(&m.ctr->top[level].v, n - avail);
            atomicOr(&m.ctr->error_flags.v, kErrHeapFull);
        }
    }
    top = __shfl(top, first);
    const int avail = top <= 0 ? 0 : (top < n ? top : n);
    const int r = rank_in_mask(mask);
    if (!want || r >= avail) return -1;
    return (int64_t)m.stack[level][top - 1 - r];
}

__device__ inline void push_pending_wave(const DevMap& m, int level, bool push, uint32_t slot, int par) {
    const unsigned long long mask = __ballot(push);
    if (!mask) return;
    const int first = __ffsll((long long)mask) - 1;
    uint32_t p = 0;
    if (lane_id() == first) {
        p = level == 0 ? atomicAdd(&m.ctr->pending0[par].v, (uint32_t)__popcll(mask))
                       : atomicAdd(&m.ctr->pending[level].v, (uint32_t)__popcll(mask));
    }
    p = (uint32_t)__shfl((int)p, first) + (uint32_t)rank_in_mask(mask);
    if (push) {
        if (level == 0) m.pend0[par][p] = slot;
        else m.pend[level][p] = slot;
    }
}

// Merge of a level-0 block into level-1 slot cslot (Sec. 3.2.1, R10): lane l pools its 2x2x2 group
// (the 8 children of coarse voxel l) and lane 0 rewrites the block's table row.  Every lane calls.
template <int ST>
__device__ inline void merge_fine_into(const DevMap& m, uint32_t id, uint32_t cslot, const float D[8],
                                       const uint32_t W[8], const float S2[8]) {
    const int lane = lane_id();
    uint32_t Wc = 0;
    float sd = 0.f, s2 = 0.f;
    for (int q = 0; q < 8; ++q) {
        if (W[q] == 0) continue;
        Wc += W[q];
        sd += (float)W[q] * D[q];
        s2 += S2[q];
    }
    float Dc = Wc > 0 ? sd / (float)Wc : 0.f;
    float Sc = Wc > 0 ? s2 : 0.f;
    Store<ST>::round(m, Dc, Wc, Sc);
    Store<ST>::put(m, 1, (size_t)cslot * 64 + lane, Dc, Wc, Sc);
    const double csum = wave_sum(var_term(m, Wc, Sc));
    const int ccnt = wave_sum(var_count(m, Wc));
    if (lane == 0) {
        m.bvsum[id] = csum;
        m.bvcnt[id] = (uint32_t)ccnt;
        m.binfo[id] = cslot | (1u << kLevelShift);
    }
}

// Merge of a level-1 block (lane = Morton position) into level-2 slot cslot: the 8 children of a
// coarse voxel are 8 consecutive lanes.  Every lane calls.
template <int ST>
__device__ inline void merge_level1_into(const DevMap& m, uint32_t id, uint32_t cslot, float D, uint32_t W, float S2) {
    const int lane = lane_id();
    uint32_t Wc = W;
    float sd = W ? (float)W * D : 0.f, s2 = W ? S2 : 0.f;
    Wc = group8_sum(Wc);
    sd = group8_sum(sd);
    s2 = group8_sum(s2);
    const bool writer = (lane & 7) == 0;
    float Dc = Wc > 0 ? sd / (float)Wc : 0.f;
    float Sc = Wc > 0 ? s2 : 0.f;
    Store<ST>::round(m, Dc, Wc, Sc);
    if (writer) Store<ST>::put(m, 2, (size_t)cslot * 8 + (size_t)(lane >> 3), Dc, Wc, Sc);
    const double csum = wave_sum(writer ? var_term(m, Wc, Sc) : 0.0);
    const int ccnt = wave_sum(writer ? var_count(m, Wc) : 0);
    if (lane == 0) {
        m.bvsum[id] = csum;
        m.bvcnt[id] = (uint32_t)ccnt;
        m.binfo[id] = cslot | (2u << kLevelShift);
    }
}

// Merges recorded during a wave's tasks and performed after them (the LiDAR update, where a scan
// merges tens of thousands of blocks): a merge candidate's update is stored as if it did not merge
// (state and table row), its id goes to the wave's LDS list, and run_deferred() later pops the
// coarse slots of all recorded merges with one atomic per level, pools each block from memory and
// pushes the freed slots with one atomic per level (pops and pushes are same-address atomics that
// serialise chip-wide).  A merge whose pop finds the heap empty leaves the block as stored and
// raises the heap-full flag, as an immediate merge would.  Merging later in the same launch is
// equivalent: no other task of the launch touches the block.
constexpr int kDefer = 16;

struct DeferList {
    uint32_t* e;  // this wave's LDS words: ids[kDefer], infos[kDefer], freed level-0 / level-1 slots
    uint32_t n;   // recorded merges (wave-uniform)

    __device__ static inline void sync() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __device__ inline void add(uint32_t id, uint32_t info) {
        if (lane_id() == 0) {
            e[n] = id;
            e[kDefer + n] = info;
        }
        n += 1;
    }
    __device__ inline bool full() const { return n >= (uint32_t)kDefer; }
};

// count pops from stack[level] by lane 0 with the semantics of count single pops: returns the old
// top; *avail receives how many succeeded (the rest is returned, heap-full flagged)
__device__ inline int32_t pop_batch(const DevMap& m, int level, uint32_t count, uint32_t* avail) {
    int32_t top = 0, got = 0;
    if (count && lane_id() == 0) {
        top = atomicSub(&m.ctr->top[level].v, (int32_t)count);
        got = top <= 0 ? 0 : (top < (int32_t)count ? top : (int32_t)count);
        if (got < (int32_t)count) {
            atomicAdd(&m.ctr->top[level].v, (int32_t)count - got);
            atomicOr(&m.ctr->error_flags.v, kErrHeapFull);
        }
    }
    *avail = uniform((uint32_t)__shfl(got, 0));
    return (int32_t)uniform((uint32_t)__shfl(top, 0));
}

// cnt freed slots (LDS list) onto the pending list of `level` with one atomic
__device__ inline void push_batch(const DevMap& m, int level, const uint32_t* list, uint32_t cnt, int par) {
    if (!cnt) return;
    const int lane = lane_id();
    uint32_t p = 0;
    if (lane == 0) p = level == 0 ? atomicAdd(&m.ctr->pending0[par].v, cnt) : atomicAdd(&m.ctr->pending[level].v, cnt);
    p = (uint32_t)__shfl((int)p, 0);
    for (uint32_t i = (uint32_t)lane; i < cnt; i += 64) {
        if (level == 0) m.pend0[par][p + i] = list[i];
        else m.pend[level][p + i] = list[i];
    }
}

// Perform the recorded merges; adds the merges done to m0 / m1 (levels 0 / 1).
template <int ST>
__device__ inline void run_deferred(const DevMap& m, DeferList& dl, int par, unsigned long long& m0,
                                    unsigned long long& m1) {
    if (dl.n == 0) return;
    DeferList::sync();
    uint32_t n0 = 0, n1 = 0;
    for (uint32_t i = 0; i < dl.n; ++i) {
        if (((uniform(dl.e[kDefer + i]) >> kLevelShift) & 3u) == 0u) ++n0;
        else ++n1;
    }
    uint32_t a0 = 0, a1 = 0;
    const int32_t t1 = pop_batch(m, 1, n0, &a0), t2 = pop_batch(m, 2, n1, &a1);
    uint32_t* fl0 = dl.e + 2 * kDefer;
    uint32_t* fl1 = dl.e + 3 * kDefer;
    uint32_t r0 = 0, r1 = 0, f0 = 0, f1 = 0;
    const int lane = lane_id();
    for (uint32_t i = 0; i < dl.n; ++i) {
        const uint32_t id = uniform(dl.e[i]), info = uniform(dl.e[kDefer + i]);
        const uint32_t slot = info & kSlotMask;
        if (((info >> kLevelShift) & 3u) == 0u) {
            const uint32_t r = r0++;
            if (r >= a0) continue;
            const uint32_t cslot = uniform(m.stack[1][t1 - 1 - (int32_t)r]);
            float D[8], S2[8];
            uint32_t W[8];
            Store<ST>::get8(m, (size_t)slot * 512 + (size_t)lane * 8, D, W, S2);
            merge_fine_into<ST>(m, id, cslot, D, W, S2);
            if (lane == 0) fl0[f0] = slot;
            ++f0;
        } else {
            const uint32_t r = r1++;
            if (r >= a1) continue;
            const uint32_t cslot = uniform(m.stack[2][t2 - 1 - (int32_t)r]);
            float D, S2;
            uint32_t W;
            Store<ST>::get(m, 1, (size_t)slot * 64 + (size_t)lane, D, W, S2);
            merge_level1_into<ST>(m, id, cslot, D, W, S2);
            if (lane == 0) fl1[f1] = slot;
            ++f1;
        }
    }
    DeferList::sync();
    push_batch(m, 0, fl0, f0, par);
    push_batch(m, 1, fl1, f1, par);
    DeferList::sync();
    m0 += f0;
    m1 += f1;
    dl.n = 0;
}

// End of a level-0 block's update.  dsum / dcnt are this lane's change of the block's variance
// sum and count, nupd the wave's number of updated voxels, dirty whether this lane's group must be
// written back, have whether D/W/S2 hold the lane's current group.  Returns 1 when the block merged.
template <int ST, bool DEFER = false>
__device__ inline int finish_fine(const DevMap& m, uint32_t id, uint32_t info, float D[8], uint32_t W[8], float S2[8],
                                   bool have, bool dirty, int nupd, double dsum, int dcnt, double bvs, uint32_t bvc,
                                   int par, DeferList* dl = nullptr) {
    const int lane = lane_id();
    const uint32_t slot = info & kSlotMask;
    const size_t base = (size_t)slot * 512 + (size_t)lane * 8;
    dsum = wave_sum(dsum);
    dcnt = wave_sum(dcnt);
    const double vsum = bvs + dsum;
    const uint32_t vcnt = bvc + (uint32_t)dcnt;
    bool merge = nupd > 0 && m.levels > 1 && vcnt > 0 && vsum / (double)vcnt < m.var_thr;
    if (DEFER && merge) {
        dl->add(id, info);
        merge = false;
    }
    int64_t cslot = -1;
    if (merge) {
        if (lane == 0) cslot = pop_slot(m, 1);
        cslot = (int64_t)__shfl((long long)cslot, 0);
        merge = cslot >= 0;
    }
    if (!merge) {
        if (dirty) Store<ST>::put8(m, base, D, W, S2);
        if (lane == 0) {
            m.bvsum[id] = vsum;
            m.bvcnt[id] = vcnt;
            if (info & kNewBit) m.binfo[id] = info & ~kNewBit;
        }
        return 0;
    }
    if (!have) Store<ST>::get8(m, base, D, W, S2);
    merge_fine_into<ST>(m, id, (uint32_t)cslot, D, W, S2);
    if (lane == 0) push_pending(m, 0, slot, par);
    return 1;
}

// End of a level-1 block's update (lane = Morton position).  The 8 children of a coarse voxel are
// 8 consecutive lanes.  Returns 1 when the block merged.
template <int ST, bool DEFER = false>
__device__ inline int finish_coarse(const DevMap& m, uint32_t id, uint32_t info, int level, float D, uint32_t W,
                                     float S2, bool dirty, int nupd, double dsum, int dcnt, double bvs, uint32_t bvc,
                                     int par, DeferList* dl = nullptr) {
    const int lane = lane_id();
    const int side = 8 >> level, nv = side * side * side;
    const uint32_t slot = info & kSlotMask;
    const size_t at = (size_t)slot * nv + lane;
    dsum = wave_sum(dsum);
    dcnt = wave_sum(dcnt);
    const double vsum = bvs + dsum;
    const uint32_t vcnt = bvc + (uint32_t)dcnt;
    bool merge = nupd > 0 && level < m.levels - 1 && vcnt > 0 && vsum / (double)vcnt < m.var_thr;
    if (DEFER && merge) {  // level 1 only: run_deferred pools level-1 blocks
        dl->add(id, info);
        merge = false;
    }
    int64_t cslot = -1;
    if (merge) {
        if (lane == 0) cslot = pop_slot(m, level + 1);
        cslot = (int64_t)__shfl((long long)cslot, 0);
        merge = cslot >= 0;
    }
    if (!merge) {
        if (dirty && lane < nv) Store<ST>::put(m, level, at, D, W, S2);
        if (lane == 0) {
            m.bvsum[id] = vsum;
            m.bvcnt[id] = vcnt;
        }
        return 0;
    }
    uint32_t Wc = W;
    float sd = W ? (float)W * D : 0.f, s2 = W ? S2 : 0.f;
    Wc = group8_sum(Wc);
    sd = group8_sum(sd);
    s2 = group8_sum(s2);
    const bool writer = lane < nv && (lane & 7) == 0;
    float Dc = Wc > 0 ? sd / (float)Wc : 0.f;
    float Sc = Wc > 0 ? s2 : 0.f;
    Store<ST>::round(m, Dc, Wc, Sc);
    if (writer) Store<ST>::put(m, level + 1, (size_t)cslot * (size_t)(nv / 8) + (size_t)(lane >> 3), Dc, Wc, Sc);
    const double csum = wave_sum(writer ? var_term(m, Wc, Sc) : 0.0);
    const int ccnt = wave_sum(writer ? var_count(m, Wc) : 0);
    if (lane == 0) {
        m.bvsum[id] = csum;
        m.bvcnt[id] = (uint32_t)ccnt;
        m.binfo[id] = (uint32_t)cslot | ((uint32_t)(level + 1) << kLevelShift);
        push_pending(m, level, slot, par);
    }
    return 1;
}

// Packed coarse blocks: `seg` consecutive lanes (8 for level 2, 1 for level 3) hold one block's
// voxels, lane % seg = Morton position.  All reductions stay inside the segment.  Returns, on the
// segment's first lane, 1 when its block merged.
template <int ST>
__device__ inline int finish_packed(const DevMap& m, bool live, uint32_t id, uint32_t info, int level, int seg, float D,
                                    uint32_t W, float S2, bool dirty, int nupd, double dsum, int dcnt) {
    const int par = 0;  // levels >= 2 free into the single list of their level
    const int lane = lane_id();
    if (seg == 8) {
        dsum = group8_sum(dsum);
        dcnt = group8_sum(dcnt);
        nupd = group8_sum(nupd);
    }
    const bool leader = (lane % seg) == 0;
    double vsum = 0.0;
    uint32_t vcnt = 0;
    if (live) {
        vsum = m.bvsum[id] + dsum;
        vcnt = m.bvcnt[id] + (uint32_t)dcnt;
    }
    bool merge = live && nupd > 0 && level < m.levels - 1 && vcnt > 0 && vsum / (double)vcnt < m.var_thr;
    int64_t cslot = -1;
    cslot = pop_slots_wave(m, level + 1, merge && leader);
    if (seg > 1) cslot = (int64_t)__shfl((long long)cslot, lane - (lane % seg));
    merge = merge && cslot >= 0;
    const uint32_t slot = info & kSlotMask;
    if (!merge) {
        if (live && dirty) Store<ST>::put(m, level, (size_t)slot * seg + (lane % seg), D, W, S2);
        if (live && leader) {
            m.bvsum[id] = vsum;
            m.bvcnt[id] = vcnt;
        }
        return 0;
    }
    // only level 2 (seg = 8) can merge: pool the segment's 8 voxels into the single level-3 voxel
    uint32_t Wc = W;
    float sd = W ? (float)W * D : 0.f, s2 = W ? S2 : 0.f;
    if (seg == 8) {
        Wc = group8_sum(Wc);
        sd = group8_sum(sd);
        s2 = group8_sum(s2);
    }
    if (leader) {
        float Dc = Wc > 0 ? sd / (float)Wc : 0.f;
        float Sc = Wc > 0 ? s2 : 0.f;
        Store<ST>::round(m, Dc, Wc, Sc);
        Store<ST>::put(m, level + 1, (size_t)cslot, Dc, Wc, Sc);
        m.bvsum[id] = var_term(m, Wc, Sc);
        m.bvcnt[id] = (uint32_t)var_count(m, Wc);
        m.binfo[id] = (uint32_t)cslot | ((uint32_t)(level + 1) << kLevelShift);
        push_pending_wave(m, level, true, slot, par);
        return 1;
    }
    return 0;
}

// What one update task adds to its wave's statistics (wave-uniform).  Task routines return it and
// the caller adds every field: updates of different fields in different branches would otherwise
// be merged into one dynamically addressed update, which forces the sums into scratch memory.
struct TaskOut {
    uint32_t obs = 0, fresh = 0, merge0 = 0, merge1 = 0, merge2 = 0;
    uint32_t distinct = 0;  // LiDAR: voxels with at least one observation (RGB-D: equal to obs, not set)
};

// Statistics gathered by one wave over its tasks.
struct TaskStats {
    unsigned long long obs = 0, fresh = 0, merge0 = 0, merge1 = 0, merge2 = 0, distinct = 0;
    __device__ inline void add(const TaskOut& o) {
        obs += o.obs;
        fresh += o.fresh;
        merge0 += o.merge0;
        merge1 += o.merge1;
        merge2 += o.merge2;
        distinct += o.distinct;
    }
    // the same with the (wave-uniform) counts summed in scalar registers: for kernels that are
    // short of vector registers but not of scalar ones
    __device__ inline void add_uniform(const TaskOut& o) {
        obs += uniform(o.obs);
        fresh += uniform(o.fresh);
        merge0 += uniform(o.merge0);
        merge1 += uniform(o.merge1);
        merge2 += uniform(o.merge2);
        distinct += uniform(o.distinct);
    }
};

// A frame's update task space: [queued level-0 blocks | blocks allocated this frame (ids
// new_base ..) | level-1 blocks | level-2 blocks in groups of 8 | level-3 blocks in groups of 64].
struct TaskCounts {
    uint32_t n[4];
    uint32_t new_base, n_new;
};

__device__ inline uint32_t update_task_count(const TaskCounts& c) {
    return c.n[0] + c.n_new + c.n[1] + (c.n[2] + 7) / 8 + (c.n[3] + 63) / 64;
}

// Counts of the current frame; with_new: the blocks allocated this frame are update tasks of their
// own (RGB-D); otherwise they are queued like every other block (LiDAR first touch).
__device__ inline TaskCounts frame_task_counts(const DevMap& m, bool with_new, int par) {
    TaskCounts c;
    for (int l = 0; l < 4; ++l) c.n[l] = m.ctr->vis_n[par][l].v;
    c.new_base = m.ctr->n_prev[par];
    const uint32_t nb = m.ctr->n_blocks < m.max_blocks ? m.ctr->n_blocks : m.max_blocks;
    c.n_new = with_new && nb > c.new_base ? nb - c.new_base : 0u;
    return c;
}

// flush one wave's statistics (lane 0); an RGB-D frame updates a voxel at most once, so its
// distinct voxels are its observations
__device__ inline void flush_task_stats(const DevMap& m, const TaskStats& ts, bool depth_frame) {
    if (lane_id() == 0) {
        stat_add(m, S_OBS, ts.obs);
        stat_add(m, S_DISTINCT, depth_frame ? ts.obs : ts.distinct);
        stat_add(m, S_OBS_FRESH, ts.fresh);
        stat_add(m, S_MERGE0, ts.merge0);
        stat_add(m, S_MERGE1, ts.merge1);
        stat_add(m, S_MERGE2, ts.merge2);
    }
}

// Queue block `id` for this frame's update on the list of its level (lanes with level < 0 queue
// nothing).  Called by every lane of the wave; one atomic per level per wave.
__device__ inline void queue_block(const DevMap& m, int level, uint32_t id, uint32_t info, unsigned long long key,
                                   int par) {
    const int lane = lane_id();
    for (int lv = 0; lv < 4; ++lv) {
        const unsigned long long msk = __ballot(level == lv);
        if (!msk) continue;
        const int f0 = __ffsll((long long)msk) - 1;
        uint32_t vb = 0;
        if (lane == f0) vb = atomicAdd(&m.ctr->vis_n[par][lv].v, (uint32_t)__popcll(msk));
        vb = (uint32_t)__shfl((int)vb, f0);
        if (level == lv) m.vis[lv][vb + rank_in_mask(msk)] = make_entry(id, info, key);
    }
}

// Frame hand-off, part 1: run by one workgroup of a frame's allocation launch (frame parity par).
// Clears the other parity's update-queue counts (the previous frame's, used by the next one) and
// returns the slots freed at levels >= 1 by the previous frame's merges to their stacks; nothing
// else in the allocation launch touches those counts or stacks.
__device__ inline void alloc_duties(const DevMap& m, int par) {
    DevCounters* c = m.ctr;
    __shared__ int32_t s_top[4];
    __shared__ uint32_t s_pend[4];
    if (threadIdx.x < 4) {
        const int n = threadIdx.x;
        c->vis_n[par ^ 1][n].v = 0;
        s_top[n] = n >= 1 && n < m.levels ? c->top[n].v : 0;
        s_pend[n] = n >= 1 && n < m.levels ? c->pending[n].v : 0u;
    }
    __syncthreads();
    for (int n = 1; n < m.levels; ++n)
        for (uint32_t i = threadIdx.x; i < s_pend[n]; i += blockDim.x) m.stack[n][s_top[n] + i] = m.pend[n][i];
    if (threadIdx.x >= 1 && threadIdx.x < 4 && (int)threadIdx.x < m.levels && s_pend[threadIdx.x]) {
        c->top[threadIdx.x].v = s_top[threadIdx.x] + (int32_t)s_pend[threadIdx.x];
        c->pending[threadIdx.x].v = 0;
    }
}

// Frame hand-off, part 2: run by one workgroup of a frame's update launch (frame parity par).
// Takes the frame's level-0 pops off the stack, returns the level-0 slots freed by the previous
// frame's merges, and records where the next frame's new block ids start.  Nothing else in the
// update launch pops level 0 or reads the other parity.
__device__ inline void update_duties(const DevMap& m, int par) {
    DevCounters* c = m.ctr;
    __shared__ int32_t s_t0;
    __shared__ uint32_t s_p;
    if (threadIdx.x == 0) {
        const int32_t t0 = c->top[0].v;
        const uint32_t avail = t0 > 0 ? (uint32_t)t0 : 0u;
        const uint32_t pops = c->pops0;
        s_t0 = t0 - (int32_t)(pops < avail ? pops : avail);
        s_p = c->pending0[par ^ 1].v;
        unsigned long long q = 0;  // blocks the frame queued for this launch (all levels)
        for (int l = 0; l < 4; ++l) q += c->vis_n[par][l].v;
        stat_add(m, S_QUEUED, q);
        c->pops0 = 0;
        c->n_prev[par ^ 1] = c->n_blocks < m.max_blocks ? c->n_blocks : m.max_blocks;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < s_p; i += blockDim.x) m.stack[0][s_t0 + i] = m.pend0[par ^ 1][i];
    if (threadIdx.x == 0) {
        c->top[0].v = s_t0 + (int32_t)s_p;
        c->pending0[par ^ 1].v = 0;
    }
}

// Queue block `id` on the update list of `level` (level < 0 queues nothing).  Called by every
// thread of the workgroup (a barrier inside): positions come from LDS counters and one global
// atomic per level per workgroup, since same-address device atomics serialise chip-wide.
__device__ inline void queue_block_wg(const DevMap& m, int level, uint32_t id, uint32_t info, unsigned long long key,
                                      int par) {
    __shared__ uint32_t lcnt[4], lbase[4];
    if (threadIdx.x < 4) lcnt[threadIdx.x] = 0;
    __syncthreads();
    uint32_t local = 0;
    if (level >= 0) local = atomicAdd(&lcnt[level], 1u);
    __syncthreads();
    if (threadIdx.x < 4 && lcnt[threadIdx.x])
        lbase[threadIdx.x] = atomicAdd(&m.ctr->vis_n[par][threadIdx.x].v, lcnt[threadIdx.x]);
    __syncthreads();
    if (level >= 0) m.vis[level][lbase[level] + local] = make_entry(id, info, key);
}

// The block table entry of a new key that took hash slot `slot`: block id `id` and, as the
// frame's `pop`-th level-0 slot, the slot below the stack top of the frame's start (top[0] does
// not change while allocation runs).  Ids beyond max_blocks or pops beyond the stack latch errors.
__device__ inline void register_block(const DevMap& m, unsigned long long key, uint32_t slot, uint32_t id,
                                      uint32_t pop) {
    if (id >= m.max_blocks) {
        m.hvals[slot] = kInvalidId;
        atomicOr(&m.ctr->error_flags.v, kErrBlockLimit);
        stat_add(m, S_FAILED, 1ull);
        return;
    }
    const int32_t t0 = m.ctr->top[0].v;
    uint32_t info;
    if ((int64_t)pop < (int64_t)t0) {
        info = m.stack[0][(uint32_t)t0 - 1u - pop] | kNewBit;
    } else {
        info = kNoBlockBit;
        atomicOr(&m.ctr->error_flags.v, kErrHeapFull);
        stat_add(m, S_FAILED, 1ull);
    }
    m.bkey[id] = key;
    m.binfo[id] = info;
    m.bvsum[id] = 0.0;
    m.bvcnt[id] = 0;
    m.hvals[slot] = id;
}

// k new blocks: one atomic on the allocation word; returns the old word (ids and pops start there).
__device__ inline unsigned long long take_new_blocks(const DevMap& m, uint32_t k) {
    stat_add(m, S_NEW, (unsigned long long)k);
    return atomicAdd(reinterpret_cast<unsigned long long*>(&m.ctr->n_blocks),
                     (unsigned long long)k | ((unsigned long long)k << 32));
}

// Wave-cooperative registration of the lanes that inserted a new key (is_new).
__device__ inline void register_new(const DevMap& m, bool is_new, unsigned long long key, uint32_t slot) {
    const unsigned long long newmask = __ballot(is_new);
    if (!newmask) return;
    const int first = __ffsll((long long)newmask) - 1;
    unsigned long long old = 0;
    if (lane_id() == first) old = take_new_blocks(m, (uint32_t)__popcll(newmask));
    old = shfl_u64(old, first);
    const uint32_t rank = (uint32_t)rank_in_mask(newmask);
    if (is_new) register_block(m, key, slot, (uint32_t)old + rank, (uint32_t)(old >> 32) + rank);
}

// Wave-cooperative claim of one key per lane (has_key): keys found by a read-only probe need
// nothing; the missing ones are deduplicated across the wave (register-only ballots) and then one
// leader per distinct key does the CAS insert, all leaders at once, so that a wave with several
// new keys waits for one insert, not one after another.  Returns true on the lane that inserted a
// new key; *slot receives, on every lane with a key, the hash slot holding it (kInvalidId when the
// table was full).
__device__ inline bool claim_keys(const DevMap& m, bool has_key, unsigned long long key, uint32_t* slot) {
    const int lane = lane_id();
    uint32_t stop = kInvalidId, found = kInvalidId;
    bool need = false;
    if (has_key) {
        found = probe_find(m, key, &stop);
        need = found == kInvalidId;
    }
    bool leader = false;
    int src = lane;  // the lane whose insert decides this lane's key
    unsigned long long pending = __ballot(need);
    while (pending) {
        const int first = __ffsll((long long)pending) - 1;
        const unsigned long long lkey = shfl_u64(key, first);
        const bool same = need && key == lkey;
        pending &= ~__ballot(same);
        if (same) src = first;
        leader |= lane == first;
    }
    bool is_new = false;
    uint32_t got = kInvalidId;
    if (leader) {
        const int r = stop == kInvalidId ? INS_FULL : probe_insert(m, key, stop, &got);
        if (r == INS_NEW) {
            is_new = true;
        } else if (r == INS_FULL) {
            got = kInvalidId;
            atomicOr(&m.ctr->error_flags.v, kErrTableFull);
            stat_add(m, S_FAILED, 1ull);
        }
    }
    const uint32_t from_leader = (uint32_t)__shfl((int)got, src);
    *slot = need ? from_leader : found;
    return is_new;
}


}  // namespace mrh
