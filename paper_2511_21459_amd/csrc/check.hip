// Host-side consistency check of a map's bookkeeping (Sec. 3.1: the spatial hash of Eq. 4 that
// maps block keys to blocks, and the per-level heaps whose slots the blocks hold).  The table,
// the block rows, the free stacks and the pending-free lists are copied to the host between
// frames and checked against each other; nothing on the device is changed.
#include <cstring>
#include <unordered_map>
#include <vector>

#include "mrh_internal.h"

namespace mrh {
namespace {

constexpr unsigned long long kTombstone = ~0ull - 1ull;  // key of a streamed-out block's table slot

template <typename T>
mrh_status fetch(mrh_map* map, std::vector<T>& v, const void* src, size_t n, const char* what) {
    v.resize(n);
    if (n == 0) return MRH_OK;
    return check_hip(map, hipMemcpy(v.data(), src, n * sizeof(T), hipMemcpyDeviceToHost), what);
}

}  // namespace
}  // namespace mrh

using namespace mrh;

extern "C" mrh_status mrh_map_check(mrh_map* map, mrh_check* out) {
    if (!map || !out) return MRH_ERR_INVALID_ARG;
    std::memset(out, 0, sizeof(*out));
    mrh_status st = check_hip(map, hipStreamSynchronize(map->stream), "check");
    if (st != MRH_OK) return st;
    DevCounters c;
    st = check_hip(map, hipMemcpy(&c, map->ctr, sizeof(c), hipMemcpyDeviceToHost), "check");
    if (st != MRH_OK) return st;
    const DevMap& d = map->dm;
    const size_t nh = (size_t)d.hmask + 1;
    const uint32_t nb = c.n_blocks < d.max_blocks ? c.n_blocks : d.max_blocks;
    std::vector<unsigned long long> hkeys, bkey;
    std::vector<uint32_t> hvals, binfo;
    if (st == MRH_OK) st = fetch(map, hkeys, d.hkeys, nh, "check");
    if (st == MRH_OK) st = fetch(map, hvals, d.hvals, nh, "check");
    if (st == MRH_OK) st = fetch(map, bkey, d.bkey, nb, "check");
    if (st == MRH_OK) st = fetch(map, binfo, d.binfo, nb, "check");
    if (st != MRH_OK) return st;

    // the hash table: every present key once, reachable from its home slot within the probe limit
    std::unordered_map<unsigned long long, uint32_t> where;  // key -> table slot
    where.reserve(nh / 2);
    double probe_sum = 0.0;
    for (size_t h = 0; h < nh; ++h) {
        const unsigned long long k = hkeys[h];
        if (k == kEmptyKey) continue;
        if (k == kTombstone) {
            ++out->tombstones;
            continue;
        }
        ++out->table_keys;
        if (!where.emplace(k, (uint32_t)h).second) ++out->duplicate_keys;
        int32_t x, y, z;
        unpack_key(k, x, y, z);
        const uint32_t home = spatial_hash(x, y, z) & d.hmask;
        // the probe from home must reach h without meeting an empty slot
        uint32_t dist = ((uint32_t)h - home) & d.hmask;
        bool blocked = false;
        for (uint32_t s = home; s != (uint32_t)h; s = (s + 1) & d.hmask)
            if (hkeys[s] == kEmptyKey) {
                blocked = true;
                break;
            }
        if (blocked || (int64_t)dist + 1 > (int64_t)d.max_probe) ++out->unreachable_keys;
        probe_sum += (double)dist + 1.0;
        if ((int32_t)dist + 1 > out->max_probe) out->max_probe = (int32_t)dist + 1;
        const uint32_t id = hvals[h];
        if (id == kInvalidId) {
            ++out->idless_keys;  // a key inserted when the block table was full
        } else if (id >= nb || bkey[id] != k || (binfo[id] & kGoneBit)) {
            ++out->bad_table_entries;
        }
    }
    out->mean_probe = out->table_keys ? probe_sum / (double)out->table_keys : 0.0;

    // the block rows: each row not streamed out is the table's block for its key
    std::vector<std::vector<uint8_t>> owner(4);  // per level and heap slot: 1 held, 2 free, 3 pending
    for (int n = 0; n < d.levels; ++n) owner[n].assign((size_t)d.heap_cap[n], 0);
    auto take = [&](int n, uint32_t slot, uint8_t as) {
        if (n >= d.levels || slot >= (uint32_t)d.heap_cap[n] || owner[n][slot]) {
            ++out->slot_conflicts;
            return;
        }
        owner[n][slot] = as;
    };
    out->blocks = nb;
    for (uint32_t id = 0; id < nb; ++id) {
        const uint32_t info = binfo[id];
        if (info & kGoneBit) {
            ++out->gone_blocks;
            continue;
        }
        auto it = where.find(bkey[id]);
        if (it == where.end() || hvals[it->second] != id) ++out->unreachable_keys;
        if (info & kNoBlockBit) {
            ++out->slotless_blocks;  // a key that found its level-0 heap empty
            continue;
        }
        ++out->live_blocks;
        take((int)((info >> kLevelShift) & 3u), info & kSlotMask, 1);
    }

    // free stacks and pending-free lists: disjoint from the held slots, together covering each heap
    for (int n = 0; n < d.levels; ++n) {
        const uint32_t cap = (uint32_t)d.heap_cap[n];
        const int32_t top = c.top[n].v;
        if (top < 0 || (uint32_t)top > cap) {
            ++out->slot_conflicts;
            continue;
        }
        std::vector<uint32_t> s;
        st = fetch(map, s, d.stack[n], (size_t)top, "check");
        if (st != MRH_OK) return st;
        for (uint32_t v : s) take(n, v, 2);
        out->free_slots[n] = top;
        std::vector<const uint32_t*> lists;
        std::vector<uint32_t> counts;
        if (n == 0) {
            for (int p = 0; p < 2; ++p) lists.push_back(d.pend0[p]), counts.push_back(c.pending0[p].v);
        } else {
            lists.push_back(d.pend[n]), counts.push_back(c.pending[n].v);
        }
        for (size_t q = 0; q < lists.size(); ++q) {
            if (counts[q] > cap) {
                ++out->slot_conflicts;
                continue;
            }
            st = fetch(map, s, lists[q], counts[q], "check");
            if (st != MRH_OK) return st;
            for (uint32_t v : s) take(n, v, 3);
            out->pending_slots[n] += counts[q];
        }
        for (uint32_t v = 0; v < cap; ++v)
            if (!owner[n][v]) ++out->lost_slots;
    }
    out->consistent = out->duplicate_keys == 0 && out->unreachable_keys == 0 && out->bad_table_entries == 0 &&
                      out->slot_conflicts == 0 && out->lost_slots == 0;
    return MRH_OK;
}
