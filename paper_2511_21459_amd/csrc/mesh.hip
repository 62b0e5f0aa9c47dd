// Multi-resolution Marching Cubes (Sec. 3.4): the zero set of the fused TSDF as a triangle soup.
//
// Lattice positions are integers in units of half a finest voxel (nu_0 / 2), relative to the
// origin of the block being meshed: along one axis the centre of voxel i of a level-n block is at
// (2 i + 1) 2^n and the block's upper face at 16.  Cell indices and trilinear weights are exact.
//
// Cubes: voxel (i, j, k) of a level-n block spans from its centre to the next lattice point along
// +x, +y, +z.  On the block's upper face along an axis that point is the first voxel-centre plane
// of the face neighbour: a finer neighbour truncates the coarse cube (the transition rule), a
// coarser one stretches it; without a face neighbour there is no cube.  Corner values are the
// multi-resolution trilinear interpolant of the query at the corner (at a voxel centre: the voxel's
// own D, valid iff W > 0); a cube is meshed only when all 8 corners are valid.
//
// Surface: corners with D < 0 are inside.  Per face of the cube, the crossing edges are joined by
// directed segments, each running from an edge where the face's counter-clockwise corner order
// (seen from outside) goes from outside to inside, to the nearest such edge before it going from
// inside to outside -- so an ambiguous face keeps its inside corners connected and the outside
// lies to the left of every segment.  The segments close into loops (the per-case table below,
// built at compile time); a loop is fanned from its lowest edge, or around the mean of its
// vertices when it passes through all four surface points of one face.  Triangles face the
// outside.  Vertex collapse: a surface point closer than collapse * nu_n to an end of its edge is
// moved onto that end, and triangles with two vertices on one point are dropped.
//
// Launch: one wave per block, four blocks per 256-thread workgroup.  The wave caches the 27 blocks
// around its block (ids and levels, one probe per lane) and its block's TSDF (NaN where W = 0) in
// LDS; cubes whose corners all lie in the block read LDS only, the others evaluate the interpolant
// through the cached neighbours.  A first pass counts each cube's triangles, one atomic per
// workgroup reserves the output range, a second pass recomputes the surface cubes and writes.
#include <cmath>

#include "mrh_store.h"

namespace mrh {

// ---- per-case loop table, derived at compile time from the face rule above --------------------

struct McCase {
    uint8_t nloops;
    uint8_t full;     // bit k: loop k is fanned around its centre
    uint8_t len[4];   // edges per loop
    uint8_t edge[12]; // the loops' edges, loop after loop, each starting at its lowest edge
};

struct McTable {
    McCase c[256];
};

// edge joining corners a and b (differing in one bit): 4 * axis + the other two coordinates
constexpr int mc_edge(int a, int b) {
    int axis = 0;
    while (((a ^ b) >> axis) != 1) ++axis;
    int r = 0, bit = 0;
    for (int k = 0; k < 3; ++k) {
        if (k == axis) continue;
        r |= ((a >> k) & 1) << bit;
        ++bit;
    }
    return 4 * axis + r;
}

constexpr McTable make_mc_table() {
    // faces: corners in counter-clockwise order seen from outside the cube
    const int face[6][4] = {{0, 4, 6, 2}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 6, 7, 3}, {0, 2, 3, 1}, {4, 5, 7, 6}};
    McTable t{};
    for (int cs = 0; cs < 256; ++cs) {
        int nxt[12] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
        bool crossing[12] = {};
        int face_edges[6][4] = {};
        int face_cuts[6] = {};
        for (int f = 0; f < 6; ++f) {
            // edge q runs from corner q to corner q + 1 (cyclic); in[q]: corner q is inside
            bool in[4] = {};
            int e[4] = {};
            for (int q = 0; q < 4; ++q) {
                in[q] = ((cs >> face[f][q]) & 1) != 0;
                e[q] = mc_edge(face[f][q], face[f][(q + 1) & 3]);
            }
            for (int q = 0; q < 4; ++q) {
                const bool qin = in[q], nin = in[(q + 1) & 3];
                if (qin == nin) continue;
                crossing[e[q]] = true;
                face_edges[f][face_cuts[f]++] = e[q];
                if (qin) continue;  // this edge goes inside -> outside: an end, found from its start
                // outside -> inside: a start; its end is the nearest earlier inside -> outside edge
                for (int back = 1; back < 4; ++back) {
                    const int p = (q - back + 4) & 3;
                    if (in[p] && !in[(p + 1) & 3]) {
                        nxt[e[q]] = e[p];
                        break;
                    }
                }
            }
        }
        McCase& c = t.c[cs];
        bool used[12] = {};
        int at = 0;
        for (int e0 = 0; e0 < 12; ++e0) {
            if (!crossing[e0] || used[e0]) continue;
            const int start = at;
            for (int x = e0; !used[x]; x = nxt[x]) {
                used[x] = true;
                c.edge[at++] = (uint8_t)x;
            }
            const int k = c.nloops++;
            c.len[k] = (uint8_t)(at - start);
            for (int f = 0; f < 6; ++f) {
                if (face_cuts[f] != 4) continue;
                int on = 0;
                for (int q = 0; q < 4; ++q)
                    for (int y = start; y < at; ++y)
                        if (c.edge[y] == face_edges[f][q]) ++on;
                if (on == 4) c.full |= (uint8_t)(1u << k);
            }
        }
    }
    return t;
}

__constant__ McTable kMc = make_mc_table();

// ---- device side ----------------------------------------------------------------------------

constexpr int kMeshWaves = 4;  // blocks per 256-thread workgroup

__device__ inline int floor16(int p) { return p >> 4; }  // floor(p / 16) for p in [-32, 48)

// The 27 blocks around the meshed one, per wave in LDS: table row (info) or NOBLOCK, and the
// block's voxels (D, NaN where unobserved) in Morton order.
struct MeshLds {
    uint32_t nb[kMeshWaves][27];
    float D[kMeshWaves][512];
    uint32_t ntri[kMeshWaves][512 / 4];  // per cube, packed 8 bits x 4
};

__device__ inline int nb_index(int ox, int oy, int oz) { return (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1); }

template <int ST>
__device__ inline bool voxel_value(const DevMap& m, uint32_t info, int i, int j, int k, float& v) {
    const int n = (int)((info >> kLevelShift) & 3u);
    const int sh = 3 - n;
    const size_t at = (size_t)(info & kSlotMask) * (size_t)(1 << (3 * sh)) + (size_t)morton3(i, j, k);
    if (Store<ST>::getW(m, n, at) == 0u) return false;
    v = Store<ST>::getD(m, n, at);
    return true;
}

// The interpolant at local lattice position P (half-finest units, relative to the meshed block),
// through the cached neighbours.  Zero-weight corners are skipped (they change neither the value
// nor the validity), which keeps every lookup inside the 3 x 3 x 3 neighbourhood.
template <int ST>
__device__ inline bool lattice_value(const DevMap& m, const uint32_t* nbw, const int P[3], float& out) {
    const int h0 = floor16(P[0]), h1 = floor16(P[1]), h2 = floor16(P[2]);
    if (h0 < -1 || h0 > 1 || h1 < -1 || h1 > 1 || h2 < -1 || h2 > 1) return false;
    const uint32_t hinfo = nbw[nb_index(h0, h1, h2)];
    if (hinfo & kNoBlockBit) return false;
    const int n = (int)((hinfo >> kLevelShift) & 3u);
    const int s = 2 << n, half = 1 << n;
    const int hh[3] = {h0, h1, h2};
    int i0[3];
    float f[3];
    for (int a = 0; a < 3; ++a) {
        const int q = P[a] - 16 * hh[a] - half;  // in [-s, 16 + ...)
        const int c = q >= 0 ? q / s : -((-q + s - 1) / s);
        i0[a] = c;
        f[a] = (float)(q - c * s) / (float)s;  // exact: s is a power of two
    }
    float wsum = 0.f, num = 0.f;
    bool any = false;
    for (int c = 0; c < 8; ++c) {
        const int d0 = c & 1, d1 = (c >> 1) & 1, d2 = (c >> 2) & 1;
        const float w = (d0 ? f[0] : 1.f - f[0]) * (d1 ? f[1] : 1.f - f[1]) * (d2 ? f[2] : 1.f - f[2]);
        if (!(w > 0.f)) continue;
        int p2[3], ob[3];
        const int dd[3] = {d0, d1, d2};
        bool inside = true;
        for (int a = 0; a < 3; ++a) {
            p2[a] = 16 * hh[a] + (i0[a] + dd[a]) * s + half;
            ob[a] = floor16(p2[a]);
            inside &= ob[a] >= -1 && ob[a] <= 1;
        }
        if (!inside) continue;
        const uint32_t info = nbw[nb_index(ob[0], ob[1], ob[2])];
        if (info & kNoBlockBit) continue;
        const int n2 = (int)((info >> kLevelShift) & 3u);
        float v;
        if (!voxel_value<ST>(m, info, (p2[0] - 16 * ob[0]) >> (n2 + 1), (p2[1] - 16 * ob[1]) >> (n2 + 1),
                             (p2[2] - 16 * ob[2]) >> (n2 + 1), v))
            continue;
        wsum += w;
        num += w * v;
        any = true;
    }
    if (!any) return false;
    out = num / wsum;
    return true;
}

struct Cube {
    int lo[3], hi[3];
    float v[8];
    int inside;  // bit c: corner c inside (D < 0)
};

// Corner values of cube (i, j, k) of a level-n block of side ms; false when the cube is absent or
// a corner is invalid.
template <int ST>
__device__ inline bool load_cube(const DevMap& m, const uint32_t* nbw, const float* sD, int n, int ms, const int nbl[3],
                                 int i, int j, int k, Cube& cb) {
    const int s = 2 << n, half = 1 << n;
    const int idx[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        cb.lo[a] = (2 * idx[a] + 1) * half;
        if (idx[a] + 1 < ms) cb.hi[a] = cb.lo[a] + s;
        else if (nbl[a] >= 0) cb.hi[a] = 16 + (1 << nbl[a]);
        else return false;
    }
    cb.inside = 0;
    for (int c = 0; c < 8; ++c) {
        const int d0 = c & 1, d1 = (c >> 1) & 1, d2 = (c >> 2) & 1;
        float v;
        if ((!d0 || i + 1 < ms) && (!d1 || j + 1 < ms) && (!d2 || k + 1 < ms)) {
            v = sD[morton3(i + d0, j + d1, k + d2)];
            if (v != v) return false;  // unobserved voxel
        } else {
            const int P[3] = {d0 ? cb.hi[0] : cb.lo[0], d1 ? cb.hi[1] : cb.lo[1], d2 ? cb.hi[2] : cb.lo[2]};
            if (!lattice_value<ST>(m, nbw, P, v)) return false;
        }
        cb.v[c] = v;
        if (v < 0.f) cb.inside |= 1 << c;
    }
    return true;
}

// Vertex id and block-local position (half units) of the surface point of crossing edge e.
__device__ inline int edge_vertex(const Cube& cb, int e, float snap_units, float pos[3]) {
    const int a = e >> 2, r = e & 3;
    const int o1 = a == 0 ? 1 : 0, o2 = a == 2 ? 1 : 2;
    const int c0 = ((r & 1) << o1) | (((r >> 1) & 1) << o2), c1 = c0 | (1 << a);
    const float L = (float)(cb.hi[a] - cb.lo[a]);
    const float t = cb.v[c0] / (cb.v[c0] - cb.v[c1]);
    const float d0 = t * L, d1 = (1.f - t) * L;
    int corner = -1, id = e;
    if (d0 < snap_units) corner = c0, id = 12 + c0;
    else if (d1 < snap_units) corner = c1, id = 12 + c1;
    for (int q = 0; q < 3; ++q) {
        const float p0 = (float)(((c0 >> q) & 1) ? cb.hi[q] : cb.lo[q]);
        const float p1 = (float)(((c1 >> q) & 1) ? cb.hi[q] : cb.lo[q]);
        pos[q] = corner == c0 ? p0 : corner == c1 ? p1 : (q == a ? p0 + t * (p1 - p0) : p0);
    }
    return id;
}

__device__ inline int edge_id(const Cube& cb, int e, float snap_units) {
    float p[3];
    return edge_vertex(cb, e, snap_units, p);
}

// Triangles of a cube after the collapse (count only).
__device__ inline int count_triangles(const Cube& cb, float snap_units) {
    const McCase& mc = kMc.c[cb.inside];
    int ids[12];
    for (int q = 0, at = 0; q < mc.nloops; ++q)
        for (int y = 0; y < mc.len[q]; ++y, ++at) ids[at] = edge_id(cb, mc.edge[at], snap_units);
    int cnt = 0;
    for (int q = 0, at = 0; q < mc.nloops; at += mc.len[q], ++q) {
        const int nl = mc.len[q];
        if ((mc.full >> q) & 1) {
            for (int y = 0; y < nl; ++y) cnt += ids[at + y] != ids[at + (y + 1) % nl];
        } else {
            for (int y = 1; y + 1 < nl; ++y) {
                const int a0 = ids[at], a1 = ids[at + y], a2 = ids[at + y + 1];
                cnt += a0 != a1 && a1 != a2 && a0 != a2;
            }
        }
    }
    return cnt;
}

struct MeshOut {
    float* verts;        // [cap][9] world metres
    int32_t* blocks;     // [cap][3] or null
    uint32_t* codes;     // [cap] or null
    long long cap;
    unsigned long long* count;
    double h;            // metres per half-unit
};

__device__ inline void put_triangle(const MeshOut& o, long long at, const int32_t b[3], uint32_t code,
                                    const float* p0, const float* p1, const float* p2) {
    if (at >= o.cap) return;
    const float* p[3] = {p0, p1, p2};
    for (int x = 0; x < 3; ++x)
        for (int q = 0; q < 3; ++q)
            o.verts[9 * at + 3 * x + q] = (float)((double)(16 * b[q]) * o.h + (double)p[x][q] * o.h);
    if (o.blocks) {
        o.blocks[3 * at] = b[0];
        o.blocks[3 * at + 1] = b[1];
        o.blocks[3 * at + 2] = b[2];
    }
    if (o.codes) o.codes[at] = code;
}

__device__ inline long long write_cube(const Cube& cb, float snap_units, const int32_t b[3], uint32_t code_base,
                                       const MeshOut& o, long long at) {
    const McCase& mc = kMc.c[cb.inside];
    int ids[12];
    float pos[12][3];
    for (int q = 0, y = 0; q < mc.nloops; ++q)
        for (int z = 0; z < mc.len[q]; ++z, ++y) ids[y] = edge_vertex(cb, mc.edge[y], snap_units, pos[y]);
    for (int q = 0, st = 0; q < mc.nloops; st += mc.len[q], ++q) {
        const int nl = mc.len[q];
        if ((mc.full >> q) & 1) {
            float c[3] = {0.f, 0.f, 0.f};
            for (int y = 0; y < nl; ++y)
                for (int x = 0; x < 3; ++x) c[x] += pos[st + y][x];
            for (int x = 0; x < 3; ++x) c[x] /= (float)nl;
            const int cid = 20 + q;
            for (int y = 0; y < nl; ++y) {
                const int u = st + y, w = st + (y + 1) % nl;
                if (ids[u] == ids[w]) continue;
                put_triangle(o, at++, b, code_base | ((uint32_t)ids[u] << 10) | ((uint32_t)ids[w] << 5) | (uint32_t)cid,
                             pos[u], pos[w], c);
            }
        } else {
            for (int y = 1; y + 1 < nl; ++y) {
                const int u = st, v = st + y, w = st + y + 1;
                if (ids[u] == ids[v] || ids[v] == ids[w] || ids[u] == ids[w]) continue;
                put_triangle(o, at++, b, code_base | ((uint32_t)ids[u] << 10) | ((uint32_t)ids[v] << 5) | (uint32_t)ids[w],
                             pos[u], pos[v], pos[w]);
            }
        }
    }
    return at;
}

__device__ inline unsigned long long wave_excl_scan(unsigned long long v, unsigned long long& total) {
    const int lane = lane_id();
    unsigned long long x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = shfl_u64(x, lane >= o ? lane - o : lane);
        if (lane >= o) x += y;
    }
    total = shfl_u64(x, 63);
    return x - v;
}

template <int ST>
__global__ __launch_bounds__(256) void k_mesh(const DevMap* __restrict__ pm, uint32_t n_blocks, float collapse,
                                              MeshOut o) {
    const DevMap& m = *pm;
    __shared__ MeshLds L;
    __shared__ unsigned long long wbase[kMeshWaves];
    __shared__ unsigned long long gbase;
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6);
    const uint32_t id = blockIdx.x * kMeshWaves + (uint32_t)wv;
    uint32_t info = kNoBlockBit;
    unsigned long long key = 0;
    if (id < n_blocks) {
        info = m.binfo[id];
        key = m.bkey[id];
    }
    info = uniform(info);
    key = ((unsigned long long)uniform((uint32_t)(key >> 32)) << 32) | uniform((uint32_t)key);
    const bool live = !(info & kNoBlockBit);
    int32_t b[3] = {0, 0, 0};
    unpack_key(key, b[0], b[1], b[2]);
    const int n = (int)((info >> kLevelShift) & 3u), ms = 8 >> n, nvox = ms * ms * ms;
    uint32_t* nbw = L.nb[wv];
    float* sD = L.D[wv];
    if (live) {
        // the 27 surrounding blocks (one probe per lane) and the block's own voxels
        if (lane < 27) {
            const int ox = lane % 3 - 1, oy = (lane / 3) % 3 - 1, oz = lane / 9 - 1;
            uint32_t ni = kNoBlockBit;
            if (ox == 0 && oy == 0 && oz == 0) {
                ni = info;
            } else {
                const uint32_t bid = find_block(m, pack_key(b[0] + ox, b[1] + oy, b[2] + oz));
                if (bid != kInvalidId) ni = m.binfo[bid];
            }
            nbw[lane] = ni;
        }
        const size_t base = (size_t)(info & kSlotMask) * (size_t)nvox;
        for (int v = lane; v < nvox; v += 64) {
            const bool seen = Store<ST>::getW(m, n, base + v) != 0u;
            sD[v] = seen ? Store<ST>::getD(m, n, base + v) : __builtin_nanf("");
        }
    }
    __syncthreads();
    int nbl[3] = {-1, -1, -1};
    if (live) {
        const uint32_t fx = nbw[nb_index(1, 0, 0)], fy = nbw[nb_index(0, 1, 0)], fz = nbw[nb_index(0, 0, 1)];
        nbl[0] = (fx & kNoBlockBit) ? -1 : (int)((fx >> kLevelShift) & 3u);
        nbl[1] = (fy & kNoBlockBit) ? -1 : (int)((fy >> kLevelShift) & 3u);
        nbl[2] = (fz & kNoBlockBit) ? -1 : (int)((fz >> kLevelShift) & 3u);
    }
    const float snap_units = collapse * (float)(2 << n);  // collapse * nu_n in half units
    // pass 1: triangles per cube
    unsigned long long mine = 0;
    uint8_t* cnt8 = reinterpret_cast<uint8_t*>(L.ntri[wv]);
    if (live) {
        for (int cidx = lane; cidx < nvox; cidx += 64) {
            const int i = cidx % ms, j = (cidx / ms) % ms, k = cidx / (ms * ms);
            Cube cb;
            int c = 0;
            if (load_cube<ST>(m, nbw, sD, n, ms, nbl, i, j, k, cb) && cb.inside != 0 && cb.inside != 255)
                c = count_triangles(cb, snap_units);
            cnt8[cidx] = (uint8_t)c;
            mine += (unsigned long long)c;
        }
    }
    unsigned long long wtot = 0;
    const unsigned long long lane_off = wave_excl_scan(mine, wtot);
    if (lane == 0) wbase[wv] = wtot;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int w = 0; w < kMeshWaves; ++w) {
            const unsigned long long t = wbase[w];
            wbase[w] = tot;
            tot += t;
        }
        gbase = tot ? atomicAdd(o.count, tot) : 0ull;
    }
    __syncthreads();
    if (!live || !o.verts || mine == 0) return;
    // pass 2: the surface cubes again, written at this lane's range
    long long at = (long long)(gbase + wbase[wv] + lane_off);
    for (int cidx = lane; cidx < nvox; cidx += 64) {
        if (cnt8[cidx] == 0) continue;
        const int i = cidx % ms, j = (cidx / ms) % ms, k = cidx / (ms * ms);
        Cube cb;
        load_cube<ST>(m, nbw, sD, n, ms, nbl, i, j, k, cb);
        const uint32_t code_base = ((uint32_t)n << 30) | ((uint32_t)cidx << 15);
        at = write_cube(cb, snap_units, b, code_base, o, at);
    }
}

}  // namespace mrh

using namespace mrh;

extern "C" mrh_status mrh_extract_mesh(mrh_map* map, double collapse, float* verts_dev, int32_t* blocks_dev,
                                       uint32_t* codes_dev, int64_t cap, int64_t* n_tris) {
    if (!map || !n_tris || cap < 0 || !(collapse >= 0.0 && collapse < 0.5)) return MRH_ERR_INVALID_ARG;
    if (!verts_dev && (blocks_dev || codes_dev)) return MRH_ERR_INVALID_ARG;
    DevCounters h;
    mrh_status st = check_hip(map, hipMemcpyAsync(&h, map->ctr, sizeof(h), hipMemcpyDeviceToHost, map->stream), "mesh");
    if (st == MRH_OK) st = check_hip(map, hipMemsetAsync(map->count_dev, 0, 8, map->stream), "mesh");
    if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "mesh");
    if (st != MRH_OK) return st;
    const uint32_t nb = h.n_blocks < map->dm.max_blocks ? h.n_blocks : map->dm.max_blocks;
    MeshOut o;
    o.verts = verts_dev;
    o.blocks = blocks_dev;
    o.codes = codes_dev;
    o.cap = verts_dev ? cap : 0;
    o.count = map->count_dev;
    o.h = 0.5 * map->cfg.voxel;
    if (nb) {
        const unsigned grid = (nb + kMeshWaves - 1) / kMeshWaves;
        const float cf = (float)collapse;
        launch(map, K_MESH, [&] {
            switch (map->cfg.storage) {
                case MRH_STORE_F16: hipLaunchKernelGGL(k_mesh<MRH_STORE_F16>, dim3(grid), dim3(256), 0, map->stream, map->dmd, nb, cf, o); break;
                case MRH_STORE_BF16: hipLaunchKernelGGL(k_mesh<MRH_STORE_BF16>, dim3(grid), dim3(256), 0, map->stream, map->dmd, nb, cf, o); break;
                default: hipLaunchKernelGGL(k_mesh<MRH_STORE_F32>, dim3(grid), dim3(256), 0, map->stream, map->dmd, nb, cf, o);
            }
        });
        st = check_hip(map, hipGetLastError(), "mesh");
        if (st != MRH_OK) return st;
    }
    unsigned long long total = 0;
    st = check_hip(map, hipMemcpyAsync(&total, map->count_dev, 8, hipMemcpyDeviceToHost, map->stream), "mesh");
    if (st == MRH_OK) st = check_hip(map, hipStreamSynchronize(map->stream), "mesh");
    if (st != MRH_OK) return st;
    *n_tris = (int64_t)total;
    if (verts_dev && (int64_t)total > cap)
        return set_error(map, MRH_ERR_BUFFER_TOO_SMALL, "mesh has %llu triangles, buffer holds %lld", total, (long long)cap);
    return MRH_OK;
}
