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
// Launch: one wave per block, four blocks of one level per workgroup (a small kernel lists the
// block ids by level first, so that the waves of a workgroup, which meet at barriers, do work of
// one size).  The wave caches the 27 blocks around its block (ids and levels, one probe per lane)
// and stages its cubes' corner lattice in LDS: its own voxels (TSDF, NaN where W = 0) read
// coalesced in heap order, then the upper-face corners from the cached neighbours, each lane's
// reads issued together.  A first pass counts each cube's triangles, one atomic per workgroup
// reserves the output range, a second pass recomputes the surface cubes and writes.
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

// The same table packed for the kernel: per case the loops' edges as 4-bit fields (position y at
// bits 4 y .. 4 y + 3) and a word with the loop count (bits 0-2), the centre-fan mask (bits 3-6)
// and the loop lengths (4 bits each from bit 8).
struct McPacked {
    unsigned long long edges[256];
    uint32_t meta[256];
};

constexpr McPacked pack_mc_table(const McTable& t) {
    McPacked p{};
    for (int cs = 0; cs < 256; ++cs) {
        const McCase& c = t.c[cs];
        int total = 0;
        uint32_t meta = (uint32_t)c.nloops | ((uint32_t)c.full << 3);
        for (int q = 0; q < c.nloops; ++q) {
            meta |= (uint32_t)c.len[q] << (8 + 4 * q);
            total += c.len[q];
        }
        unsigned long long e = 0;
        for (int y = 0; y < total; ++y) e |= (unsigned long long)c.edge[y] << (4 * y);
        p.edges[cs] = e;
        p.meta[cs] = meta;
    }
    return p;
}

__constant__ McPacked kMc = pack_mc_table(make_mc_table());

// ---- device side ----------------------------------------------------------------------------

constexpr int kMeshWaves = 4;  // blocks per workgroup, one wave each
constexpr int kMeshThreads = 64 * kMeshWaves;

// corners of edge e (compile-time after unrolling): low end and high end
__host__ __device__ constexpr int edge_c0(int e) {
    return (((e & 3) & 1) << ((e >> 2) == 0 ? 1 : 0)) | ((((e & 3) >> 1) & 1) << ((e >> 2) == 2 ? 1 : 2));
}
__host__ __device__ constexpr int edge_c1(int e) { return edge_c0(e) | (1 << (e >> 2)); }

// Morton position of (i, j, k), coordinates below 8
__device__ inline int spread3(int x) { return (x & 1) | ((x & 2) << 2) | ((x & 4) << 4); }
__device__ inline int morton_of(int i, int j, int k) { return spread3(i) | (spread3(j) << 1) | (spread3(k) << 2); }

// Per workgroup: the case table, and per wave the 27 blocks around its block (table row or
// NOBLOCK); the corner values of all the block's cubes, (m + 1)^3 values in x-fastest order (the
// block's voxels, then the interpolant at the upper-face corners, which lie on the first
// voxel-centre plane of each face neighbour; NaN where invalid) and per row of them the sign and
// validity bits; each lane's edge parameters t of the cube it is writing; the block's surface
// cubes and their triangle counts.
struct MeshLds {
    McPacked tab;
    uint32_t rows[kMeshWaves][81];   // per lattice row (j, k): inside bits along x | valid bits << 16
    uint32_t nb[kMeshWaves][27];
    float D[kMeshWaves][729];
    float t[kMeshWaves][12][64];
    uint16_t surf[kMeshWaves][512];  // the block's surface cubes (valid corners of both signs)
    uint8_t cnt[kMeshWaves][512];    // their triangle counts
};

__device__ inline int nb_index(int ox, int oy, int oz) { return (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1); }

template <int ST>
__device__ __forceinline__ bool voxel_value(const DevMap& m, uint32_t info, int i, int j, int k, float& v) {
    const int n = (int)((info >> kLevelShift) & 3u);
    const size_t at = ((size_t)(info & kSlotMask) << (3 * (3 - n))) + (size_t)morton_of(i, j, k);
    // both reads issued together (the TSDF read does not wait for the weight)
    const uint32_t w = Store<ST>::getW(m, n, at);
    const float d = Store<ST>::getD(m, n, at);
    if (w == 0u) return false;
    v = d;
    return true;
}

// Where lattice_value reads a single voxel (position P on a voxel centre of its block): that
// voxel's level and heap position, and true; false when P is outside the neighbourhood, in no
// block, or between voxel centres.
__device__ __forceinline__ bool lattice_voxel(const uint32_t* nbw, int P0, int P1, int P2, size_t& at, int& level) {
    const int hh[3] = {P0 >> 4, P1 >> 4, P2 >> 4};
    if (hh[0] < -1 || hh[0] > 1 || hh[1] < -1 || hh[1] > 1 || hh[2] < -1 || hh[2] > 1) return false;
    const uint32_t hinfo = nbw[nb_index(hh[0], hh[1], hh[2])];
    if (hinfo & kNoBlockBit) return false;
    const int n = (int)((hinfo >> kLevelShift) & 3u);
    const int sh = n + 1, half = 1 << n;
    const int P[3] = {P0, P1, P2};
    int i0[3], r = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int q = P[a] - 16 * hh[a] - half;
        i0[a] = q >> sh;
        r |= q - (i0[a] << sh);
    }
    if (r != 0) return false;
    at = ((size_t)(hinfo & kSlotMask) << (3 * (3 - n))) + (size_t)morton_of(i0[0], i0[1], i0[2]);
    level = n;
    return true;
}

// The interpolant at local lattice position P (half-finest units, relative to the meshed block),
// through the cached neighbours.  A position on the home block's own lattice reads one voxel;
// elsewhere zero-weight corners are skipped (they change neither the value nor the validity),
// which keeps every lookup inside the 3 x 3 x 3 neighbourhood.
template <int ST>
__device__ __forceinline__ bool lattice_value(const DevMap& m, const uint32_t* nbw, int P0, int P1, int P2, float& out) {
    const int hh[3] = {P0 >> 4, P1 >> 4, P2 >> 4};
    if (hh[0] < -1 || hh[0] > 1 || hh[1] < -1 || hh[1] > 1 || hh[2] < -1 || hh[2] > 1) return false;
    const uint32_t hinfo = nbw[nb_index(hh[0], hh[1], hh[2])];
    if (hinfo & kNoBlockBit) return false;
    const int n = (int)((hinfo >> kLevelShift) & 3u);
    const int sh = n + 1, half = 1 << n;
    const float inv_s = __builtin_bit_cast(float, (uint32_t)(126 - n) << 23);  // 2^-(n + 1), exact
    const int P[3] = {P0, P1, P2};
    int i0[3], r[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int q = P[a] - 16 * hh[a] - half;
        i0[a] = q >> sh;  // floor division by s = 2^(n + 1)
        r[a] = q - (i0[a] << sh);
    }
    if ((r[0] | r[1] | r[2]) == 0) return voxel_value<ST>(m, hinfo, i0[0], i0[1], i0[2], out);
    const float f[3] = {(float)r[0] * inv_s, (float)r[1] * inv_s, (float)r[2] * inv_s};
    // the corners' heap positions first, then all their reads at once, then the weighted sum
    size_t at[8];
    int lvl[8];
    float wt[8];
    uint32_t live = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int dd[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
        wt[c] = (dd[0] ? f[0] : 1.f - f[0]) * (dd[1] ? f[1] : 1.f - f[1]) * (dd[2] ? f[2] : 1.f - f[2]);
        at[c] = 0;
        lvl[c] = 0;
        if (!(wt[c] > 0.f)) continue;
        int p2[3], ob[3];
        bool inside = true;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p2[a] = 16 * hh[a] + ((i0[a] + dd[a]) << sh) + half;
            ob[a] = p2[a] >> 4;
            inside &= ob[a] >= -1 && ob[a] <= 1;
        }
        if (!inside) continue;
        const uint32_t info = nbw[nb_index(ob[0], ob[1], ob[2])];
        if (info & kNoBlockBit) continue;
        const int n2 = (int)((info >> kLevelShift) & 3u), s2 = n2 + 1;
        at[c] = ((size_t)(info & kSlotMask) << (3 * (3 - n2))) +
                (size_t)morton_of((p2[0] - 16 * ob[0]) >> s2, (p2[1] - 16 * ob[1]) >> s2, (p2[2] - 16 * ob[2]) >> s2);
        lvl[c] = n2;
        live |= 1u << c;
    }
    uint32_t W[8];
    float D[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        W[c] = 0u;
        D[c] = 0.f;
        if (live & (1u << c)) {
            W[c] = Store<ST>::getW(m, lvl[c], at[c]);
            D[c] = Store<ST>::getD(m, lvl[c], at[c]);
        }
    }
    float wsum = 0.f, num = 0.f;
    bool any = false;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (!(live & (1u << c)) || W[c] == 0u) continue;  // zero-weight corners drop out
        wsum += wt[c];
        num += wt[c] * D[c];
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
// Corner values of cube (i, j, k) of a level-n block of side ms, from the staged corner lattice;
// false when the cube is absent (no face neighbour) or a corner is invalid.
__device__ __forceinline__ bool load_cube(const float* sD, int n, int ms, const int nbl[3], int i, int j, int k, Cube& cb) {
    const int s = 2 << n, half = 1 << n;
    const int idx[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cb.lo[a] = (2 * idx[a] + 1) * half;
        const bool edge = idx[a] + 1 >= ms;
        if (edge && nbl[a] < 0) return false;
        cb.hi[a] = edge ? 16 + (1 << nbl[a]) : cb.lo[a] + s;
    }
    cb.inside = 0;
    const int ma = ms + 1, base = i + ma * (j + ma * k);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float v = sD[base + (c & 1) + ma * (((c >> 1) & 1) + ma * ((c >> 2) & 1))];
        if (v != v) return false;
        cb.v[c] = v;
        cb.inside |= (v < 0.f ? 1 : 0) << c;
    }
    return true;
}

// Vertex ids (5 bits per edge, 12 edges) of a surface cube after the collapse; with tl, the edge
// parameters t of the crossing edges are left in this lane's LDS column.
__device__ __forceinline__ unsigned long long edge_ids(const Cube& cb, float snap_units, float (*tl)[64], int lane) {
    unsigned long long ids = 0;
#pragma unroll
    for (int e = 0; e < 12; ++e) {
        // evaluated for every edge (no branch); only crossing edges are ever looked up
        const int c0 = edge_c0(e), c1 = edge_c1(e), a = e >> 2;
        const float t = cb.v[c0] * __builtin_amdgcn_rcpf(cb.v[c0] - cb.v[c1]);
        const float L = (float)(cb.hi[a] - cb.lo[a]);
        const float d0 = t * L, d1 = (1.f - t) * L;
        const int id = d0 < snap_units ? 12 + c0 : d1 < snap_units ? 12 + c1 : e;
        ids |= (unsigned long long)id << (5 * e);
        if (tl) tl[e][lane] = t;
    }
    return ids;
}

__device__ inline int vid_of(unsigned long long ids, int e) { return (int)((ids >> (5 * e)) & 31ull); }

__device__ inline int tab_edge(unsigned long long edges, int y) { return (int)((edges >> (4 * y)) & 15ull); }

// Triangles of a surface cube (case edges / meta) after the collapse.
__device__ __forceinline__ int count_triangles(unsigned long long edges, uint32_t meta, unsigned long long ids) {
    int cnt = 0;
    const int nloops = (int)(meta & 7u);
    for (int q = 0, at = 0; q < nloops; ++q) {
        const int nl = (int)((meta >> (8 + 4 * q)) & 15u);
        if ((meta >> (3 + q)) & 1u) {
            for (int y = 0; y < nl; ++y)
                cnt += vid_of(ids, tab_edge(edges, at + y)) != vid_of(ids, tab_edge(edges, at + (y + 1 == nl ? 0 : y + 1)));
        } else {
            const int a0 = vid_of(ids, tab_edge(edges, at));
            for (int y = 1; y + 1 < nl; ++y) {
                const int a1 = vid_of(ids, tab_edge(edges, at + y)), a2 = vid_of(ids, tab_edge(edges, at + y + 1));
                cnt += a0 != a1 && a1 != a2 && a0 != a2;
            }
        }
        at += nl;
    }
    return cnt;
}

// Block-local position (half units) of the vertex on edge e with id `id`.
__device__ __forceinline__ void vertex_pos(const Cube& cb, int e, int id, float t, float p[3]) {
    const int c = id >= 12 ? id - 12 : edge_c0(e);
    const int ax = id < 12 ? e >> 2 : -1;  // the axis along which the point lies inside its edge
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = (float)cb.lo[a], hi = (float)cb.hi[a];
        p[a] = a == ax ? lo + t * (hi - lo) : (((c >> a) & 1) ? hi : lo);
    }
}

struct MeshOut {
    float* verts;        // [cap][9] world metres
    int32_t* blocks;     // [cap][3] or null
    uint32_t* codes;     // [cap] or null
    long long cap;
    unsigned long long* count;
    double h;            // metres per half-unit
};

__device__ __forceinline__ void put_triangle(const MeshOut& o, long long at, const double org[3], const int32_t b[3],
                                    uint32_t code, const float* p0, const float* p1, const float* p2) {
    if (at >= o.cap) return;
    const float* p[3] = {p0, p1, p2};
#pragma unroll
    for (int x = 0; x < 3; ++x) {
        float3 w;
        w.x = (float)(org[0] + (double)p[x][0] * o.h);
        w.y = (float)(org[1] + (double)p[x][1] * o.h);
        w.z = (float)(org[2] + (double)p[x][2] * o.h);
        *reinterpret_cast<float3*>(o.verts + 9 * at + 3 * x) = w;
    }
    if (o.blocks) {
        o.blocks[3 * at] = b[0];
        o.blocks[3 * at + 1] = b[1];
        o.blocks[3 * at + 2] = b[2];
    }
    if (o.codes) o.codes[at] = code;
}

__device__ __forceinline__ long long write_cube(const Cube& cb, unsigned long long edges, uint32_t meta,
                                                unsigned long long ids, const float (*tl)[64], int lane,
                                                const double org[3], const int32_t b[3], uint32_t code_base,
                                                const MeshOut& o, long long at) {
    const int nloops = (int)(meta & 7u);
    for (int q = 0, st = 0; q < nloops; ++q) {
        const int nl = (int)((meta >> (8 + 4 * q)) & 15u);
        if ((meta >> (3 + q)) & 1u) {
            float c[3] = {0.f, 0.f, 0.f};
            for (int y = 0; y < nl; ++y) {
                const int e = tab_edge(edges, st + y);
                float p[3];
                vertex_pos(cb, e, vid_of(ids, e), tl[e][lane], p);
                c[0] += p[0], c[1] += p[1], c[2] += p[2];
            }
            const float inv = 1.0f / (float)nl;
            c[0] *= inv, c[1] *= inv, c[2] *= inv;
            for (int y = 0; y < nl; ++y) {
                const int eu = tab_edge(edges, st + y), ew = tab_edge(edges, st + (y + 1 == nl ? 0 : y + 1));
                const int iu = vid_of(ids, eu), iw = vid_of(ids, ew);
                if (iu == iw) continue;
                float pu[3], pw[3];
                vertex_pos(cb, eu, iu, tl[eu][lane], pu);
                vertex_pos(cb, ew, iw, tl[ew][lane], pw);
                put_triangle(o, at++, org, b, code_base | ((uint32_t)iu << 10) | ((uint32_t)iw << 5) | (uint32_t)(20 + q),
                             pu, pw, c);
            }
        } else {
            const int e0 = tab_edge(edges, st);
            const int i0 = vid_of(ids, e0);
            float p0[3];
            vertex_pos(cb, e0, i0, tl[e0][lane], p0);
            for (int y = 1; y + 1 < nl; ++y) {
                const int e1 = tab_edge(edges, st + y), e2 = tab_edge(edges, st + y + 1);
                const int i1 = vid_of(ids, e1), i2 = vid_of(ids, e2);
                if (i0 == i1 || i1 == i2 || i0 == i2) continue;
                float p1[3], p2[3];
                vertex_pos(cb, e1, i1, tl[e1][lane], p1);
                vertex_pos(cb, e2, i2, tl[e2][lane], p2);
                put_triangle(o, at++, org, b, code_base | ((uint32_t)i0 << 10) | ((uint32_t)i1 << 5) | (uint32_t)i2,
                             p0, p1, p2);
            }
        }
        st += nl;
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

// The blocks to mesh, grouped by level so that the waves of a workgroup (which meet at barriers)
// do work of one size: block ids of level l are appended to order[l * stride ...], counts[32 l]
// holding their number (counts start at zero; one 128-byte line per level, so that the levels'
// atomics do not queue behind each other).  Blocks without voxels (no heap slot, streamed out) are
// left out.  Positions are taken in LDS per workgroup, then one atomic per level per workgroup.
constexpr int kOrderLine = 32;  // counter stride in uint32 (128 bytes)

__global__ __launch_bounds__(256) void k_mesh_order(const DevMap* __restrict__ pm, uint32_t n_blocks, uint32_t stride,
                                                    uint32_t* __restrict__ order, uint32_t* __restrict__ counts) {
    const DevMap& m = *pm;
    __shared__ uint32_t lcnt[4], lbase[4];
    if (threadIdx.x < 4) lcnt[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
    int level = -1;
    if (id < n_blocks) {
        const uint32_t info = m.binfo[id];
        if (!(info & kNoBlockBit)) level = (int)((info >> kLevelShift) & 3u);
    }
    uint32_t local = 0;
    for (int l = 0; l < 4; ++l) {
        const unsigned long long mask = __ballot(level == l);
        if (!mask) continue;
        const int first = __ffsll((long long)mask) - 1;
        uint32_t at = 0;
        if (lane_id() == first) at = atomicAdd(&lcnt[l], (uint32_t)__popcll(mask));
        at = (uint32_t)__shfl((int)at, first) + (uint32_t)rank_in_mask(mask);
        if (level == l) local = at;
    }
    __syncthreads();
    if (threadIdx.x < 4 && lcnt[threadIdx.x]) lbase[threadIdx.x] = atomicAdd(&counts[kOrderLine * threadIdx.x], lcnt[threadIdx.x]);
    __syncthreads();
    if (level >= 0) order[(size_t)level * stride + lbase[level] + local] = id;
}

template <int ST>
__global__ __launch_bounds__(kMeshThreads) void k_mesh(const DevMap* __restrict__ pm, const uint32_t* __restrict__ order,
                                              const uint32_t* __restrict__ counts, uint32_t stride, float collapse,
                                              MeshOut o) {
    const DevMap& m = *pm;
    __shared__ MeshLds L;
    __shared__ unsigned long long wbase[kMeshWaves];
    __shared__ unsigned long long gbase;
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6);
    {
        // the case table into LDS (256 x 12 bytes, copied as 32-bit words)
        const uint32_t* src = reinterpret_cast<const uint32_t*>(&kMc);
        uint32_t* dst = reinterpret_cast<uint32_t*>(&L.tab);
        for (int w = threadIdx.x; w < (int)(sizeof(McPacked) / 4); w += kMeshThreads) dst[w] = src[w];
    }
    // this wave's block: workgroups take the levels' lists in turn, kMeshWaves blocks each
    uint32_t id = kInvalidId;
    {
        const uint32_t w = blockIdx.x;
        uint32_t first = 0;
        for (int l = 0; l < 4; ++l) {
            const uint32_t c = counts[kOrderLine * l], g = (c + kMeshWaves - 1) / kMeshWaves;
            if (w < first + g) {
                const uint32_t k = (w - first) * kMeshWaves + (uint32_t)wv;
                if (k < c) id = order[(size_t)l * stride + k];
                break;
            }
            first += g;
        }
    }
    uint32_t info = kNoBlockBit;
    unsigned long long key = 0;
    if (id != kInvalidId) {
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
        // the 27 surrounding blocks (one probe per lane)
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
    }
    __syncthreads();
    int nbl[3] = {-1, -1, -1};
    if (live) {
        const uint32_t fx = nbw[nb_index(1, 0, 0)], fy = nbw[nb_index(0, 1, 0)], fz = nbw[nb_index(0, 0, 1)];
        nbl[0] = (fx & kNoBlockBit) ? -1 : (int)((fx >> kLevelShift) & 3u);
        nbl[1] = (fy & kNoBlockBit) ? -1 : (int)((fy >> kLevelShift) & 3u);
        nbl[2] = (fz & kNoBlockBit) ? -1 : (int)((fz >> kLevelShift) & 3u);
        // the corner lattice: along each axis position (2 i + 1) 2^n for i < m, and the face
        // neighbour's first voxel-centre plane 16 + 2^level for i = m
        const int ma = ms + 1, na = ma * ma * ma, half = 1 << n;
        const float inv_ma = 1.0f / (float)ma;
        const size_t own = (size_t)(info & kSlotMask) * (size_t)nvox;
        // the block's own voxels, read in heap (Morton) order, coalesced: every weight and TSDF
        // read is issued before any is used
        float dq[8];
        uint32_t wq[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int p = lane + 64 * t;
            dq[t] = 0.f;
            wq[t] = 0u;
            if (p < nvox) {
                wq[t] = Store<ST>::getW(m, n, own + (size_t)p);
                dq[t] = Store<ST>::getD(m, n, own + (size_t)p);
            }
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int p = lane + 64 * t;
            if (p < nvox) {
                int i, j, k;
                demorton3(p, i, j, k);
                sD[i + ma * (j + ma * k)] = wq[t] != 0u ? dq[t] : __builtin_nanf("");
            }
        }
        // the upper-face lattice points (na - nvox <= 217 of them, at most 4 per lane): the faces
        // i = m (ma^2 points), then j = m with i < m (m ma), then k = m with i, j < m (m^2).  A point
        // on a voxel centre of its block is read directly, all such reads of a lane issued
        // together; a point between voxel centres (a coarser neighbour) is interpolated.
        const int nface = na - nvox;
        int pv[4];
        size_t pat[4];
        int plv[4], pk[4];
        int pP[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            int bq = lane + 64 * u;
            pk[u] = 0;  // 0 no point, 1 invalid, 2 voxel read, 3 interpolated
            pv[u] = 0;
            pat[u] = 0;
            plv[u] = 0;
            pP[u][0] = pP[u][1] = pP[u][2] = 0;
            if (bq >= nface) continue;
            int i, j, k;
            if (bq < ma * ma) {
                i = ms;
                k = (int)(((float)bq + 0.5f) * inv_ma);
                j = bq - ma * k;
            } else if ((bq -= ma * ma) < ms * ma) {
                j = ms;
                k = bq >> (3 - n);
                i = bq & (ms - 1);
            } else {
                bq -= ms * ma;
                k = ms;
                j = bq >> (3 - n);
                i = bq & (ms - 1);
            }
            pv[u] = i + ma * (j + ma * k);
            pk[u] = 1;
            if (!((i < ms || nbl[0] >= 0) && (j < ms || nbl[1] >= 0) && (k < ms || nbl[2] >= 0))) continue;
            pP[u][0] = i < ms ? (2 * i + 1) * half : 16 + (1 << nbl[0]);
            pP[u][1] = j < ms ? (2 * j + 1) * half : 16 + (1 << nbl[1]);
            pP[u][2] = k < ms ? (2 * k + 1) * half : 16 + (1 << nbl[2]);
            pk[u] = 3;
            if (lattice_voxel(nbw, pP[u][0], pP[u][1], pP[u][2], pat[u], plv[u])) pk[u] = 2;
        }
        uint32_t pw[4];
        float pd[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pw[u] = 0u;
            pd[u] = 0.f;
            if (pk[u] == 2) {
                pw[u] = Store<ST>::getW(m, plv[u], pat[u]);
                pd[u] = Store<ST>::getD(m, plv[u], pat[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (pk[u] == 0) continue;
            float val = __builtin_nanf("");
            if (pk[u] == 2) {
                if (pw[u] != 0u) val = pd[u];
            } else if (pk[u] == 3) {
                float w;
                if (lattice_value<ST>(m, nbw, pP[u][0], pP[u][1], pP[u][2], w)) val = w;
            }
            sD[pv[u]] = val;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // sign and validity bits per lattice row (j, k), x along the bits
        for (int r = lane; r < ma * ma; r += 64) {
            uint32_t bits = 0;
            for (int i = 0; i < ma; ++i) {
                const float v = sD[r * ma + i];
                bits |= (v == v ? 1u : 0u) << (16 + i);
                bits |= (v < 0.f ? 1u : 0u) << i;
            }
            L.rows[wv][r] = bits;
        }
    }
    // the rows are this wave's own: a wave barrier (not a workgroup one) lets each wave go on
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const float snap_units = collapse * (float)(2 << n);  // collapse * nu_n in half units
    const int lg = 3 - n;                                 // log2 of the block side
    // pass 1: the surface cubes (all 8 corners valid, both signs), one row of cubes along x per
    // lane from the row bits, compacted into a list (the triangle work then runs on full waves)
    uint16_t* surf = L.surf[wv];
    uint8_t* cnt8 = L.cnt[wv];
    int nsurf = 0;
    if (live) {
        const int ma = ms + 1, nrows = ms * ms;
        uint32_t smask = 0;  // bit i: cube i of this lane's row is a surface cube
        int row = lane;
        if (row < nrows) {
            const int j = row & (ms - 1), k = row >> lg;
            const uint32_t r00 = L.rows[wv][j + ma * k], r10 = L.rows[wv][j + 1 + ma * k];
            const uint32_t r01 = L.rows[wv][j + ma * (k + 1)], r11 = L.rows[wv][j + 1 + ma * (k + 1)];
            // per cube i: corners (i, i + 1) of the four rows; valid bits from bit 16
            const uint32_t both = (r00 & (r00 >> 1)) & (r10 & (r10 >> 1)) & (r01 & (r01 >> 1)) & (r11 & (r11 >> 1));
            const uint32_t any_in = (r00 | (r00 >> 1) | r10 | (r10 >> 1) | r01 | (r01 >> 1) | r11 | (r11 >> 1)) & 0xFFFFu;
            const uint32_t all_in = (r00 & (r00 >> 1) & r10 & (r10 >> 1) & r01 & (r01 >> 1) & r11 & (r11 >> 1)) & 0xFFFFu;
            const uint32_t valid = (both >> 16) & ((1u << ms) - 1u);
            smask = valid & any_in & ~all_in;
        }
        const int cnt = __popc(smask);
        int tot = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(tot, o);
            if (lane >= o) tot += y;
        }
        int at = tot - cnt;
        nsurf = __shfl(tot, 63);
        while (smask) {
            const int i = __ffs(smask) - 1;
            smask &= smask - 1;
            surf[at++] = (uint16_t)(i + ms * row);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // pass 2: triangles per surface cube after the collapse
    unsigned long long mine = 0;
    for (int q = lane; q < nsurf; q += 64) {
        const int cidx = surf[q];
        Cube cb;
        load_cube(sD, n, ms, nbl, cidx & (ms - 1), (cidx >> lg) & (ms - 1), cidx >> (2 * lg), cb);
        const int c = count_triangles(L.tab.edges[cb.inside], L.tab.meta[cb.inside], edge_ids(cb, snap_units, nullptr, lane));
        cnt8[q] = (uint8_t)c;
        mine += (unsigned long long)c;
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
    // pass 3: the triangles, written at this lane's range
    long long at = (long long)(gbase + wbase[wv] + lane_off);
    const double org[3] = {(double)(16 * b[0]) * o.h, (double)(16 * b[1]) * o.h, (double)(16 * b[2]) * o.h};
    float(*tl)[64] = L.t[wv];
    for (int q = lane; q < nsurf; q += 64) {
        if (cnt8[q] == 0) continue;
        const int cidx = surf[q];
        Cube cb;
        load_cube(sD, n, ms, nbl, cidx & (ms - 1), (cidx >> lg) & (ms - 1), cidx >> (2 * lg), cb);
        const unsigned long long ids = edge_ids(cb, snap_units, tl, lane);
        const uint32_t code_base = ((uint32_t)n << 30) | ((uint32_t)cidx << 15);
        at = write_cube(cb, L.tab.edges[cb.inside], L.tab.meta[cb.inside], ids, tl, lane, org, b, code_base, o, at);
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
        // block ids by level: 4 regions of nb entries, then the 4 counts, one 128-byte line each
        const size_t need = (size_t)4 * nb + 4 * kOrderLine;
        if (need > map->mesh_order_cap) {
            if (map->mesh_order) (void)hipFree(map->mesh_order);
            map->mesh_order = nullptr;
            map->mesh_order_cap = 0;
            st = check_hip(map, hipMalloc((void**)&map->mesh_order, need * sizeof(uint32_t)), "mesh order");
            if (st != MRH_OK) return st;
            map->mesh_order_cap = need;
        }
        uint32_t* order = map->mesh_order;
        uint32_t* counts = order + (size_t)4 * nb;
        st = check_hip(map, hipMemsetAsync(counts, 0, 4 * kOrderLine * sizeof(uint32_t), map->stream), "mesh");
        if (st != MRH_OK) return st;
        // enough workgroups for every level's list rounded up to whole workgroups
        const unsigned grid = (nb + kMeshWaves - 1) / kMeshWaves + 3;
        const float cf = (float)collapse;
        launch(map, K_MESH, [&] {
            hipLaunchKernelGGL(k_mesh_order, dim3((nb + 255) / 256), dim3(256), 0, map->stream, map->dmd, nb, nb, order,
                               counts);
            switch (map->cfg.storage) {
                case MRH_STORE_F16: hipLaunchKernelGGL(k_mesh<MRH_STORE_F16>, dim3(grid), dim3(kMeshThreads), 0, map->stream, map->dmd, order, counts, nb, cf, o); break;
                case MRH_STORE_BF16: hipLaunchKernelGGL(k_mesh<MRH_STORE_BF16>, dim3(grid), dim3(kMeshThreads), 0, map->stream, map->dmd, order, counts, nb, cf, o); break;
                default: hipLaunchKernelGGL(k_mesh<MRH_STORE_F32>, dim3(grid), dim3(kMeshThreads), 0, map->stream, map->dmd, order, counts, nb, cf, o);
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
