/*
 * CPU oracle of the MrHash fusion hot path -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain C++17, FP64 values, a std::map keyed by integer block coordinates, no threads, no SIMD.
 * Built with -ffp-contract=off so every expression below is evaluated exactly as written: the
 * discrete decisions (block keys, traversal cells, pixel indices, the -tau gate, the query lattice
 * index) follow one fixed sequence of IEEE-754 double operations, and multiplications by inverses
 * computed once stand in for divisions wherever a decision depends on them.
 *
 * Per frame the steps follow the paper's pipeline order (Sec. 3, system overview figure):
 *   1. points from the sensor (Sec. 3.1),
 *   2. allocation of every block a measurement segment crosses, by a DDA walk (Sec. 3.2),
 *   3. TSDF / weight / Welford update of the voxels (Eq. 1 or Eq. 2, then Eq. 3 and Eq. 5),
 *   4. block mean variance and the merging criterion (Sec. 3.2.1, Eq. 6).
 */
#include "oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <map>
#include <vector>

namespace {

using Key = std::array<int32_t, 3>;

/* Block coordinates must stay within +-(2^20 - 2) so that every cell a walk may reach fits a
 * 21-bit signed field. A point whose segment end cells leave that range is dropped. */
constexpr int64_t kKeyLimit = (int64_t(1) << 20) - 2;

struct Block {
    int level = 0;
    std::vector<double> D, S2;   /* running mean (Eq. 3) and sum of squared deviations (Eq. 5) */
    std::vector<uint64_t> W;     /* integer weight, w_k = 1 per observation (Sec. 3.1) */
    std::vector<double> C;       /* colour (Sec. 3): running mean of the RGB observations, 3 per voxel */
    bool touched = false;        /* some voxel was updated in the current frame */
};

struct NearEvent {
    Key key;
    int64_t frame;
    double margin;
};

struct Map {
    orc_config cfg;
    double B = 0, invB = 0;      /* constant metric block edge (Sec. 3.2) and its inverse */
    double nu[4] = {0}, inv_nu[4] = {0};
    std::map<Key, Block> blocks;
    orc_stats last{};
    std::vector<NearEvent> near;
    int64_t frame = 0;
};

int side(int level) { return 8 >> level; }

void new_block(Block& b, int level) {
    const int m = side(level);
    b.level = level;
    b.D.assign(size_t(m) * m * m, 0.0);
    b.S2.assign(size_t(m) * m * m, 0.0);
    b.W.assign(size_t(m) * m * m, 0);
    b.C.assign(size_t(3) * m * m * m, 0.0);
    b.touched = false;
}

struct Pose {
    double R[3][3];
    double t[3];
    explicit Pose(const double* T) {
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) R[r][c] = T[4 * r + c];
            t[r] = T[4 * r + 3];
        }
    }
    /* world <- sensor: ((R00 x + R01 y) + R02 z) + t0 */
    void apply(const double p[3], double out[3]) const {
        for (int r = 0; r < 3; ++r) out[r] = ((R[r][0] * p[0] + R[r][1] * p[1]) + R[r][2] * p[2]) + t[r];
    }
    /* sensor <- world for a point: R^T (x - t) */
    void inverse(const double x[3], double out[3]) const {
        const double d0 = x[0] - t[0], d1 = x[1] - t[1], d2 = x[2] - t[2];
        for (int r = 0; r < 3; ++r) out[r] = (R[0][r] * d0 + R[1][r] * d1) + R[2][r] * d2;
    }
};

/* Unit direction from the sensor origin o to the world point p (Eq. 1, n-hat). */
void unit_dir(const double p[3], const double o[3], double n[3]) {
    const double v0 = p[0] - o[0], v1 = p[1] - o[1], v2 = p[2] - o[2];
    const double inv = 1.0 / std::sqrt((v0 * v0 + v1 * v1) + v2 * v2);
    n[0] = v0 * inv;
    n[1] = v1 * inv;
    n[2] = v2 * inv;
}

/*
 * Amanatides-Woo traversal (the DDA of Sec. 3.1 / 3.2) of the segment a -> e over the lattice of
 * cubic cells of edge 1 / inv_cell.  Cells are half-open; the walk starts in the cell holding a,
 * steps across the nearest boundary (lowest axis first on ties), and stops once the next boundary
 * lies beyond e.  Each boundary parameter is evaluated afresh from the cell index, not accumulated.
 */
void block_walk(const double a[3], const double e[3], double inv_cell, std::vector<std::array<int64_t, 3>>& out) {
    double A[3], E[3], invD[3], tmax[3];
    int64_t c[3];
    int st[3];
    int64_t guard = 3;
    for (int k = 0; k < 3; ++k) {
        A[k] = a[k] * inv_cell;
        E[k] = e[k] * inv_cell;
        c[k] = (int64_t)std::floor(A[k]);
        const double dv = E[k] - A[k];
        guard += std::llabs((int64_t)std::floor(E[k]) - c[k]);
        if (dv > 0.0) {
            st[k] = 1;
            invD[k] = 1.0 / dv;
            tmax[k] = ((double)(c[k] + 1) - A[k]) * invD[k];
        } else if (dv < 0.0) {
            st[k] = -1;
            invD[k] = 1.0 / dv;
            tmax[k] = ((double)c[k] - A[k]) * invD[k];
        } else {
            st[k] = 0;
            invD[k] = 0.0;
            tmax[k] = std::numeric_limits<double>::infinity();
        }
    }
    out.push_back({c[0], c[1], c[2]});
    for (int64_t s = 0; s < guard; ++s) {
        int k = 0;
        if (tmax[1] < tmax[k]) k = 1;
        if (tmax[2] < tmax[k]) k = 2;
        if (!(tmax[k] <= 1.0)) break;
        c[k] += st[k];
        tmax[k] = ((double)(c[k] + (st[k] > 0 ? 1 : 0)) - A[k]) * invD[k];
        out.push_back({c[0], c[1], c[2]});
    }
}

/*
 * The same traversal restricted to one block: the segment is clipped to the block's box, the walk
 * starts in the (clamped) cell holding the clipped entry point and continues on the block's own
 * lattice of m^3 voxels until it leaves the block or passes the clipped exit parameter.
 */
void voxel_walk(const double a[3], const double e[3], const Key& b, double B, double inv_nu, int m,
                std::vector<std::array<int, 3>>& out) {
    double Al[3], Dl[3], invD[3], tmax[3];
    int st[3], c[3];
    double tin = 0.0, tout = 1.0;
    for (int k = 0; k < 3; ++k) {
        const double ob = (double)b[k] * B;
        Al[k] = (a[k] - ob) * inv_nu;
        const double El = (e[k] - ob) * inv_nu;
        Dl[k] = El - Al[k];
        if (Dl[k] != 0.0) {
            invD[k] = 1.0 / Dl[k];
            const double nearb = Dl[k] > 0.0 ? 0.0 : (double)m;
            const double farb = Dl[k] > 0.0 ? (double)m : 0.0;
            const double t0 = (nearb - Al[k]) * invD[k];
            const double t1 = (farb - Al[k]) * invD[k];
            if (t0 > tin) tin = t0;
            if (t1 < tout) tout = t1;
            st[k] = Dl[k] > 0.0 ? 1 : -1;
        } else {
            invD[k] = 0.0;
            st[k] = 0;
        }
    }
    for (int k = 0; k < 3; ++k) {
        const double P = Al[k] + tin * Dl[k];
        double f = std::floor(P);
        if (f < 0.0) f = 0.0;
        if (f > (double)(m - 1)) f = (double)(m - 1);
        c[k] = (int)f;
        tmax[k] = st[k] != 0 ? ((double)(c[k] + (st[k] > 0 ? 1 : 0)) - Al[k]) * invD[k]
                             : std::numeric_limits<double>::infinity();
    }
    out.push_back({c[0], c[1], c[2]});
    for (int s = 0; s < 3 * m; ++s) {
        int k = 0;
        if (tmax[1] < tmax[k]) k = 1;
        if (tmax[2] < tmax[k]) k = 2;
        if (!(tmax[k] <= tout)) break;
        c[k] += st[k];
        if (c[k] < 0 || c[k] >= m) break;
        tmax[k] = ((double)(c[k] + (st[k] > 0 ? 1 : 0)) - Al[k]) * invD[k];
        out.push_back({c[0], c[1], c[2]});
    }
}

bool in_key_range(const double a[3], const double e[3], double invB) {
    for (int k = 0; k < 3; ++k) {
        const double fa = std::floor(a[k] * invB), fe = std::floor(e[k] * invB);
        if (!(std::fabs(fa) <= (double)kKeyLimit && std::fabs(fe) <= (double)kKeyLimit)) return false;
    }
    return true;
}

/* Allocate every block the segment crosses at the finest level (Sec. 3.2.1: blocks start fine). */
void allocate(Map& m, const double a[3], const double e[3]) {
    std::vector<std::array<int64_t, 3>> cells;
    block_walk(a, e, m.invB, cells);
    m.last.candidate_keys += (int64_t)cells.size();
    for (const auto& c : cells) {
        const Key k{(int32_t)c[0], (int32_t)c[1], (int32_t)c[2]};
        auto it = m.blocks.find(k);
        if (it == m.blocks.end()) {
            new_block(m.blocks[k], 0);
            m.last.new_blocks++;
        }
    }
}

/* Voxel centre: block origin b * B plus (i + 1/2) voxel edges of the block's level. */
void voxel_centre(const Map& m, const Key& b, int level, int i, int j, int k, double c[3]) {
    const double nu = m.nu[level];
    c[0] = (double)b[0] * m.B + ((double)i + 0.5) * nu;
    c[1] = (double)b[1] * m.B + ((double)j + 0.5) * nu;
    c[2] = (double)b[2] * m.B + ((double)k + 0.5) * nu;
}

/* Eq. 3 with w_k = 1 and the Welford recurrence of Eq. 5, in incremental form. */
void observe(Block& blk, int idx, double d) {
    const uint64_t W = blk.W[idx] + 1;
    const double Dold = blk.D[idx];
    const double Dnew = Dold + (d - Dold) / (double)W;
    blk.S2[idx] = blk.S2[idx] + (d - Dold) * (d - Dnew);
    blk.D[idx] = Dnew;
    blk.W[idx] = W;
    blk.touched = true;
}

/*
 * Merging criterion (Sec. 3.2.1): the block mean of the voxel variances sigma^2 = S2 / W (Eq. 6),
 * over voxels with at least min_obs observations, is compared with the threshold; a block below it
 * is re-sampled one level coarser.  Pooling of the 2x2x2 children of each coarse voxel keeps the
 * total weight and the weighted TSDF sum, and adds up the children's S2.
 */
void merge_block(Map& m, Block& blk) {
    const int n = blk.level, mf = side(n), mc = mf / 2;
    std::vector<double> D(size_t(mc) * mc * mc), S2(size_t(mc) * mc * mc), C(size_t(3) * mc * mc * mc);
    std::vector<uint64_t> W(size_t(mc) * mc * mc);
    for (int K = 0; K < mc; ++K)
        for (int J = 0; J < mc; ++J)
            for (int I = 0; I < mc; ++I) {
                uint64_t w = 0;
                double sd = 0.0, s2 = 0.0, sc[3] = {0.0, 0.0, 0.0};
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            const int f = (2 * I + a) + mf * ((2 * J + b) + mf * (2 * K + c));
                            if (blk.W[f] == 0) continue;
                            w += blk.W[f];
                            sd += (double)blk.W[f] * blk.D[f];
                            s2 += blk.S2[f];
                            for (int ch = 0; ch < 3; ++ch) sc[ch] += (double)blk.W[f] * blk.C[3 * (size_t)f + ch];
                        }
                const int o = I + mc * (J + mc * K);
                W[o] = w;
                D[o] = w > 0 ? sd / (double)w : 0.0;
                S2[o] = w > 0 ? s2 : 0.0;
                /* colour pools like the TSDF: the weighted mean of the observed children */
                for (int ch = 0; ch < 3; ++ch) C[3 * (size_t)o + ch] = w > 0 ? sc[ch] / (double)w : 0.0;
            }
    blk.level = n + 1;
    blk.D.swap(D);
    blk.W.swap(W);
    blk.S2.swap(S2);
    blk.C.swap(C);
    (void)m;
}

void variance_and_merge(Map& m) {
    const double thr = m.cfg.var_thr;
    for (auto& kv : m.blocks) {
        Block& blk = kv.second;
        if (!blk.touched) continue;
        blk.touched = false;
        if (blk.level >= m.cfg.levels - 1) continue;
        double sum = 0.0;
        int64_t cnt = 0;
        for (size_t v = 0; v < blk.W.size(); ++v) {
            if (blk.W[v] >= (uint64_t)m.cfg.min_obs) {
                sum += blk.S2[v] / (double)blk.W[v];
                cnt++;
            }
        }
        if (cnt == 0) continue;
        const double mv = sum / (double)cnt;
        const double margin = std::fabs(mv - thr) / thr;
        if (margin < 5e-2) m.near.push_back({kv.first, m.frame, margin});
        if (margin < 1e-3) m.last.near_threshold++;
        if (mv < thr) {
            m.last.merges[blk.level]++;
            merge_block(m, blk);
        }
    }
}

bool depth_ok(double d, double max_depth) { return std::isfinite(d) && d > 0.0 && d <= max_depth; }

int64_t floor_div(int64_t c, int64_t m) { return c >= 0 ? c / m : -((-c + m - 1) / m); }

const Block* find(const Map& m, int64_t x, int64_t y, int64_t z) {
    if (std::llabs(x) > kKeyLimit + 2 || std::llabs(y) > kKeyLimit + 2 || std::llabs(z) > kKeyLimit + 2) return nullptr;
    auto it = m.blocks.find(Key{(int32_t)x, (int32_t)y, (int32_t)z});
    return it == m.blocks.end() ? nullptr : &it->second;
}

/*
 * Multi-resolution trilinear interpolation (Sec. 3.4): the point's own block fixes the lattice
 * (its level n); the 8 surrounding level-n lattice points are read from whichever voxel, at any
 * level, contains them; corners in absent blocks or with W = 0 drop out and the remaining
 * trilinear weights are renormalised.
 */
struct QueryOut {
    bool valid = false;
    double sdf = 0.0;
    double grad[3] = {0, 0, 0};
};

QueryOut query_one(const Map& m, const double x[3], bool strict) {
    QueryOut q;
    int64_t bk[3];
    for (int k = 0; k < 3; ++k) {
        const double f = std::floor(x[k] * m.invB);
        if (!(std::fabs(f) <= (double)kKeyLimit)) return q;
        bk[k] = (int64_t)f;
    }
    const Block* home = find(m, bk[0], bk[1], bk[2]);
    if (!home) return q;
    const int n = home->level;
    int64_t i0[3];
    double f[3];
    for (int k = 0; k < 3; ++k) {
        const double g = x[k] * m.inv_nu[n] - 0.5;
        const double fl = std::floor(g);
        i0[k] = (int64_t)fl;
        f[k] = g - fl;
    }
    const int64_t mn = side(n);
    double wsum = 0.0, num = 0.0;
    double cw[8], cd[8];
    bool cv[8];
    int nvalid = 0;
    bool any_pos = false;
    for (int c = 0; c < 8; ++c) {
        const int dl[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
        int64_t cell[3], cb[3];
        for (int k = 0; k < 3; ++k) {
            cell[k] = i0[k] + dl[k];
            cb[k] = floor_div(cell[k], mn);
        }
        cw[c] = (dl[0] ? f[0] : 1.0 - f[0]) * (dl[1] ? f[1] : 1.0 - f[1]) * (dl[2] ? f[2] : 1.0 - f[2]);
        cv[c] = false;
        cd[c] = 0.0;
        const Block* blk = find(m, cb[0], cb[1], cb[2]);
        if (!blk) continue;
        const int n2 = blk->level, m2 = side(n2);
        int idx[3];
        for (int k = 0; k < 3; ++k) {
            /* lattice point (cell + 1/2) nu_n expressed in half finest voxels, relative to the block */
            const int64_t p2 = cell[k] * (int64_t(2) << n) + (int64_t(1) << n);
            const int64_t local2 = p2 - 16 * cb[k];
            idx[k] = (int)(local2 / (int64_t(2) << n2));
        }
        const int v = idx[0] + m2 * (idx[1] + m2 * idx[2]);
        if (blk->W[v] == 0) continue;
        cv[c] = true;
        cd[c] = blk->D[v];
        nvalid++;
        wsum += cw[c];
        num += cw[c] * cd[c];
        if (cw[c] > 0.0) any_pos = true;
    }
    if (strict ? nvalid < 8 : !any_pos) return q;
    q.valid = true;
    q.sdf = num / wsum;
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int c = 0; c < 8; ++c) {
            if (!cv[c]) continue;
            const int dl[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
            double dw = dl[a] ? 1.0 : -1.0;
            for (int b = 0; b < 3; ++b)
                if (b != a) dw *= dl[b] ? f[b] : 1.0 - f[b];
            s += dw * (cd[c] - q.sdf);
        }
        q.grad[a] = s / wsum * m.inv_nu[n];
    }
    return q;
}

/*
 * ---- Multi-resolution Marching Cubes (Sec. 3.4) ----------------------------------------------
 *
 * Positions are integers in units of half a finest voxel (nu_0 / 2): along one axis the centre of
 * voxel i of a level-n block with coordinate b sits at 16 b + (2 i + 1) 2^n, and a block face at
 * 16 b.  Every position the mesher evaluates is such an integer, so the cell indices and the
 * trilinear weights below are exact.
 *
 * Cubes.  Each voxel (i, j, k) of a level-n block spans one cube from its own centre to the next
 * lattice point along +x, +y and +z.  Inside the block that is the next voxel centre of the same
 * level.  On the block's upper face along an axis the cube reaches the first voxel-centre plane of
 * the face neighbour: when the neighbour is finer the coarse cube is truncated there, so that it
 * ends where the finer block's own cubes begin (the transition rule of Sec. 3.4); when the
 * neighbour is coarser the cube is stretched to its first centre plane, so that no gap opens
 * between the two levels.  Without a face neighbour there is no cube.
 *
 * Corner values are the map's multi-resolution trilinear interpolant (the one of the query,
 * Sec. 3.4) at the corner: the corner's own block fixes the lattice, the 8 surrounding lattice
 * points take the TSDF of the voxel, at any level, containing them, absent or unobserved ones
 * drop out and the weights are renormalised.  At a voxel centre this is the voxel's own D (valid
 * iff W > 0).  A cube is meshed only when all 8 corner values are valid.
 *
 * Surface.  Corners with D < 0 are inside.  On each of the cube's 6 faces every edge whose two
 * corners differ in sign carries a surface point; the points are joined in pairs by segments, one
 * pair on a face with two such edges, two on a face with four (then each segment cuts off one
 * outside corner, so the inside corners stay connected across the face).  Each segment is
 * directed so that, with the face's outward normal N, N x (end - start) points to the outside
 * corners.  The directed segments close into loops; each loop is fanned into triangles from its
 * edge of lowest index, so every triangle's normal (right-hand rule) points to the outside.  A
 * loop that passes through all four surface points of one face is fanned around the mean of its
 * vertices instead (from a vertex, a triangle could lie flat on that face, on top of one of the
 * neighbouring cube's); the k-th loop's centre has vertex id 20 + k.
 *
 * Vertex collapse.  An edge's surface point lies at t = v0 / (v0 - v1) from its lower corner.  When
 * it is closer than collapse * nu_n (nu_n: the cube's voxel size) to a corner of the edge it is
 * moved onto that corner; triangles with two vertices on one point are dropped.
 *
 * Numbering: corner c = x + 2 y + 4 z (x, y, z in {0, 1}); edge e lies along axis a = e / 4, its
 * two other coordinates are bit 0 and bit 1 of e % 4 on the other axes in increasing order.
 */
struct MeshOut {
    std::vector<double>* verts;
    std::vector<int32_t>* blocks;
    std::vector<uint32_t>* codes;
    std::vector<uint8_t>* near;
};

int edge_axis(int e) { return e / 4; }

/* the corners of edge e: low end c0, high end c1 */
void edge_corners(int e, int& c0, int& c1) {
    const int a = e / 4, r = e % 4;
    int other[2], o = 0;
    for (int k = 0; k < 3; ++k)
        if (k != a) other[o++] = k;
    c0 = ((r & 1) << other[0]) | (((r >> 1) & 1) << other[1]);
    c1 = c0 | (1 << a);
}

/* Interpolant at an exact lattice position P (half-finest units); false when no corner counts. */
bool lattice_value(const Map& m, const int64_t P[3], double& out) {
    int64_t hb[3];
    for (int k = 0; k < 3; ++k) hb[k] = floor_div(P[k], 16);
    const Block* home = find(m, hb[0], hb[1], hb[2]);
    if (!home) return false;
    const int n = home->level;
    const int64_t s = int64_t(2) << n, half = int64_t(1) << n;
    int64_t i0[3];
    double f[3];
    for (int k = 0; k < 3; ++k) {
        const int64_t q = P[k] - half; /* = (cell index + fraction) * s */
        i0[k] = floor_div(q, s);
        f[k] = (double)(q - i0[k] * s) / (double)s;
    }
    double wsum = 0.0, num = 0.0;
    bool any = false;
    for (int c = 0; c < 8; ++c) {
        const int dl[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
        const double w = (dl[0] ? f[0] : 1.0 - f[0]) * (dl[1] ? f[1] : 1.0 - f[1]) * (dl[2] ? f[2] : 1.0 - f[2]);
        int64_t p2[3], cb[3];
        for (int k = 0; k < 3; ++k) {
            p2[k] = (i0[k] + dl[k]) * s + half;
            cb[k] = floor_div(p2[k], 16);
        }
        const Block* blk = find(m, cb[0], cb[1], cb[2]);
        if (!blk) continue;
        const int n2 = blk->level, m2 = side(n2);
        int idx[3];
        for (int k = 0; k < 3; ++k) idx[k] = (int)((p2[k] - 16 * cb[k]) / (int64_t(2) << n2));
        const int v = idx[0] + m2 * (idx[1] + m2 * idx[2]);
        if (blk->W[v] == 0) continue;
        wsum += w;
        num += w * blk->D[v];
        if (w > 0.0) any = true;
    }
    if (!any) return false;
    out = num / wsum;
    return true;
}

/* Mesh one block (key b); appends its triangles. */
void mesh_block(const Map& m, const Key& b, const Block& blk, double collapse, MeshOut& o) {
    const int n = blk.level, mside = side(n);
    const int64_t half = int64_t(1) << n, s = int64_t(2) << n;
    const double h = 0.5 * m.cfg.voxel; /* metres per lattice unit */
    const double snap = collapse * m.nu[n];
    int nb_level[3];
    for (int a = 0; a < 3; ++a) {
        int64_t q[3] = {b[0], b[1], b[2]};
        q[a] += 1;
        const Block* nb = find(m, q[0], q[1], q[2]);
        nb_level[a] = nb ? nb->level : -1;
    }
    for (int k = 0; k < mside; ++k)
        for (int j = 0; j < mside; ++j)
            for (int i = 0; i < mside; ++i) {
                const int idx[3] = {i, j, k};
                int64_t lo[3], hi[3];
                bool ok = true;
                for (int a = 0; a < 3; ++a) {
                    lo[a] = 16 * (int64_t)b[a] + (2 * idx[a] + 1) * half;
                    if (idx[a] + 1 < mside) {
                        hi[a] = lo[a] + s;
                    } else if (nb_level[a] >= 0) {
                        hi[a] = 16 * ((int64_t)b[a] + 1) + (int64_t(1) << nb_level[a]);
                    } else {
                        ok = false;
                    }
                }
                if (!ok) continue;
                double v[8];
                int64_t P[8][3];
                for (int c = 0; c < 8 && ok; ++c) {
                    for (int a = 0; a < 3; ++a) P[c][a] = ((c >> a) & 1) ? hi[a] : lo[a];
                    ok = lattice_value(m, P[c], v[c]);
                }
                if (!ok) continue;
                bool near = false;
                int inside = 0;
                for (int c = 0; c < 8; ++c) {
                    if (v[c] < 0.0) inside |= 1 << c;
                    if (std::fabs(v[c]) < 1e-6) near = true;
                }
                if (inside == 0 || inside == 255) continue;
                /* surface points of the crossing edges, with vertex collapse */
                bool cross[12];
                int vid[12];
                double pos[12][3];
                for (int e = 0; e < 12; ++e) {
                    int c0, c1;
                    edge_corners(e, c0, c1);
                    cross[e] = ((inside >> c0) & 1) != ((inside >> c1) & 1);
                    if (!cross[e]) continue;
                    const int a = edge_axis(e);
                    const double L = (double)(hi[a] - lo[a]) * h;
                    const double t = v[c0] / (v[c0] - v[c1]);
                    if (std::fabs(v[c0] - v[c1]) < 1e-3) near = true;
                    const double d0 = t * L, d1 = (1.0 - t) * L;
                    if (std::fabs(d0 - snap) < 1e-6 * m.nu[n] || std::fabs(d1 - snap) < 1e-6 * m.nu[n]) near = true;
                    if (d0 < snap) {
                        vid[e] = 12 + c0;
                        for (int q = 0; q < 3; ++q) pos[e][q] = (double)P[c0][q] * h;
                    } else if (d1 < snap) {
                        vid[e] = 12 + c1;
                        for (int q = 0; q < 3; ++q) pos[e][q] = (double)P[c1][q] * h;
                    } else {
                        vid[e] = e;
                        for (int q = 0; q < 3; ++q)
                            pos[e][q] = (double)P[c0][q] * h + t * ((double)P[c1][q] * h - (double)P[c0][q] * h);
                    }
                }
                /* directed segments on the 6 faces */
                int next[12];
                for (int e = 0; e < 12; ++e) next[e] = -1;
                for (int a = 0; a < 3; ++a)
                    for (int sd = 0; sd < 2; ++sd) {
                        /* the face's 4 edges: along the two other axes, with coordinate sd on axis a */
                        int fe[4], nf = 0;
                        for (int e = 0; e < 12; ++e) {
                            if (edge_axis(e) == a) continue;
                            int c0, c1;
                            edge_corners(e, c0, c1);
                            if (((c0 >> a) & 1) == sd) fe[nf++] = e;
                        }
                        int cut[4], nc = 0;
                        for (int q = 0; q < 4; ++q)
                            if (cross[fe[q]]) cut[nc++] = fe[q];
                        if (nc == 0) continue;
                        /* pairs of cut edges and, for each pair, an outside corner on its outside side */
                        int pairs[2][2], outc[2], np = 0;
                        if (nc == 2) {
                            pairs[0][0] = cut[0], pairs[0][1] = cut[1];
                            outc[0] = -1;
                            for (int c = 0; c < 8; ++c)
                                if (((c >> a) & 1) == sd && !((inside >> c) & 1)) outc[0] = c;
                            np = 1;
                        } else {
                            /* each outside corner of the face is cut off with its two face edges */
                            for (int c = 0; c < 8; ++c) {
                                if (((c >> a) & 1) != sd || ((inside >> c) & 1)) continue;
                                int q2 = 0;
                                for (int q = 0; q < 4; ++q) {
                                    int c0, c1;
                                    edge_corners(cut[q], c0, c1);
                                    if (c0 == c || c1 == c) pairs[np][q2++] = cut[q];
                                }
                                outc[np++] = c;
                            }
                        }
                        const double N[3] = {a == 0 ? 2.0 * sd - 1.0 : 0.0, a == 1 ? 2.0 * sd - 1.0 : 0.0,
                                             a == 2 ? 2.0 * sd - 1.0 : 0.0};
                        for (int p = 0; p < np; ++p) {
                            /* unit-cube midpoints of the two edges */
                            double M[2][3];
                            for (int q = 0; q < 2; ++q) {
                                int c0, c1;
                                edge_corners(pairs[p][q], c0, c1);
                                for (int x = 0; x < 3; ++x) M[q][x] = 0.5 * (((c0 >> x) & 1) + ((c1 >> x) & 1));
                            }
                            const double d[3] = {M[1][0] - M[0][0], M[1][1] - M[0][1], M[1][2] - M[0][2]};
                            const double cr[3] = {N[1] * d[2] - N[2] * d[1], N[2] * d[0] - N[0] * d[2],
                                                  N[0] * d[1] - N[1] * d[0]};
                            double dot = 0.0;
                            for (int x = 0; x < 3; ++x)
                                dot += cr[x] * ((double)((outc[p] >> x) & 1) - 0.5 * (M[0][x] + M[1][x]));
                            if (dot > 0.0) next[pairs[p][0]] = pairs[p][1];
                            else next[pairs[p][1]] = pairs[p][0];
                        }
                    }
                /* loops, fanned from their lowest edge; a loop through all four surface points of
                 * one face is fanned around the mean of its vertices instead (a fan from one of
                 * those points would lay a triangle flat on the face, where the neighbouring cube
                 * lays its own) */
                bool seen[12] = {false};
                const uint32_t vox = (uint32_t)(i + mside * (j + mside * k));
                int nloops = 0;
                for (int e = 0; e < 12; ++e) {
                    if (!cross[e] || seen[e]) continue;
                    int loop[12], nl = 0;
                    for (int x = e; !seen[x]; x = next[x]) {
                        seen[x] = true;
                        loop[nl++] = x;
                    }
                    bool on_loop[12] = {false};
                    for (int q = 0; q < nl; ++q) on_loop[loop[q]] = true;
                    bool full_face = false;
                    for (int a = 0; a < 3; ++a)
                        for (int sd = 0; sd < 2; ++sd) {
                            int cnt = 0;
                            for (int x = 0; x < 12; ++x) {
                                if (edge_axis(x) == a || !on_loop[x]) continue;
                                int c0, c1;
                                edge_corners(x, c0, c1);
                                if (((c0 >> a) & 1) == sd) ++cnt;
                            }
                            if (cnt == 4) full_face = true;
                        }
                    const int centre_id = 20 + nloops++;
                    double centre[3] = {0.0, 0.0, 0.0};
                    if (full_face) {
                        for (int q = 0; q < nl; ++q)
                            for (int y = 0; y < 3; ++y) centre[y] += pos[loop[q]][y];
                        for (int y = 0; y < 3; ++y) centre[y] /= (double)nl;
                    }
                    const int ntri = full_face ? nl : nl - 2;
                    for (int q = 0; q < ntri; ++q) {
                        const double* p3[3];
                        int a3[3];
                        if (full_face) {
                            p3[0] = pos[loop[q]], a3[0] = vid[loop[q]];
                            p3[1] = pos[loop[(q + 1) % nl]], a3[1] = vid[loop[(q + 1) % nl]];
                            p3[2] = centre, a3[2] = centre_id;
                        } else {
                            p3[0] = pos[loop[0]], a3[0] = vid[loop[0]];
                            p3[1] = pos[loop[q + 1]], a3[1] = vid[loop[q + 1]];
                            p3[2] = pos[loop[q + 2]], a3[2] = vid[loop[q + 2]];
                        }
                        if (a3[0] == a3[1] || a3[1] == a3[2] || a3[0] == a3[2]) continue;
                        for (int x = 0; x < 3; ++x)
                            for (int y = 0; y < 3; ++y) o.verts->push_back(p3[x][y]);
                        for (int x = 0; x < 3; ++x) o.blocks->push_back(b[x]);
                        o.codes->push_back(((uint32_t)n << 30) | (vox << 15) | ((uint32_t)a3[0] << 10) |
                                           ((uint32_t)a3[1] << 5) | (uint32_t)a3[2]);
                        o.near->push_back(near ? 1 : 0);
                    }
                }
            }
}

struct MeshCache {
    std::vector<double> verts;
    std::vector<int32_t> blocks;
    std::vector<uint32_t> codes;
    std::vector<uint8_t> near;
};

}  // namespace

extern "C" {

void* orc_create(const orc_config* cfg) {
    if (!cfg || cfg->levels < 1 || cfg->levels > 4 || !(cfg->voxel > 0.0)) return nullptr;
    Map* m = new Map();
    m->cfg = *cfg;
    m->B = 8.0 * cfg->voxel;
    m->invB = 1.0 / m->B;
    for (int n = 0; n < 4; ++n) {
        m->nu[n] = cfg->voxel * (double)(1 << n);
        m->inv_nu[n] = 1.0 / m->nu[n];
    }
    return m;
}

void orc_destroy(void* map) { delete static_cast<Map*>(map); }

int orc_integrate_rgbd(void* map, const float* depth, const uint8_t* rgb, int32_t width, int32_t height,
                       const double K[4], const double T_ws[16]);

int orc_integrate_depth(void* map, const float* depth, int32_t width, int32_t height,
                        const double K[4], const double T_ws[16]) {
    return orc_integrate_rgbd(map, depth, nullptr, width, height, K, T_ws);
}

int orc_integrate_rgbd(void* map, const float* depth, const uint8_t* rgb, int32_t width, int32_t height,
                       const double K[4], const double T_ws[16]) {
    Map& m = *static_cast<Map*>(map);
    m.last = orc_stats{};
    const Pose P(T_ws);
    const double fx = K[0], fy = K[1], cx = K[2], cy = K[3];
    const double ifx = 1.0 / fx, ify = 1.0 / fy;
    const double tau = m.cfg.tau;

    /* 1-2: back-project every valid pixel and allocate the blocks its band [p - tau n, p + tau n]
     * crosses. */
    for (int v = 0; v < height; ++v)
        for (int u = 0; u < width; ++u) {
            const double d = (double)depth[(int64_t)v * width + u];
            if (!depth_ok(d, m.cfg.max_depth)) continue;
            m.last.valid_points++;
            const double ps[3] = {(((double)u - cx) * ifx) * d, (((double)v - cy) * ify) * d, d};
            double pw[3], n[3];
            P.apply(ps, pw);
            unit_dir(pw, P.t, n);
            const double a[3] = {pw[0] - tau * n[0], pw[1] - tau * n[1], pw[2] - tau * n[2]};
            const double e[3] = {pw[0] + tau * n[0], pw[1] + tau * n[1], pw[2] + tau * n[2]};
            if (!in_key_range(a, e, m.invB)) {
                m.last.dropped_points++;
                continue;
            }
            allocate(m, a, e);
        }

    /* 3: projective update of every voxel of every allocated block, at the block's level (Eq. 2). */
    for (auto& kv : m.blocks) {
        const Key& b = kv.first;
        Block& blk = kv.second;
        const int mm = side(blk.level);
        const int64_t obs_before = m.last.observations;
        for (int k = 0; k < mm; ++k)
            for (int j = 0; j < mm; ++j)
                for (int i = 0; i < mm; ++i) {
                    double c[3], x[3];
                    voxel_centre(m, b, blk.level, i, j, k, c);
                    P.inverse(c, x);
                    if (!(x[2] > 0.0)) continue;
                    const double iz = 1.0 / x[2];
                    const double uu = (fx * (x[0] * iz)) + cx;
                    const double vv = (fy * (x[1] * iz)) + cy;
                    const double fu = std::floor(uu + 0.5), fv = std::floor(vv + 0.5);
                    if (!(fu >= 0.0 && fu <= (double)(width - 1) && fv >= 0.0 && fv <= (double)(height - 1)))
                        continue;
                    const double d = (double)depth[(int64_t)fv * width + (int64_t)fu];
                    if (!depth_ok(d, m.cfg.max_depth)) continue;
                    double raw;
                    if (m.cfg.form == 0) {
                        /* measured range along the voxel's ray minus the voxel's range ||x|| */
                        const double nx = std::sqrt((x[0] * x[0] + x[1] * x[1]) + x[2] * x[2]);
                        raw = nx * ((d * iz) - 1.0);
                    } else {
                        raw = d - x[2];
                    }
                    if (raw < -tau) continue; /* occluded beyond the truncation band */
                    const double obs = raw < tau ? raw : tau;
                    const int vi = i + mm * (j + mm * k);
                    observe(blk, vi, obs);
                    m.last.observations++;
                    m.last.distinct_voxels++; /* one pixel per voxel: each update is a distinct voxel */
                    if (rgb) {
                        /* colour of the same pixel, averaged like the TSDF (Eq. 3 with w = 1) */
                        const size_t px = 3 * ((size_t)fv * width + (size_t)fu);
                        const double Wn = (double)blk.W[vi];
                        for (int ch = 0; ch < 3; ++ch) {
                            double& c = blk.C[3 * (size_t)vi + ch];
                            c = c + ((double)rgb[px + ch] - c) / Wn;
                        }
                    }
                }
        if (m.last.observations > obs_before) m.last.touched_blocks++;
    }

    /* 4: variance and merging criterion. */
    variance_and_merge(m);
    m.frame++;
    return 0;
}

int orc_integrate_points(void* map, const float* xyz, int64_t n, const double T_ws[16]) {
    Map& m = *static_cast<Map*>(map);
    m.last = orc_stats{};
    const Pose P(T_ws);
    const double tau = m.cfg.tau;
    const double r2lo = m.cfg.min_range * m.cfg.min_range;
    const double r2hi = m.cfg.max_range * m.cfg.max_range;

    struct Seg {
        double a[3], e[3], p[3], n[3];
    };
    std::vector<Seg> segs;
    segs.reserve((size_t)n);
    /* 1-2: valid points and allocation along each segment. */
    for (int64_t i = 0; i < n; ++i) {
        const double ps[3] = {(double)xyz[3 * i], (double)xyz[3 * i + 1], (double)xyz[3 * i + 2]};
        if (!(std::isfinite(ps[0]) && std::isfinite(ps[1]) && std::isfinite(ps[2]))) continue;
        const double r2 = (ps[0] * ps[0] + ps[1] * ps[1]) + ps[2] * ps[2];
        if (!(r2 >= r2lo && r2 <= r2hi)) continue;
        m.last.valid_points++;
        Seg s;
        P.apply(ps, s.p);
        unit_dir(s.p, P.t, s.n);
        for (int k = 0; k < 3; ++k) {
            s.a[k] = m.cfg.carve ? P.t[k] : s.p[k] - tau * s.n[k];
            s.e[k] = s.p[k] + tau * s.n[k];
        }
        if (!in_key_range(s.a, s.e, m.invB)) {
            m.last.dropped_points++;
            continue;
        }
        allocate(m, s.a, s.e);
        segs.push_back(s);
    }

    /* 3: every voxel a ray crosses, at its block's level, receives clip((p - x) . n, -tau, tau)
     * (Eq. 1); observations are applied in point order, then in walk order along each ray. */
    std::vector<std::array<int64_t, 3>> cells;
    std::vector<std::array<int, 3>> vox;
    std::map<Key, std::vector<char>> seen; /* voxels observed this scan, for the distinct count */
    for (const Seg& s : segs) {
        cells.clear();
        block_walk(s.a, s.e, m.invB, cells);
        for (const auto& c : cells) {
            const Key b{(int32_t)c[0], (int32_t)c[1], (int32_t)c[2]};
            Block& blk = m.blocks.at(b);
            const int mm = side(blk.level);
            vox.clear();
            voxel_walk(s.a, s.e, b, m.B, m.inv_nu[blk.level], mm, vox);
            for (const auto& v : vox) {
                double x[3];
                voxel_centre(m, b, blk.level, v[0], v[1], v[2], x);
                const double sd = ((s.p[0] - x[0]) * s.n[0] + (s.p[1] - x[1]) * s.n[1]) + (s.p[2] - x[2]) * s.n[2];
                const double obs = sd < -tau ? -tau : (sd > tau ? tau : sd);
                const int vi = v[0] + mm * (v[1] + mm * v[2]);
                observe(blk, vi, obs);
                m.last.observations++;
                std::vector<char>& sv = seen[b];
                if (sv.empty()) sv.assign((size_t)mm * mm * mm, 0);
                if (!sv[(size_t)vi]) {
                    sv[(size_t)vi] = 1;
                    m.last.distinct_voxels++;
                }
            }
        }
    }

    m.last.touched_blocks = (int64_t)seen.size();

    /* 4: variance and merging criterion. */
    variance_and_merge(m);
    m.frame++;
    return 0;
}

void orc_last_stats(const void* map, orc_stats* out) { *out = static_cast<const Map*>(map)->last; }

int64_t orc_num_blocks(const void* map) { return (int64_t) static_cast<const Map*>(map)->blocks.size(); }

int64_t orc_num_voxels(const void* map) {
    int64_t s = 0;
    for (const auto& kv : static_cast<const Map*>(map)->blocks) s += (int64_t)kv.second.W.size();
    return s;
}

void orc_extract(const void* map, int32_t* keys, uint8_t* levels, int64_t* offsets, double* D,
                 uint32_t* W, double* S2) {
    const Map& m = *static_cast<const Map*>(map);
    int64_t i = 0, off = 0;
    if (offsets) offsets[0] = 0;
    for (const auto& kv : m.blocks) {
        const Block& b = kv.second;
        if (keys) {
            keys[3 * i] = kv.first[0];
            keys[3 * i + 1] = kv.first[1];
            keys[3 * i + 2] = kv.first[2];
        }
        if (levels) levels[i] = (uint8_t)b.level;
        for (size_t v = 0; v < b.W.size(); ++v) {
            if (D) D[off + (int64_t)v] = b.D[v];
            if (W) W[off + (int64_t)v] = (uint32_t)b.W[v];
            if (S2) S2[off + (int64_t)v] = b.S2[v];
        }
        off += (int64_t)b.W.size();
        ++i;
        if (offsets) offsets[i] = off;
    }
}

int64_t orc_near_threshold(const void* map, int32_t* keys, int64_t* frames, double* margins, int64_t cap) {
    const Map& m = *static_cast<const Map*>(map);
    const int64_t n = (int64_t)m.near.size();
    for (int64_t i = 0; i < n && i < cap; ++i) {
        if (keys) {
            keys[3 * i] = m.near[i].key[0];
            keys[3 * i + 1] = m.near[i].key[1];
            keys[3 * i + 2] = m.near[i].key[2];
        }
        if (frames) frames[i] = m.near[i].frame;
        if (margins) margins[i] = m.near[i].margin;
    }
    return n;
}

void orc_query(const void* map, const float* pts, int64_t n, const double* T, int32_t strict,
               double* sdf, uint8_t* valid, double* grad_world) {
    const Map& m = *static_cast<const Map*>(map);
    static const double I4[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    const Pose P(T ? T : I4);
    for (int64_t i = 0; i < n; ++i) {
        const double p[3] = {(double)pts[3 * i], (double)pts[3 * i + 1], (double)pts[3 * i + 2]};
        double x[3];
        if (T) P.apply(p, x);
        else x[0] = p[0], x[1] = p[1], x[2] = p[2];
        const QueryOut q = query_one(m, x, strict != 0);
        if (sdf) sdf[i] = q.sdf;
        if (valid) valid[i] = q.valid ? 1 : 0;
        if (grad_world)
            for (int k = 0; k < 3; ++k) grad_world[3 * i + k] = q.grad[k];
    }
}

void orc_query_backward(const void* map, const float* pts, int64_t n, const double* T, int32_t strict,
                        const double* grad_sdf, double* grad_pts, double grad_pose[6]) {
    const Map& m = *static_cast<const Map*>(map);
    static const double I4[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    const Pose P(T ? T : I4);
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; ++i) {
        const double p[3] = {(double)pts[3 * i], (double)pts[3 * i + 1], (double)pts[3 * i + 2]};
        double x[3];
        if (T) P.apply(p, x);
        else x[0] = p[0], x[1] = p[1], x[2] = p[2];
        const QueryOut q = query_one(m, x, strict != 0);
        double g[3] = {0, 0, 0};
        if (q.valid)
            for (int k = 0; k < 3; ++k) g[k] = grad_sdf[i] * q.grad[k];
        /* dL/dp = R^T g; left perturbation x' = x + rho + phi x x gives dL/drho = g, dL/dphi = x x g */
        for (int r = 0; r < 3; ++r)
            grad_pts[3 * i + r] = (P.R[0][r] * g[0] + P.R[1][r] * g[1]) + P.R[2][r] * g[2];
        acc[0] += g[0];
        acc[1] += g[1];
        acc[2] += g[2];
        acc[3] += x[1] * g[2] - x[2] * g[1];
        acc[4] += x[2] * g[0] - x[0] * g[2];
        acc[5] += x[0] * g[1] - x[1] * g[0];
    }
    for (int k = 0; k < 6; ++k) grad_pose[k] = acc[k];
}

uint32_t orc_eq4_hash(int32_t x, int32_t y, int32_t z, uint64_t n_hash) {
    const uint32_t p1 = 73856093u, p2 = 19349669u, p3 = 83492791u;
    const uint32_t h = ((uint32_t)x * p1) ^ ((uint32_t)y * p2) ^ ((uint32_t)z * p3);
    return (uint32_t)((uint64_t)h % n_hash);
}

int64_t orc_block_dda(const double a[3], const double e[3], double inv_cell, int64_t* cells, int64_t cap) {
    std::vector<std::array<int64_t, 3>> out;
    block_walk(a, e, inv_cell, out);
    const int64_t n = (int64_t)out.size();
    for (int64_t i = 0; i < n && i < cap; ++i)
        for (int k = 0; k < 3; ++k) cells[3 * i + k] = out[i][k];
    return n;
}

int64_t orc_voxel_dda(const double a[3], const double e[3], const int32_t block[3], double block_edge,
                      double inv_voxel, int32_t m, int32_t* cells, int64_t cap) {
    std::vector<std::array<int, 3>> out;
    voxel_walk(a, e, Key{block[0], block[1], block[2]}, block_edge, inv_voxel, m, out);
    const int64_t n = (int64_t)out.size();
    for (int64_t i = 0; i < n && i < cap; ++i)
        for (int k = 0; k < 3; ++k) cells[3 * i + k] = out[i][k];
    return n;
}

int64_t orc_mesh(const void* map, double collapse, const int32_t* only_keys, int64_t n_only, double* verts,
                 int32_t* blocks, uint32_t* codes, uint8_t* near, int64_t cap) {
    const Map& m = *static_cast<const Map*>(map);
    MeshCache c;
    MeshOut o{&c.verts, &c.blocks, &c.codes, &c.near};
    if (only_keys) {
        for (int64_t q = 0; q < n_only; ++q) {
            const Key k{only_keys[3 * q], only_keys[3 * q + 1], only_keys[3 * q + 2]};
            auto it = m.blocks.find(k);
            if (it != m.blocks.end()) mesh_block(m, it->first, it->second, collapse, o);
        }
    } else {
        for (const auto& kv : m.blocks) mesh_block(m, kv.first, kv.second, collapse, o);
    }
    const int64_t n = (int64_t)c.codes.size();
    for (int64_t i = 0; i < n && i < cap; ++i) {
        if (verts)
            for (int q = 0; q < 9; ++q) verts[9 * i + q] = c.verts[9 * i + q];
        if (blocks)
            for (int q = 0; q < 3; ++q) blocks[3 * i + q] = c.blocks[3 * i + q];
        if (codes) codes[i] = c.codes[i];
        if (near) near[i] = c.near[i];
    }
    return n;
}

int orc_set_block(void* map, const int32_t key[3], int32_t level, const double* D, const uint32_t* W) {
    Map& m = *static_cast<Map*>(map);
    if (level < 0 || level >= m.cfg.levels) return -1;
    Block& b = m.blocks[Key{key[0], key[1], key[2]}];
    new_block(b, level);
    for (size_t v = 0; v < b.D.size(); ++v) {
        b.D[v] = D[v];
        b.W[v] = W[v];
    }
    return 0;
}

/*
 * Streaming region (Sec. 3.3): does block key[3] stay on the GPU?  The block's bounding sphere
 * (centre of the block, radius half its diagonal) is tested against the region: for a LiDAR scan
 * the ball of the given radius around the sensor origin; for an RGB-D frame the frustum of the
 * image's pixels (u in [-1/2, width - 1/2], v in [-1/2, height - 1/2]) in front of the camera,
 * bounded by the sphere of radius lambda (max_depth + tau) around it, lambda the largest ray
 * length per unit depth over the image corners.  The sphere meets the region when its centre lies
 * no farther than the radius outside each bounding surface.  margin receives the smallest of those
 * signed clearances (m): how far the decision is from flipping.
 */
int orc_region_holds(const void* map, int32_t kind, int32_t width, int32_t height, const double K[4],
                     const double T_ws[16], double radius, const int32_t key[3], double* margin) {
    const Map& m = *static_cast<const Map*>(map);
    const double Bm = m.B;
    const double c[3] = {((double)key[0] + 0.5) * Bm, ((double)key[1] + 0.5) * Bm, ((double)key[2] + 0.5) * Bm};
    const double rb = 0.5 * std::sqrt(3.0) * Bm;
    const Pose P(T_ws);
    const double d[3] = {c[0] - P.t[0], c[1] - P.t[1], c[2] - P.t[2]};
    double best;
    if (kind == 2) {
        best = radius + rb - std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    } else {
        double x[3];
        for (int r = 0; r < 3; ++r) x[r] = P.R[0][r] * d[0] + P.R[1][r] * d[1] + P.R[2][r] * d[2];
        const double ax[2] = {(-0.5 - K[2]) / K[0], ((double)width - 0.5 - K[2]) / K[0]};
        const double ay[2] = {(-0.5 - K[3]) / K[1], ((double)height - 0.5 - K[3]) / K[1]};
        const double xlo = std::min(ax[0], ax[1]), xhi = std::max(ax[0], ax[1]);
        const double ylo = std::min(ay[0], ay[1]), yhi = std::max(ay[0], ay[1]);
        double lam = 1.0;
        for (double a : ax)
            for (double b : ay) lam = std::max(lam, std::sqrt(1.0 + a * a + b * b));
        /* inward unit normals of the four side planes x = a z, y = b z */
        const double planes[4][3] = {{1.0, 0.0, -xlo}, {-1.0, 0.0, xhi}, {0.0, 1.0, -ylo}, {0.0, -1.0, yhi}};
        best = x[2] + rb;
        for (const auto& pl : planes) {
            const double nrm = std::sqrt(pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2]);
            best = std::min(best, (pl[0] * x[0] + pl[1] * x[1] + pl[2] * x[2]) / nrm + rb);
        }
        const double range = lam * (m.cfg.max_depth + m.cfg.tau);
        best = std::min(best, range + rb - std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]));
    }
    if (margin) *margin = best;
    return best >= 0.0 ? 1 : 0;
}

/*
 * Image-space quadtree by contrast (Sec. 3.5, Eq. 10, Algorithm 1).  Contrast of a node: the Rec. 601
 * luma weights l = (0.2989, 0.5870, 0.1140) times the per-channel mean squared deviation of its
 * pixels' RGB values from their mean (two passes, FP64).  Breadth first from the whole image: a
 * node whose contrast exceeds the threshold and whose size (its shorter side) exceeds the minimum
 * is split at the midpoints (x0 + w / 2, y0 + h / 2, rounded down) into top-left, bottom-left,
 * top-right and bottom-right children (children without pixels dropped); every other node is a
 * leaf.  Leaves are written as (x0, y0, w, h) in breadth-first order with their contrast; near
 * counts the split decisions (of nodes large enough to split, with nonzero contrast: a flat node's
 * zero is exact) within 1e-9 (relative) of the threshold.
 */
int64_t orc_quadtree(const uint8_t* rgb, int32_t width, int32_t height, double threshold, int32_t min_size,
                     int32_t* leaves, double* contrast, int64_t cap, int64_t* near) {
    struct Node {
        int32_t x, y, w, h;
    };
    static const double l[3] = {0.2989, 0.5870, 0.1140};
    if (min_size < 1 || width < 1 || height < 1) return -1;  /* a one-pixel node is always a leaf */
    std::vector<Node> queue{{0, 0, width, height}};
    int64_t nleaf = 0, nnear = 0;
    while (!queue.empty()) {
        std::vector<Node> next;
        for (const Node& q : queue) {
            const double n = (double)q.w * (double)q.h;
            double mean[3] = {0.0, 0.0, 0.0};
            for (int32_t y = q.y; y < q.y + q.h; ++y)
                for (int32_t x = q.x; x < q.x + q.w; ++x)
                    for (int c = 0; c < 3; ++c) mean[c] += (double)rgb[3 * ((size_t)y * width + x) + c];
            for (int c = 0; c < 3; ++c) mean[c] /= n;
            double sq[3] = {0.0, 0.0, 0.0};
            for (int32_t y = q.y; y < q.y + q.h; ++y)
                for (int32_t x = q.x; x < q.x + q.w; ++x)
                    for (int c = 0; c < 3; ++c) {
                        const double dv = (double)rgb[3 * ((size_t)y * width + x) + c] - mean[c];
                        sq[c] += dv * dv;
                    }
            double con = 0.0;
            for (int c = 0; c < 3; ++c) con += l[c] * (sq[c] / n);
            /* a split decision within rounding of the threshold (a flat node's zero is exact) */
            if (std::min(q.w, q.h) > min_size && con != 0.0 &&
                std::fabs(con - threshold) <= 1e-9 * std::max(1.0, std::fabs(threshold)))
                ++nnear;
            if (con > threshold && std::min(q.w, q.h) > min_size) {
                const int32_t wl = q.w / 2, ht = q.h / 2;
                const Node kids[4] = {{q.x, q.y, wl, ht}, {q.x, q.y + ht, wl, q.h - ht},
                                      {q.x + wl, q.y, q.w - wl, ht}, {q.x + wl, q.y + ht, q.w - wl, q.h - ht}};
                for (const Node& k : kids)
                    if (k.w > 0 && k.h > 0) next.push_back(k);
            } else {
                if (nleaf < cap) {
                    if (leaves) {
                        leaves[4 * nleaf] = q.x;
                        leaves[4 * nleaf + 1] = q.y;
                        leaves[4 * nleaf + 2] = q.w;
                        leaves[4 * nleaf + 3] = q.h;
                    }
                    if (contrast) contrast[nleaf] = con;
                }
                ++nleaf;
            }
        }
        queue.swap(next);
    }
    if (near) *near = nnear;
    return nleaf;
}

void orc_extract_color(const void* map, double* rgb) {
    const Map& m = *static_cast<const Map*>(map);
    int64_t off = 0;
    for (const auto& kv : m.blocks) {
        const Block& b = kv.second;
        for (size_t v = 0; v < b.C.size(); ++v) rgb[off + (int64_t)v] = b.C[v];
        off += (int64_t)b.C.size();
    }
}

}  // extern "C"
