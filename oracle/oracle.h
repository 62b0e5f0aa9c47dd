/*
 * CPU oracle of the MrHash fusion hot path (arXiv 2511.21459) -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 implementation of what the per-frame fusion computes, written from the
 * paper's text (Sec. 3, 3.1, 3.2, 3.2.1, 3.4; Eq. 1-3, 5, 6).  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.  It shares no code, header, table or
 * helper with the HIP library; the two are written independently from the same definitions.
 *
 * What pins each entry point against something other than itself is listed beside it; every
 * function here has such a pin (none is "parity unpinned").  The merge rule's readings (which
 * voxels enter the block mean, one level per frame, pooling) are fixed by the closed-form
 * threshold case and the conservation checks, not by a worked example from the paper.
 */
#ifndef MRH_ORACLE_H
#define MRH_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_config {
    double voxel;       /* finest voxel edge nu_0 (m); block edge is 8 * voxel */
    int32_t levels;     /* number of resolution levels L, 1..4 (level n holds (8>>n)^3 voxels) */
    int32_t min_obs;    /* voxels with W >= min_obs enter the block mean variance */
    double tau;         /* truncation distance (m) */
    double var_thr;     /* merge when the block mean variance is below this (m^2) */
    double max_depth;   /* RGB-D: valid depth is (0, max_depth] */
    double min_range;   /* LiDAR: valid range is [min_range, max_range] */
    double max_range;
    int32_t carve;      /* LiDAR: 1 = segment [o, p + tau n], 0 = band [p - tau n, p + tau n] */
    int32_t form;       /* RGB-D signed distance: 0 = range along the voxel ray, 1 = z difference */
} orc_config;

typedef struct orc_stats {
    int64_t valid_points;
    int64_t new_blocks;
    int64_t observations;      /* voxel updates applied (one per voxel per observation) */
    int64_t dropped_points;    /* valid points whose segment left the key range */
    int64_t merges[4];         /* merges out of level n this frame */
    int64_t near_threshold;    /* merge decisions with |mv - thr| / thr < 1e-3 this frame */
    int64_t distinct_voxels;   /* voxels with at least one observation this frame */
    int64_t candidate_keys;    /* block keys the allocation walks visited, repeats included */
    int64_t touched_blocks;    /* blocks with at least one observed voxel this frame */
} orc_stats;

void* orc_create(const orc_config* cfg);
void orc_destroy(void* map);

/* RGB-D projective fusion of one z-depth frame (Eq. 2, 3, 5).  depth is row-major H x W.
 * Pinned by: closed-form Eq. 2 values on a plane seen head-on by an identity camera and by a
 * yawed, pitched, rolled and translated one (both forms; the updated-voxel set and the allocated
 * blocks too); the sphere's zero crossing; a two-pass mean and variance of each voxel's
 * observation history (Eq. 3, 5, 6); the closed-form merge threshold of two planes. */
int orc_integrate_depth(void* map, const float* depth, int32_t width, int32_t height,
                        const double K[4], const double T_ws[16]);

/* RGB-D fusion with colour (Sec. 3: a voxel stores a colour): orc_integrate_depth, and every voxel
 * the frame updates also averages the RGB value of its pixel (rgb: 8-bit, H x W x 3 interleaved)
 * into its colour, C <- C + (c - C) / W with the voxel's updated weight; merging pools colour as
 * the weighted mean of the observed children.  Pinned by: a constant colour; the mean of the
 * per-frame colours of a plane seen by a fixed camera, through merges. */
int orc_integrate_rgbd(void* map, const float* depth, const uint8_t* rgb, int32_t width, int32_t height,
                       const double K[4], const double T_ws[16]);

/* Colours of all voxels, 3 per voxel, in the voxel order of orc_extract. */
void orc_extract_color(const void* map, double* rgb);

/* LiDAR ray fusion of one scan of n sensor-frame points (Eq. 1, 3, 5).
 * Pinned by: the exact voxel column of an axis-aligned beam holding clip(Zp - z); point-order
 * independence; free space merging to the coarsest level at exactly +tau; exact cell sets of the
 * traversals (below). */
int orc_integrate_points(void* map, const float* xyz, int64_t n, const double T_ws[16]);

void orc_last_stats(const void* map, orc_stats* out);
int64_t orc_num_blocks(const void* map);
int64_t orc_num_voxels(const void* map);

/* Blocks in ascending (x, y, z) key order.  offsets has num_blocks + 1 entries; D/W/S2 hold the
 * voxels of block i at [offsets[i], offsets[i+1]), x fastest.  Any output may be NULL. */
void orc_extract(const void* map, int32_t* keys, uint8_t* levels, int64_t* offsets,
                 double* D, uint32_t* W, double* S2);

/* Merge decisions taken within 5e-2 relative of the threshold so far: per event the block key,
 * the frame index and the relative margin |mv - thr| / thr.  Returns the total count; fills at
 * most cap. */
int64_t orc_near_threshold(const void* map, int32_t* keys, int64_t* frames, double* margins,
                           int64_t cap);

/* Trilinear SDF query (Sec. 3.4): T may be NULL (identity).  strict = 1 requires all 8 corners.
 * Pinned by: exact reproduction of a linear field on one level; the closed-form blend across a
 * boundary between two levels (corner values at their containing voxels' centres); the query
 * pose; axis finite differences of the returned gradient. */
void orc_query(const void* map, const float* pts, int64_t n, const double* T, int32_t strict,
               double* sdf, uint8_t* valid, double* grad_world);

/* Adjoint of orc_query: grad_pts = dL/dp (n x 3), grad_pose = dL/dxi for a left perturbation
 * xi = (rho, phi) of T (6 values).  Pinned by finite differences of the pose perturbation and the
 * chain rule through R. */
void orc_query_backward(const void* map, const float* pts, int64_t n, const double* T,
                        int32_t strict, const double* grad_sdf, double* grad_pts,
                        double grad_pose[6]);

/* Multi-resolution Marching Cubes (Sec. 3.4) over the whole map, or over the blocks listed in
 * only_keys (n_only keys, x y z each) when it is not NULL.  Each triangle gives 9 doubles (three
 * vertices, world metres, counter-clockwise seen from outside, D >= 0), its block key (3 ints), a
 * code (level << 30 | voxel << 15 | v0 << 10 | v1 << 5 | v2; voxel = i + m (j + m k); a vertex id
 * is an edge 0..11, after collapse 12 + corner, or 20 + k for the centre of the cube's k-th loop
 * when that loop is fanned around its centre) and a flag set when a decision of its cube
 * (a corner sign, a collapse, a badly conditioned crossing) lay within rounding of its threshold.
 * The rules (cube extents, transition truncation, corner interpolation, face segments, loop
 * fans, collapse) are stated in oracle.cpp.  Returns the number of triangles; fills at most cap.
 * Pinned by: vertices of linear fields on one level and across a level boundary lying on the
 * field's zero plane; closed sphere meshes whose every directed edge has its reverse (watertight,
 * consistently oriented) with vertices within the trilinear error of the sphere; the partition of
 * space by the cubes of a two-level map; the collapse distance. */
int64_t orc_mesh(const void* map, double collapse, const int32_t* only_keys, int64_t n_only, double* verts,
                 int32_t* blocks, uint32_t* codes, uint8_t* near, int64_t cap);

/* Streaming region test (Sec. 3.3): 1 when block key[3] lies inside the region of a sensor at
 * pose T_ws -- its bounding sphere meets the ball of `radius` around the sensor (kind 2, LiDAR) or
 * the camera frustum of a width x height image with intrinsics K bounded by the sphere of radius
 * lambda (max_depth + tau) (kind 1, RGB-D) -- else 0.  margin (may be NULL) receives the signed
 * clearance of the decision in metres.  Pinned by: blocks straight ahead, behind the camera, beside
 * the frustum and beyond its range at closed-form distances; every block holding a point of the
 * frustum (or ball) is inside; blocks farther than their diagonal from the region are outside. */
int orc_region_holds(const void* map, int32_t kind, int32_t width, int32_t height, const double K[4],
                     const double T_ws[16], double radius, const int32_t key[3], double* margin);

/* Image-space quadtree by contrast (Sec. 3.5, Eq. 10, Algorithm 1) of an interleaved 8-bit RGB
 * image (height x width x 3): breadth-first splitting of every node whose contrast (luma-weighted
 * per-channel mean squared deviation) exceeds `threshold` and whose shorter side exceeds
 * `min_size`, at the rounded-down midpoints.  Writes up to cap leaves (x0, y0, w, h) and their
 * contrast in breadth-first order, and the number of split decisions within 1e-9 of the
 * threshold to *near; returns the number of leaves.  Pinned by: a flat image (one leaf, zero
 * contrast); two flat halves (contrast in closed form); a checkerboard splitting down to the
 * minimum size; leaves tiling the image; every leaf below the threshold or at the minimum size. */
int64_t orc_quadtree(const uint8_t* rgb, int32_t width, int32_t height, double threshold, int32_t min_size,
                     int32_t* leaves, double* contrast, int64_t cap, int64_t* near);

/* Test hook: replace block key[3] by a level-`level` block holding D, W (voxels x fastest). */
int orc_set_block(void* map, const int32_t key[3], int32_t level, const double* D, const uint32_t* W);

/* Eq. 4: (x p1 xor y p2 xor z p3) mod n_hash, products and xor in 32-bit unsigned arithmetic.
 * The oracle's own map does not need it (a std::map keyed by block coordinates holds the blocks);
 * it is here to write the stored hash vectors the library's hash is checked against. */
uint32_t orc_eq4_hash(int32_t x, int32_t y, int32_t z, uint64_t n_hash);

/* The traversals, exposed for brute-force pins.  Return the number of cells written (<= cap).
 * Pinned by the exact (rational-arithmetic) set of cells each segment meets. */
int64_t orc_block_dda(const double a[3], const double e[3], double inv_cell, int64_t* cells,
                      int64_t cap);
int64_t orc_voxel_dda(const double a[3], const double e[3], const int32_t block[3], double block_edge,
                      double inv_voxel, int32_t m, int32_t* cells, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif
