/*
 * mrhash -- MI355X (gfx950) fusion of depth frames and LiDAR scans into a spatially hashed,
 * variance-adaptive multi-resolution TSDF voxel-block map (MrHash, arXiv 2511.21459).
 *
 * C ABI.  Every function is extern "C", never throws, and returns an mrh_status (0 = success,
 * negative = error) unless stated otherwise.  Arguments are plain host or device pointers and
 * sizes; "device" pointers must be device memory of the GPU the map was created on (for example
 * the data pointer of a torch tensor on that GPU).  The caller owns every buffer it passes in;
 * the library owns the map's own device memory and releases it in mrh_map_destroy.  No call
 * keeps a caller pointer after it returns.
 *
 * Streams.  A map is bound to one HIP stream at creation (a hipStream_t passed as void*; NULL
 * is the default stream).  All work is enqueued on that stream, asynchronously, unless a call
 * writes a host output (counts, host gradients, statistics) -- those calls synchronise the
 * stream before returning.  Errors a kernel detects (hash table full, heap full, block limit)
 * are latched in device memory and returned by the next synchronising call (mrh_sync,
 * mrh_extract_blocks with a count output, mrh_query_sdf_backward).
 */
#ifndef MRHASH_H
#define MRHASH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MRH_ABI_VERSION 2

typedef int32_t mrh_status;
enum {
    MRH_OK = 0,
    MRH_ERR_INVALID_ARG = -1,      /* null pointer, bad size, bad config, non-finite pose */
    MRH_ERR_OOM = -2,              /* device allocation failed */
    MRH_ERR_TABLE_FULL = -3,       /* a hash insert found no free slot within the probe limit */
    MRH_ERR_HEAP_FULL = -4,        /* a level's block heap had no free block */
    MRH_ERR_BUFFER_TOO_SMALL = -5, /* an output buffer is smaller than the result */
    MRH_ERR_HIP = -6,              /* a HIP runtime call failed; mrh_last_error has its text */
    MRH_ERR_BLOCK_LIMIT = -7       /* more distinct blocks than cfg.max_blocks */
};

/* Signed-distance form of the projective (RGB-D) update, Eq. 2 (Sec. 3.1). */
enum {
    MRH_FORM_RANGE = 0, /* range measured along the voxel's viewing ray minus ||x|| */
    MRH_FORM_ZDIFF = 1  /* depth minus the voxel's z (fronto-parallel distance) */
};

/* Storage precision of the voxel state (arithmetic is always FP32 in registers; the 16-bit formats
 * round to nearest even on store).  The 16-bit formats keep the per-voxel variance S2 / W divided
 * by tau^2 in place of S2; extraction returns S2 in m^2 for every format. */
enum {
    MRH_STORE_F32 = 0,  /* D: float metres, S2: float m^2                      | W: uint32 (12 B) */
    MRH_STORE_F16 = 1,  /* D: half of D / tau, variance: half of S2/(W tau^2)  | W: uint16, saturating (6 B) */
    MRH_STORE_BF16 = 2  /* D: bfloat16 of D / tau, variance: half, as for F16  | W: half, saturating (6 B) */
};
/* Weight ranges of the 16-bit formats: the uint16 weight is exact up to 65535 and saturates there;
 * the half weight is exact up to 2048, rounds to the nearest half above it (so one more observation
 * of a voxel with W >= 2048 may leave the stored W unchanged) and saturates at 65504.  A saturated
 * weight keeps averaging new observations as if W stayed at the cap. */

typedef struct mrh_config {
    double voxel;          /* finest voxel edge nu_0 (m); every block is 8 nu_0 wide (Sec. 3.2) */
    int32_t levels;        /* resolution levels L in [1, 4]; level n holds (8 >> n)^3 voxels */
    int32_t min_obs;       /* voxels with W >= min_obs enter the block mean variance (>= 1) */
    double tau;            /* truncation distance (m), > 0 (Sec. 3.1) */
    double var_thr;        /* merge a block whose mean voxel variance is below this (m^2) */
    double max_depth;      /* RGB-D: a depth d is valid iff finite and 0 < d <= max_depth */
    double min_range;      /* LiDAR: a point is valid iff min_range <= |p_s| <= max_range */
    double max_range;
    int32_t carve;         /* LiDAR: 1 = traverse [o, p + tau n], 0 = only [p - tau n, p + tau n] */
    int32_t form;          /* MRH_FORM_* */
    int64_t hash_slots;    /* open-addressing table size, a power of two >= 2 * max_blocks */
    int64_t max_blocks;    /* capacity of the block table (distinct block keys ever inserted) */
    int64_t heap_blocks[4];/* capacity of each level's block heap; 0 = max_blocks */
    int32_t storage;       /* MRH_STORE_* */
    int32_t max_probe;     /* linear-probe limit per lookup; 0 = 4096 */
    int32_t color;         /* 1 = voxels also store a colour (RGB float32, 12 B per voxel); such a map
                              fuses RGB-D frames through mrh_integrate_rgbd only, needs min_obs >= 2,
                              and is not streamed or batched */
} mrh_config;

typedef struct mrh_stats {
    int64_t frames;         /* frames integrated (totals) or since the previous mrh_sync (last) */
    int64_t valid_points;   /* valid pixels or points */
    int64_t dropped_points; /* valid points whose traversal left the 21-bit key range */
    int64_t new_blocks;     /* blocks inserted */
    int64_t observations;   /* voxel updates applied (one per voxel per observation) */
    int64_t merges[4];      /* merges out of level n */
    int64_t failed_inserts; /* inserts lost to a full table / heap / block limit */
    int64_t fresh_observations; /* of `observations`, those applied to blocks created this frame */
    int64_t blocks;         /* distinct blocks in the map after the frame */
    uint32_t error_flags;   /* bit 0 table full, bit 1 heap full, bit 2 block limit */
    uint32_t reserved;
    int64_t distinct_voxels;/* voxels that received at least one observation (per frame; RGB-D: the
                               observations, LiDAR: fewer, a voxel crossed by several rays counts once) */
    int64_t candidate_keys; /* block keys the allocation walks produced, before deduplication */
    int64_t queued_blocks;  /* blocks queued for the update: RGB-D, the existing blocks the visibility
                               cull keeps (new blocks are updated too); LiDAR, the blocks rays touched */
} mrh_stats;

typedef struct mrh_map mrh_map;

int32_t mrh_abi_version(void);

/* Home slot of block key (x, y, z) in a table of n_hash slots: Eq. 4 (Sec. 3.2),
 * ((x p1) xor (y p2) xor (z p3)) mod n_hash with p1 = 73856093, p2 = 19349669, p3 = 83492791,
 * evaluated in 32-bit unsigned wrap-around arithmetic.  Host function, no GPU needed. */
uint32_t mrh_block_hash(int32_t x, int32_t y, int32_t z, uint64_t n_hash);

/* Create an empty map (Sec. 3.2): allocates the hash table, the block table and one block heap
 * per level on the current HIP device, and clears them on `stream`.  *out receives the handle.
 * Errors: MRH_ERR_INVALID_ARG (cfg or out NULL, levels outside [1,4], voxel/tau <= 0,
 * hash_slots not a power of two or < 2 max_blocks, min_obs < 1), MRH_ERR_OOM, MRH_ERR_HIP. */
mrh_status mrh_map_create(const mrh_config* cfg, void* stream, mrh_map** out);

/* Release the map's device memory (synchronises its stream).  NULL is ignored. */
void mrh_map_destroy(mrh_map* map);

/* Empty the map in place (asynchronous): no blocks, all heaps free, counters and latched errors
 * cleared.  Device memory is kept. */
mrh_status mrh_map_reset(mrh_map* map);

/* Fuse one RGB-D frame (Sec. 3.1 "Cameras", Eq. 2, Eq. 3, Eq. 5; Sec. 3.2.1).
 *   depth_dev: device float32[height][width], z-depth in metres, row-major; pixel (u, v) =
 *              (column, row) has its centre at integer (u, v).  Non-finite, <= 0 or > max_depth
 *              values are skipped.
 *   K:         host double[4] = fx, fy, cx, cy.
 *   T_ws:      host double[16], row-major world-from-sensor rigid transform.
 * Steps: allocate at the finest level every block crossed by [p - tau n, p + tau n] for each valid
 * pixel, update every voxel of every allocated block that projects onto a valid pixel and lies
 * no more than tau behind it, then merge every updated block whose mean voxel variance is below
 * var_thr one level coarser.  Asynchronous.  Errors: MRH_ERR_INVALID_ARG (NULL pointers, sizes
 * <= 0 or >= 2^24, width * height >= 2^31, non-finite K or T_ws); MRH_ERR_OOM when the map's
 * per-tile depth summary (4 bytes per 16 x 16 pixels) cannot grow to a larger frame; kernel-side
 * capacity errors are latched (see top). */
mrh_status mrh_integrate_depth(mrh_map* map, const float* depth_dev, int32_t width, int32_t height,
                               const double K[4], const double T_ws[16]);

/* Fuse one RGB-D frame with colour into a map created with cfg.color = 1 (Sec. 3: a voxel stores a
 * colour).  The depth part is exactly mrh_integrate_depth; then a separate colour launch takes, for
 * every voxel the frame updated (the same projective decisions), the RGB value of its pixel into
 * the voxel's colour, C <- C + (c - C) / W with the voxel's updated weight (Eq. 3 with w = 1), and
 * pools the colour of a block the frame merged into its coarser block as the weighted mean of the
 * observed children (as the TSDF is pooled).
 *   rgb_dev: device uint8[height][width][3], interleaved, the same pixels as depth_dev.
 * Errors as mrh_integrate_depth; MRH_ERR_INVALID_ARG on a map without colour. */
mrh_status mrh_integrate_rgbd(mrh_map* map, const float* depth_dev, const uint8_t* rgb_dev, int32_t width,
                              int32_t height, const double K[4], const double T_ws[16]);

/* Colours of the map's voxels (device float32[n_voxels][3], RGB in [0, 255]; 0 where unobserved), in
 * the voxel order of mrh_extract_blocks.  MRH_ERR_BUFFER_TOO_SMALL (count still set) when
 * voxel_cap < n_voxels; rgb_dev NULL returns the count only.  Synchronises the stream. */
mrh_status mrh_extract_color(mrh_map* map, float* rgb_dev, int64_t voxel_cap, int64_t* n_voxels);

/* mrh_integrate_depth for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same two kernels and the same
 * result, but the per-tile depth summary (4 bytes per 16 x 16 pixels) lives in a fixed device
 * array of the library instead of a per-map buffer that grows with the frame, and the launch
 * profiler is bypassed.  The call itself allocates nothing (no hipMalloc, hipFree or event creation;
 * the map's own memory comes from mrh_map_create).  Limit: frames of at most 65536 tiles (e.g.
 * 4096 x 4096 pixels); larger frames return MRH_ERR_INVALID_ARG with the reason in mrh_last_error.
 * The array is shared by every call on one GPU and keeps the last call's contents (each call
 * rewrites the tiles it reads before reading them): calls that overlap on one GPU, on different
 * streams, race and must not be issued.  Other arguments and errors as mrh_integrate_depth. */
mrh_status mrh_integrate_depth_noalloc(mrh_map* map, const float* depth_dev, int32_t width, int32_t height,
                                       const double K[4], const double T_ws[16]);

/* Fuse one LiDAR scan (Sec. 3.1 "3D Point Cloud", Eq. 1, Eq. 3, Eq. 5; Sec. 3.2.1).
 *   xyz_dev: device float32[n][3] points in the sensor frame; non-finite points and points with
 *            range outside [min_range, max_range] are skipped.  n may be 0.
 *   T_ws:    host double[16], row-major world-from-sensor transform (origin o = its translation).
 * Every voxel each ray [o, p + tau n] (or [p - tau n, p + tau n] without carving) crosses, at its
 * block's level, receives clip((p - x) . n, -tau, tau).  Asynchronous. */
mrh_status mrh_integrate_points(mrh_map* map, const float* xyz_dev, int64_t n, const double T_ws[16]);

/* Fuse a recorded sequence: frames f = 0 .. n_frames-1 in order, exactly as n_frames calls of
 * mrh_integrate_depth (the frame loop runs in the library, not in the caller).
 *   depth_dev: device float32[n_frames][height][width];  T_ws: host double[n_frames][16].
 * Asynchronous.  Errors as mrh_integrate_depth; on a bad pose nothing is enqueued. */
mrh_status mrh_integrate_depth_sequence(mrh_map* map, const float* depth_dev, int32_t n_frames, int32_t width,
                                        int32_t height, const double K[4], const double* T_ws);

/* The same for LiDAR: xyz_dev device float32[n_frames][n][3] (n points per scan, NaN padding
 * allowed), T_ws host double[n_frames][16]. */
mrh_status mrh_integrate_points_sequence(mrh_map* map, const float* xyz_dev, int32_t n_frames, int64_t n,
                                         const double* T_ws);

/* Wait for the map's stream, then report.  last: the statistics of the frames integrated since
 * the previous mrh_sync (the last frame when called after every frame); totals: since the map's
 * creation or reset.  last / totals may be NULL.  Returns the first latched capacity error
 * (MRH_ERR_TABLE_FULL, MRH_ERR_HEAP_FULL, MRH_ERR_BLOCK_LIMIT) or MRH_OK, and clears the latch. */
mrh_status mrh_sync(mrh_map* map, mrh_stats* last, mrh_stats* totals);

/* Consistency of the map's bookkeeping (Sec. 3.1: the spatial hash of Eq. 4 from block keys to
 * blocks, and the per-level voxel heaps whose slots the blocks hold), for tests and debugging.
 * Waits for the stream, copies the hash table, the block rows, the free stacks and the pending-
 * free lists to host memory (about 25 bytes per hash slot and block row) and checks them against
 * each other; the device is not changed.  Call between frames.  Returns MRH_OK when the check ran
 * (out filled; out->consistent says whether every violation count is zero), or a HIP error.
 * With a latched capacity error the counts describe the degraded map and need not be zero. */
typedef struct mrh_check {
    int64_t blocks;            /* block rows handed out (up to max_blocks) */
    int64_t live_blocks;       /* rows holding a heap slot */
    int64_t slotless_blocks;   /* rows whose key found its level-0 heap empty */
    int64_t gone_blocks;       /* rows streamed out to the host store */
    int64_t table_keys;        /* keys in the hash table */
    int64_t tombstones;        /* table slots of streamed-out keys */
    int64_t idless_keys;       /* table keys inserted when the block table was full */
    int64_t free_slots[4];     /* free-stack entries per level */
    int64_t pending_slots[4];  /* slots freed by the last frame, returned by the next one */
    double mean_probe;         /* mean probe length of the present keys, slots (1 = home slot) */
    int32_t max_probe;         /* longest one */
    int32_t consistent;        /* 1 when the five counts below are all zero */
    /* violations */
    int64_t duplicate_keys;    /* a key in two table slots */
    int64_t unreachable_keys;  /* keys a probe from the home slot misses (empty slot first, beyond the
                                  probe limit) and rows the table does not lead to */
    int64_t bad_table_entries; /* table entries naming a row out of range, streamed out, or with
                                  another key */
    int64_t slot_conflicts;    /* heap slots out of range or claimed twice (rows, stacks, lists) */
    int64_t lost_slots;        /* heap slots neither held, free nor pending */
} mrh_check;
mrh_status mrh_map_check(mrh_map* map, mrh_check* out);

/* Trilinear SDF query (Sec. 3.4).  For each point p_i (device float32[n][3]) the world point is
 * x = T_wq p (T_wq host double[16] or NULL for identity).  The point's block fixes the lattice
 * of its level; the 8 surrounding lattice points take the TSDF of whichever voxel, at any level,
 * contains them; missing corners (no block or W = 0) are dropped and the weights renormalised.
 * strict = 1 instead requires all 8 corners.  Outputs (device): sdf float32[n] (0 where invalid),
 * valid uint8[n], grad float32[n][3] = d sdf / d x in the world frame (may be NULL).
 * Asynchronous.  n may be 0. */
mrh_status mrh_query_sdf(mrh_map* map, const float* pts_dev, int64_t n, const double* T_wq,
                         int32_t strict, float* sdf_dev, uint8_t* valid_dev, float* grad_dev);

/* Adjoint of mrh_query_sdf for L = sum_i g_i sdf_i, with g = grad_sdf_dev (device float32[n]):
 * grad_pts_dev (device float32[n][3]) = dL/dp_i, and grad_pose_host (host double[6]) = dL/dxi for
 * a left perturbation exp(xi) T_wq, xi = (rho, phi): the sum over points of (g_x, x cross g_x),
 * reduced deterministically in FP64.  Synchronises the stream. */
mrh_status mrh_query_sdf_backward(mrh_map* map, const float* pts_dev, int64_t n, const double* T_wq,
                                  int32_t strict, const float* grad_sdf_dev, float* grad_pts_dev,
                                  double grad_pose_host[6]);

/* Copy the map out (Sec. 3.2 hash entries: key b_j, level n_j, and the block's voxels).
 * Blocks are written in block-table order (blocks streamed out to the host store are not on the
 * GPU and are skipped); *n_blocks and *n_voxels (host) receive the counts.
 * Device outputs, each may be NULL: keys int32[n][3], levels uint8[n], offsets int64[n + 1]
 * (block i owns voxels [offsets[i], offsets[i+1])), D float32 (m), W uint32, S2 float32 (m^2)
 * with voxels x fastest.  With all outputs NULL only the counts are returned.  Returns
 * MRH_ERR_BUFFER_TOO_SMALL (counts still set) if block_cap < n_blocks or, when a voxel output is
 * given, voxel_cap < n_voxels.  Synchronises the stream. */
mrh_status mrh_extract_blocks(mrh_map* map, int32_t* keys_dev, uint8_t* levels_dev,
                              int64_t* offsets_dev, float* D_dev, uint32_t* W_dev, float* S2_dev,
                              int64_t block_cap, int64_t voxel_cap, int64_t* n_blocks,
                              int64_t* n_voxels);

/* Multi-resolution Marching Cubes (Sec. 3.4): the zero set of the TSDF as a triangle soup.
 * Each voxel (i, j, k) of a level-n block spans a cube from its centre to the next voxel centre
 * along +x, +y, +z; on the block's upper face that is the first voxel-centre plane of the face
 * neighbour, so a cube next to a finer block is truncated (the transition rule) and one next to a
 * coarser block stretched; a block without a face neighbour has no cubes on that face.  Corner
 * values are the trilinear interpolant of mrh_query_sdf (non-strict) at the corners; a cube with
 * an invalid corner is skipped.  Corners with D < 0 are inside; per face, crossing edges are
 * joined so that the inside corners of an ambiguous face stay connected; each loop of surface
 * points is fanned from its lowest edge, or around the mean of its vertices when it passes
 * through all four surface points of one face.  Vertex collapse: a surface point within
 * collapse * nu_n of an end of its edge moves onto that end (0 <= collapse < 0.5; 0 = off), and
 * triangles with two vertices on one point are dropped.
 *   verts_dev:  device float32[cap][3][3], world metres, counter-clockwise seen from outside
 *               (D >= 0), or NULL to count only;
 *   blocks_dev: device int32[cap][3], the block key of each triangle's cube, or NULL;
 *   codes_dev:  device uint32[cap], level << 30 | voxel << 15 | v0 << 10 | v1 << 5 | v2 with
 *               voxel = i + m (j + m k) (m = 8 >> level) and vertex ids 0..11 (a surface point on
 *               that cube edge), 12 + c (collapsed onto corner c = x + 2 y + 4 z) or 20 + k (the
 *               centre of the cube's k-th loop), or NULL.
 * Edge e lies along axis e / 4; bits 0 and 1 of e % 4 are its coordinates on the other two axes in
 * increasing order.  Triangles come in no particular order.  *n_tris (host) receives the count;
 * MRH_ERR_BUFFER_TOO_SMALL (count still set, the first cap triangles written) when it exceeds cap.
 * Errors: MRH_ERR_INVALID_ARG (NULL map or n_tris, cap < 0, collapse outside [0, 0.5), blocks or
 * codes without verts).  Synchronises the stream. */
mrh_status mrh_extract_mesh(mrh_map* map, double collapse, float* verts_dev, int32_t* blocks_dev,
                            uint32_t* codes_dev, int64_t cap, int64_t* n_tris);

/* Kernel ids of the launch profiler. */
enum {
    MRH_KERNEL_RESET = 0,
    MRH_KERNEL_ALLOC_DEPTH = 1,     /* RGB-D allocation (back-projection, band walk, insert) */
    MRH_KERNEL_INTEGRATE_DEPTH = 2, /* RGB-D projective update, variance, merge */
    MRH_KERNEL_FINALIZE = 3,        /* reserved: the frame hand-off runs inside the other launches; stays 0 */
    MRH_KERNEL_ALLOC_POINTS = 4,    /* LiDAR allocation */
    MRH_KERNEL_RAYS = 5,            /* LiDAR ray traversal and accumulation, then queueing of touched blocks */
    MRH_KERNEL_APPLY_POINTS = 6,    /* LiDAR state update, variance, merge */
    MRH_KERNEL_QUERY = 7,
    MRH_KERNEL_QUERY_BACKWARD = 8,
    MRH_KERNEL_REDUCE = 9,
    MRH_KERNEL_BATCH_ALLOC = 10,    /* batched: allocation + cull of every map */
    MRH_KERNEL_BATCH_RAYS = 11,     /* batched: LiDAR traversal of every map */
    MRH_KERNEL_BATCH_UPDATE = 12,   /* batched: update tasks of every map */
    MRH_KERNEL_BATCH_FINALIZE = 13, /* reserved, as MRH_KERNEL_FINALIZE; stays 0 */
    MRH_KERNEL_BATCH_GRAPH = 14,    /* batched: one replay of the captured step */
    MRH_KERNEL_MESH = 15,           /* multi-resolution Marching Cubes (with its block ordering by level) */
    MRH_KERNEL_COLOR = 16,          /* colour integration of an RGB-D frame */
    MRH_KERNEL_COUNT = 17
};

/* Launch profiler (measurement support, not part of the method).  With on != 0 every kernel the
 * map launches is bracketed by a pair of HIP events on the map's stream.  mrh_profile_collect
 * synchronises the stream and writes, for kernel ids 0 .. n_kernels-1, the summed event time in
 * milliseconds (ms, host double[n_kernels]) and the number of launches (launches, host
 * int64[n_kernels]) since the last collect, then recycles the events. */
mrh_status mrh_profile_enable(mrh_map* map, int32_t on);
mrh_status mrh_profile_collect(mrh_map* map, double* ms, int64_t* launches, int32_t n_kernels);

/* ---- Batched fusion of many independent maps ------------------------------------------------
 * One call fuses one frame into each map of the batch with at most five launches in total
 * (allocation and culling of every map, LiDAR traversal of the LiDAR maps and the queueing of the
 * blocks it touched, and one update launch per frame kind present), captured once into a HIP graph and replayed on later calls with the same
 * frame kinds and sizes; each frame's hand-offs run inside these launches as in the single-map
 * calls.  Per-map
 * results are identical to calling mrh_integrate_depth / mrh_integrate_points map by map. */

enum { MRH_FRAME_NONE = 0, MRH_FRAME_DEPTH = 1, MRH_FRAME_POINTS = 2 };

typedef struct mrh_frame {
    int32_t kind;          /* MRH_FRAME_* (NONE leaves the map untouched this call) */
    int32_t width, height; /* DEPTH: image size */
    const float* data_dev; /* DEPTH: float32[height][width] z-depth (m); POINTS: float32[n][3] */
    int64_t n;             /* POINTS: number of points */
    double K[4];           /* DEPTH: fx, fy, cx, cy */
    double T_ws[16];       /* row-major world-from-sensor transform */
} mrh_frame;

typedef struct mrh_batch mrh_batch;

/* Group n_maps maps (same device, same storage format, same stream) into a batch.  The batch
 * enqueues on that stream.  The batch keeps the map pointers (the maps must outlive it).
 * Errors: MRH_ERR_INVALID_ARG (NULL or repeated maps, n_maps outside [1, 64], maps on different
 * devices or streams or with different storage formats), MRH_ERR_HIP. */
mrh_status mrh_batch_create(mrh_map* const* maps, int32_t n_maps, mrh_batch** out);
void mrh_batch_destroy(mrh_batch* batch);

/* Fuse frames[i] into map i for every i (host array of n_maps descriptors; device data).
 * Asynchronous.  Errors: MRH_ERR_INVALID_ARG (bad descriptor), MRH_ERR_HIP. */
mrh_status mrh_batch_integrate(mrh_batch* batch, const mrh_frame* frames);

/* Launch shape of the batched kernels: params[0] = workgroups of the update launch, params[1] =
 * cull workgroups per depth map, params[2] = 1 to replay a captured graph, 0 to launch directly,
 * params[3] = waves per workgroup of the update launch (1, 2 or 4; a wave takes one task at a time,
 * so this sets how many tasks share a workgroup's start-up and statistics flush). */
mrh_status mrh_batch_set_launch(mrh_batch* batch, const int32_t params[4]);
mrh_status mrh_batch_get_launch(const mrh_batch* batch, int32_t params[4]);

/* Autotuner: for every candidate launch shape (update workgroups x cull workgroups x waves per
 * update workgroup), reset all maps and time `reps` calls of mrh_batch_integrate(frames) with HIP
 * events; keep the fastest shape (written to best[4]) and leave every map reset.  Meant for
 * start-up, before the real stream of frames. */
mrh_status mrh_batch_autotune(mrh_batch* batch, const mrh_frame* frames, int32_t reps, int32_t best[4]);

/* ---- Capacity-driven streaming (Sec. 3.3) -------------------------------------------------
 * Voxel blocks move between the GPU heaps and a host store owned by the map.  Streaming out is
 * deferred until the fullest level heap is filled to a threshold; then every block outside the current
 * sensor region leaves the GPU.  A block lies inside a region when its bounding sphere (block
 * centre, radius half the block diagonal) meets the camera frustum (RGB-D: the image's pixel
 * frustum up to max_depth + tau along the rays, the update's conservative cull) or the ball around
 * the sensor origin (LiDAR).  Streaming out and in is exact: a block comes back with the bits it
 * left with (voxels in the storage format, variance sums), so fusing frames with every region
 * streamed in first gives the map of fusing them without streaming.  Block ids are not reused:
 * max_blocks bounds the keys ever inserted (24 B each), the heaps bound the voxel memory.  The
 * calls synchronise the stream and run between frames. */

typedef struct mrh_region {
    int32_t kind;          /* MRH_FRAME_DEPTH (camera frustum) or MRH_FRAME_POINTS (ball) */
    int32_t width, height; /* DEPTH: image size */
    double K[4];           /* DEPTH: fx, fy, cx, cy */
    double T_ws[16];       /* sensor pose, row-major world-from-sensor */
    double radius;         /* POINTS: ball radius (m) around the pose's origin */
} mrh_region;

/* Fill of the voxel memory: the largest fraction of a level's heap in use (slots not on its free
 * stack).  Each level has its own heap, so the fullest one is the one that runs out. */
mrh_status mrh_heap_usage(mrh_map* map, double* frac);

/* If the heap usage is at least `threshold` (e.g. 0.85; 0 = always), move every block outside
 * `region` to the host store; *n_out receives the number moved.  Errors: MRH_ERR_INVALID_ARG (bad
 * region), MRH_ERR_OOM, MRH_ERR_HIP. */
mrh_status mrh_stream_out(mrh_map* map, const mrh_region* region, double threshold, int64_t* n_out);

/* Move every stored block inside `region` back to the GPU (call before fusing a frame of that
 * region); *n_in receives the number moved.  A stored key that exists on the GPU again (created by
 * a frame fused while it was stored) stays in the store.  Errors: MRH_ERR_HEAP_FULL or
 * MRH_ERR_BLOCK_LIMIT when the free heap slots or block ids cannot hold them (nothing is moved). */
mrh_status mrh_stream_in(mrh_map* map, const mrh_region* region, int64_t* n_in);

/* Counts of the host store: blocks, voxels and host bytes (each may be NULL). */
mrh_status mrh_store_info(mrh_map* map, int64_t* n_blocks, int64_t* n_voxels, int64_t* bytes);

/* Copy the host store out in ascending packed-key order, decoded as mrh_extract_blocks does but
 * into host buffers: keys int32[n][3], levels uint8[n], offsets int64[n + 1], D float32, W uint32,
 * S2 float32 (voxels x fastest).  NULL outputs are skipped; MRH_ERR_BUFFER_TOO_SMALL when
 * block_cap / voxel_cap are below the counts (which are still set). */
mrh_status mrh_store_extract(mrh_map* map, int32_t* keys_host, uint8_t* levels_host, int64_t* offsets_host,
                             float* D_host, uint32_t* W_host, float* S2_host, int64_t block_cap, int64_t voxel_cap,
                             int64_t* n_blocks, int64_t* n_voxels);

/* Load blocks held by the caller (host arrays as mrh_extract_blocks returns them: keys int32[n][3],
 * levels uint8[n], and the voxels of block after block, x fastest, (8 >> level)^3 each: D float32
 * (m), W uint32, S2 float32 (m^2)) into the map, e.g. blocks saved from an earlier session.  Values
 * are rounded to the storage format; the block's variance sums are recomputed from its voxels.
 * Keys already in the map are left alone; *n_loaded receives the number loaded.  Errors:
 * MRH_ERR_INVALID_ARG (bad level or key), MRH_ERR_HEAP_FULL, MRH_ERR_BLOCK_LIMIT (nothing loaded). */
mrh_status mrh_load_blocks(mrh_map* map, int64_t n, const int32_t* keys_host, const uint8_t* levels_host,
                           const float* D_host, const uint32_t* W_host, const float* S2_host, int64_t* n_loaded);

/* ---- Image-space quadtree by contrast (Sec. 3.5, Eq. 10, Algorithm 1) ------------------------
 * Standalone (no map).  Contrast of a node: the Rec. 601 luma weights (0.2989, 0.5870, 0.1140)
 * times the per-channel mean squared deviation of its pixels' RGB values from their mean (Eq. 10).
 * Breadth first from the whole image, a node whose contrast exceeds `threshold` and whose shorter
 * side exceeds `min_size` (>= 1) is split at (x0 + w / 2, y0 + h / 2), rounded down, into top-left,
 * bottom-left, top-right and bottom-right children (children without pixels dropped); every other
 * node is a leaf.  Images of up to 2^23 pixels. */
typedef struct mrh_quadtree mrh_quadtree;

/* Buffers for images of up to max_width x max_height (summed-area tables, 36 B per pixel, and two
 * node queues), bound to `stream`.  Errors: MRH_ERR_INVALID_ARG, MRH_ERR_OOM. */
mrh_status mrh_quadtree_create(int32_t max_width, int32_t max_height, void* stream, mrh_quadtree** out);
void mrh_quadtree_destroy(mrh_quadtree* qt);

/* Leaves of the quadtree of an 8-bit RGB image (device uint8[height][width][3], interleaved):
 * leaves_dev device int32[cap][4] = (x0, y0, w, h) and contrast_dev device float32[cap] (either may
 * be NULL; both NULL counts only), in no particular order; *n_leaves (host) receives the count.
 * MRH_ERR_BUFFER_TOO_SMALL (count still set) when it exceeds cap.  Synchronises the stream. */
mrh_status mrh_quadtree_build(mrh_quadtree* qt, const uint8_t* rgb_dev, int32_t width, int32_t height, double threshold,
                              int32_t min_size, int32_t* leaves_dev, float* contrast_dev, int64_t cap, int64_t* n_leaves);

/* ---- Storage conversions (for checking the 16-bit formats) ---------------------------------
 * The conversions the 16-bit storage formats apply, element by element: storage MRH_STORE_F16
 * (IEEE binary16) or MRH_STORE_BF16 (bfloat16), both rounding to nearest with ties to even and
 * keeping NaN a NaN.  decode = 0: float32[n] -> uint16[n] bit patterns; decode = 1: uint16[n] ->
 * float32[n].  mrh_codec_device runs the device codecs the fusion kernels use (device pointers,
 * the null stream, synchronous); mrh_codec_host their host counterparts (host pointers; no GPU
 * needed).  Errors: MRH_ERR_INVALID_ARG (another storage, n < 0, NULL with n > 0); MRH_ERR_HIP. */
mrh_status mrh_codec_device(int32_t storage, int32_t decode, const void* in_dev, void* out_dev, int64_t n);
mrh_status mrh_codec_host(int32_t storage, int32_t decode, const void* in, void* out, int64_t n);

/* Text of the last error on this map (never NULL; "" when none). */
const char* mrh_last_error(const mrh_map* map);

#ifdef __cplusplus
}
#endif
#endif /* MRHASH_H */
