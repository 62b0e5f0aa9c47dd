// Image-space quadtree by contrast (Sec. 3.5, Eq. 10, Algorithm 1), a standalone GPU kernel set.
//
// Contrast of a node Q: the Rec. 601 luma weights l = (0.2989, 0.5870, 0.1140) times the
// per-channel mean squared deviation of its pixels' RGB values from their mean (Eq. 10).  The
// quadtree is built breadth first from the whole image: a node whose contrast exceeds the threshold
// and whose shorter side exceeds the minimum size is split at the rounded-down midpoints into
// top-left, bottom-left, top-right and bottom-right children (children without pixels dropped);
// every other node is a leaf.
//
// The paper reduces each node's pixels in shared memory.  Here one pass builds summed-area tables
// of the channel values and of their squares (exact integers: 32-bit sums, 64-bit sums of
// squares), after which every node's sums come from four table reads, so each level of the tree
// costs a launch over its nodes rather than a pass over the image.  With S_c and Q_c the node's
// sums over its n pixels, n^2 times the channel variance is n Q_c - S_c^2, exact in 64 bits for
// images of up to 2^23 pixels; the contrast is then formed in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>

#include "mrhash.h"

namespace {

constexpr int64_t kMaxPixels = int64_t(1) << 23;
constexpr int kMaxLevels = 32;  // levels of the breadth-first build (at most log2(2^23) + 3 are used)

struct QtNode {
    int32_t x, y, w, h;
};

// Row pass: inclusive prefix sums along x of each channel and of its square, written at (y + 1,
// x + 1) of (H + 1) x (W + 1) planes whose row 0 and column 0 are zero.  One workgroup per row.
// Workgroup 0 also sets up the breadth-first build: the root node in the first queue, one node at
// level 0, none at the other levels and no leaves (counts: kMaxLevels level counts, then the u64
// leaf count).
__global__ __launch_bounds__(256) void k_sat_rows(const uint8_t* __restrict__ rgb, int32_t W, int32_t H,
                                                  uint32_t* __restrict__ S, unsigned long long* __restrict__ Q,
                                                  QtNode* __restrict__ queue0, uint32_t* __restrict__ counts) {
    const int32_t y = blockIdx.x;
    if (y == 0) {
        if (threadIdx.x == 0) queue0[0] = QtNode{0, 0, W, H};
        if (threadIdx.x < kMaxLevels + 2) counts[threadIdx.x] = threadIdx.x == 0 ? 1u : 0u;
    }
    const size_t pitch = (size_t)W + 1, plane = pitch * ((size_t)H + 1);
    const int per = (W + 255) / 256;
    const int x0 = threadIdx.x * per, x1 = min(W, x0 + per);
    uint32_t s[3] = {0, 0, 0};
    unsigned long long q[3] = {0, 0, 0};
    for (int x = x0; x < x1; ++x)
        for (int c = 0; c < 3; ++c) {
            const uint32_t v = rgb[3 * ((size_t)y * W + x) + c];
            s[c] += v;
            q[c] += (unsigned long long)(v * v);
        }
    __shared__ uint32_t ss[3][256];
    __shared__ unsigned long long sq[3][256];
    for (int c = 0; c < 3; ++c) ss[c][threadIdx.x] = s[c], sq[c][threadIdx.x] = q[c];
    __syncthreads();
    // inclusive scan of the per-thread totals (Hillis-Steele, 256 entries)
    for (int o = 1; o < 256; o <<= 1) {
        uint32_t a[3] = {0, 0, 0};
        unsigned long long b[3] = {0, 0, 0};
        if ((int)threadIdx.x >= o)
            for (int c = 0; c < 3; ++c) a[c] = ss[c][threadIdx.x - o], b[c] = sq[c][threadIdx.x - o];
        __syncthreads();
        for (int c = 0; c < 3; ++c) ss[c][threadIdx.x] += a[c], sq[c][threadIdx.x] += b[c];
        __syncthreads();
    }
    for (int c = 0; c < 3; ++c) {
        s[c] = threadIdx.x ? ss[c][threadIdx.x - 1] : 0u;
        q[c] = threadIdx.x ? sq[c][threadIdx.x - 1] : 0ull;
    }
    const size_t row = ((size_t)y + 1) * pitch;
    for (int x = x0; x < x1; ++x)
        for (int c = 0; c < 3; ++c) {
            const uint32_t v = rgb[3 * ((size_t)y * W + x) + c];
            s[c] += v;
            q[c] += (unsigned long long)(v * v);
            S[c * plane + row + x + 1] = s[c];
            Q[c * plane + row + x + 1] = q[c];
        }
    if (threadIdx.x < 3) {
        S[threadIdx.x * plane + row] = 0u;
        Q[threadIdx.x * plane + row] = 0ull;
    }
}

// Column pass: running sums down each column, in chunks of kColChunk rows so that the image's
// height is covered by many threads (consecutive threads take consecutive columns, so every row
// access is coalesced): the chunks' column sums, then the running sums within each chunk, started
// from the sum of the chunks above it (read together, independent loads).
constexpr int kColChunk = 16;

__global__ __launch_bounds__(64) void k_sat_cols_part(int32_t W, int32_t H, const uint32_t* __restrict__ S,
                                                      const unsigned long long* __restrict__ Q, uint32_t* __restrict__ TS,
                                                      unsigned long long* __restrict__ TQ) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x, k = blockIdx.y;
    if (x > W) return;
    const size_t pitch = (size_t)W + 1, plane = pitch * ((size_t)H + 1);
    const int32_t y0 = k * kColChunk + 1, y1 = min(H, y0 + kColChunk - 1);
    for (int c = 0; c < 3; ++c) {
        uint32_t s = 0;
        unsigned long long q = 0;
#pragma unroll
        for (int32_t r = 0; r < kColChunk; ++r) {
            const int32_t y = y0 + r;
            const size_t at = c * plane + (size_t)y * pitch + x;
            s += y <= y1 ? S[at] : 0u;
            q += y <= y1 ? Q[at] : 0ull;
        }
        TS[((size_t)k * 3 + c) * pitch + x] = s;
        TQ[((size_t)k * 3 + c) * pitch + x] = q;
    }
}

__global__ __launch_bounds__(64) void k_sat_cols_apply(int32_t W, int32_t H, uint32_t* __restrict__ S,
                                                       unsigned long long* __restrict__ Q, const uint32_t* __restrict__ TS,
                                                       const unsigned long long* __restrict__ TQ) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x, k = blockIdx.y;
    if (x > W) return;
    const size_t pitch = (size_t)W + 1, plane = pitch * ((size_t)H + 1);
    const int32_t y0 = k * kColChunk + 1, y1 = min(H, y0 + kColChunk - 1);
    for (int c = 0; c < 3; ++c) {
        if (k == 0) {
            S[c * plane + x] = 0u;
            Q[c * plane + x] = 0ull;
        }
        uint32_t s = 0;
        unsigned long long q = 0;
#pragma unroll 8
        for (int32_t j = 0; j < k; ++j) {
            s += TS[((size_t)j * 3 + c) * pitch + x];
            q += TQ[((size_t)j * 3 + c) * pitch + x];
        }
        // the chunk's rows read first (independent loads), then the running sums written
        uint32_t rs[kColChunk];
        unsigned long long rq[kColChunk];
#pragma unroll
        for (int32_t r = 0; r < kColChunk; ++r) {
            const int32_t y = y0 + r;
            const size_t at = c * plane + (size_t)y * pitch + x;
            rs[r] = y <= y1 ? S[at] : 0u;
            rq[r] = y <= y1 ? Q[at] : 0ull;
        }
#pragma unroll
        for (int32_t r = 0; r < kColChunk; ++r) {
            const int32_t y = y0 + r;
            if (y > y1) break;
            const size_t at = c * plane + (size_t)y * pitch + x;
            s += rs[r];
            q += rq[r];
            S[at] = s;
            Q[at] = q;
        }
    }
}

__device__ inline double node_contrast(const uint32_t* S, const unsigned long long* Q, int32_t W, int32_t H,
                                       const QtNode& nd) {
    const size_t pitch = (size_t)W + 1, plane = pitch * ((size_t)H + 1);
    const size_t a = (size_t)nd.y * pitch + nd.x, b = a + nd.w, c = ((size_t)nd.y + nd.h) * pitch + nd.x, d = c + nd.w;
    const unsigned long long n = (unsigned long long)nd.w * (unsigned long long)nd.h;
    const double l[3] = {0.2989, 0.5870, 0.1140};
    double con = 0.0;
    for (int k = 0; k < 3; ++k) {
        const uint32_t* s = S + k * plane;
        const unsigned long long* q = Q + k * plane;
        const unsigned long long sum = (unsigned long long)(s[d] - s[b] - s[c] + s[a]);
        const unsigned long long sq = q[d] - q[b] - q[c] + q[a];
        const unsigned long long v = n * sq - sum * sum;  // n^2 times the channel variance, exact
        con += l[k] * (double)v;
    }
    return con / ((double)n * (double)n);
}

// One breadth-first level: every node of the input queue is split into the output queue or written
// as a leaf (wave-aggregated appends).
__global__ __launch_bounds__(256) void k_qt_level(const uint32_t* __restrict__ S, const unsigned long long* __restrict__ Q,
                                                  int32_t W, int32_t H, double threshold, int32_t min_size,
                                                  const QtNode* __restrict__ in, const uint32_t* __restrict__ n_in,
                                                  QtNode* __restrict__ out, uint32_t* __restrict__ n_out,
                                                  int32_t* leaves, float* contrast, unsigned long long* n_leaves,
                                                  long long cap) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t count = *n_in;
    QtNode kids[4];
    int nk = 0;
    bool leaf = false;
    double con = 0.0;
    QtNode nd{0, 0, 0, 0};
    if (i < count) {
        nd = in[i];
        con = node_contrast(S, Q, W, H, nd);
        if (con > threshold && min(nd.w, nd.h) > min_size) {
            const int32_t wl = nd.w / 2, ht = nd.h / 2;
            const QtNode cand[4] = {{nd.x, nd.y, wl, ht}, {nd.x, nd.y + ht, wl, nd.h - ht},
                                    {nd.x + wl, nd.y, nd.w - wl, ht}, {nd.x + wl, nd.y + ht, nd.w - wl, nd.h - ht}};
            for (int k = 0; k < 4; ++k)
                if (cand[k].w > 0 && cand[k].h > 0) kids[nk++] = cand[k];
        } else {
            leaf = true;
        }
    }
    // children: per-lane counts, one atomic per wave
    const int lane = __lane_id();
    int incl = nk;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    const int wtot = __shfl(incl, 63);
    uint32_t base = 0;
    if (lane == 63 && wtot) base = atomicAdd(n_out, (uint32_t)wtot);
    base = (uint32_t)__shfl((int)base, 63);
    for (int k = 0; k < nk; ++k) out[base + (uint32_t)(incl - nk + k)] = kids[k];
    const unsigned long long lm = __ballot(leaf);
    if (lm) {
        unsigned long long lb = 0;
        const int first = __ffsll((long long)lm) - 1;
        if (lane == first) lb = atomicAdd(n_leaves, (unsigned long long)__popcll(lm));
        lb = ((unsigned long long)__shfl((int)(uint32_t)(lb >> 32), first) << 32) | (uint32_t)__shfl((int)(uint32_t)lb, first);
        if (leaf) {
            const long long at = (long long)(lb + (unsigned long long)__builtin_amdgcn_mbcnt_hi(
                                                        (uint32_t)(lm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)lm, 0)));
            if (at < cap) {
                if (leaves) {
                    leaves[4 * at] = nd.x;
                    leaves[4 * at + 1] = nd.y;
                    leaves[4 * at + 2] = nd.w;
                    leaves[4 * at + 3] = nd.h;
                }
                if (contrast) contrast[at] = (float)con;
            }
        }
    }
}

}  // namespace

struct mrh_quadtree {
    hipStream_t stream = nullptr;
    int32_t max_w = 0, max_h = 0;
    uint32_t* S = nullptr;
    unsigned long long* Q = nullptr;
    QtNode* queue[2] = {nullptr, nullptr};
    uint32_t* counts = nullptr;  // queue length of every level (kMaxLevels), then the leaf count (u64)
    unsigned long long* n_leaves = nullptr;
    size_t queue_cap = 0;
    uint32_t* TS = nullptr;      // column pass: per chunk of rows, channel and column
    unsigned long long* TQ = nullptr;
};

extern "C" {

mrh_status mrh_quadtree_create(int32_t max_width, int32_t max_height, void* stream, mrh_quadtree** out) {
    if (!out || max_width < 1 || max_height < 1 || (int64_t)max_width * max_height > kMaxPixels) return MRH_ERR_INVALID_ARG;
    *out = nullptr;
    mrh_quadtree* q = new mrh_quadtree();
    q->stream = static_cast<hipStream_t>(stream);
    q->max_w = max_width;
    q->max_h = max_height;
    const size_t plane = ((size_t)max_width + 1) * ((size_t)max_height + 1);
    // a level never holds more nodes than pixels
    q->queue_cap = (size_t)max_width * (size_t)max_height;
    const size_t chunks = ((size_t)max_height + kColChunk - 1) / kColChunk;
    bool ok = hipMalloc((void**)&q->S, 3 * plane * 4) == hipSuccess && hipMalloc((void**)&q->Q, 3 * plane * 8) == hipSuccess &&
              hipMalloc((void**)&q->queue[0], q->queue_cap * sizeof(QtNode)) == hipSuccess &&
              hipMalloc((void**)&q->queue[1], q->queue_cap * sizeof(QtNode)) == hipSuccess &&
              hipMalloc((void**)&q->counts, kMaxLevels * 4 + 8) == hipSuccess &&
              hipMalloc((void**)&q->TS, chunks * 3 * ((size_t)max_width + 1) * 4) == hipSuccess &&
              hipMalloc((void**)&q->TQ, chunks * 3 * ((size_t)max_width + 1) * 8) == hipSuccess;
    if (ok) q->n_leaves = reinterpret_cast<unsigned long long*>(q->counts + kMaxLevels);
    if (!ok) {
        mrh_quadtree_destroy(q);
        return MRH_ERR_OOM;
    }
    *out = q;
    return MRH_OK;
}

void mrh_quadtree_destroy(mrh_quadtree* q) {
    if (!q) return;
    if (q->stream) (void)hipStreamSynchronize(q->stream);
    else (void)hipDeviceSynchronize();
    void* ptrs[] = {q->S, q->Q, q->queue[0], q->queue[1], q->counts, q->TS, q->TQ};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete q;
}

mrh_status mrh_quadtree_build(mrh_quadtree* q, const uint8_t* rgb_dev, int32_t width, int32_t height, double threshold,
                              int32_t min_size, int32_t* leaves_dev, float* contrast_dev, int64_t cap, int64_t* n_leaves) {
    if (!q || !rgb_dev || !n_leaves || width < 1 || height < 1 || width > q->max_w || height > q->max_h || min_size < 1 ||
        cap < 0 || !(threshold == threshold))
        return MRH_ERR_INVALID_ARG;
    hipStream_t s = q->stream;
    // the summed-area tables; the row pass also puts the root in the first queue and clears the counts
    hipLaunchKernelGGL(k_sat_rows, dim3(height), dim3(256), 0, s, rgb_dev, width, height, q->S, q->Q, q->queue[0],
                       q->counts);
    const int32_t chunks = (height + kColChunk - 1) / kColChunk;
    const dim3 cg((unsigned)((width + 1 + 63) / 64), (unsigned)chunks);
    hipLaunchKernelGGL(k_sat_cols_part, cg, dim3(64), 0, s, width, height, q->S, q->Q, q->TS, q->TQ);
    hipLaunchKernelGGL(k_sat_cols_apply, cg, dim3(64), 0, s, width, height, q->S, q->Q, q->TS, q->TQ);
    // levels: a node's shorter side halves at each split, so the tree is at most
    // log2(min(width, height)) + 2 levels deep
    int depth = 1;
    for (int32_t side = std::min(width, height); side > 1; side = (side + 1) / 2) ++depth;
    const int64_t pixels = (int64_t)width * height;
    int64_t bound = 1;
    for (int d = 0; d <= depth; ++d) {
        const int cur = d & 1;
        const unsigned grid = (unsigned)((std::min(bound, pixels) + 255) / 256);
        hipLaunchKernelGGL(k_qt_level, dim3(grid), dim3(256), 0, s, q->S, q->Q, width, height, threshold, min_size,
                           q->queue[cur], q->counts + d, q->queue[cur ^ 1], q->counts + d + 1, leaves_dev,
                           contrast_dev, q->n_leaves, (long long)(leaves_dev || contrast_dev ? cap : 0));
        bound *= 4;
    }
    if (hipGetLastError() != hipSuccess) return MRH_ERR_HIP;
    unsigned long long n = 0;
    if (hipMemcpyAsync(&n, q->n_leaves, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return MRH_ERR_HIP;
    *n_leaves = (int64_t)n;
    if ((leaves_dev || contrast_dev) && (int64_t)n > cap) return MRH_ERR_BUFFER_TOO_SMALL;
    return MRH_OK;
}

}  // extern "C"
