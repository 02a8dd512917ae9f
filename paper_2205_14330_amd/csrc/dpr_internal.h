// Internal definitions shared by the HIP sources of libdpr (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpr.h"

namespace dpr {

constexpr int kTile = 16;                 // screen tile edge in pixels
constexpr int kTilePix = kTile * kTile;   // 256 pixels per tile
constexpr int kChunkItems = 512;          // depth-sorted items per binning chunk
constexpr int kBandTiles = 8192;          // tiles of one view handled per LDS band
constexpr int kSegChunks = 16;            // chunks per column-scan segment
constexpr int kBwdSeg = 256;              // list positions per backward work item
constexpr int kSortThreads = 256;
constexpr int kSortItemsPerThread = 8;
constexpr int kSortTile = kSortThreads * kSortItemsPerThread;   // 2048 keys per sort block
constexpr int kDepthSortThreads = 1024;
constexpr int kDepthSortTile = 8 * kDepthSortThreads;              // 8192 keys per depth-sort block
constexpr int kScanThreads = 256;
constexpr int kScanItemsPerThread = 8;
constexpr int kScanTile = kScanThreads * kScanItemsPerThread;   // 2048 elements per scan block
constexpr uint32_t kDroppedKey = 0xFFFFFFFFu;
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kTwoPi = 6.283185307179586f;

// Per-view descriptor in device memory.
struct ViewDesc {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    int32_t tiles_x, tiles_y;
    int32_t scene;
    int32_t sh_degree;
    int32_t n;                  // points of the scene
    uint32_t item_off;          // first item id of this view
    uint32_t tile_off;          // first global tile id of this view
    uint32_t chunk_off;         // first global chunk id of this view
    uint32_t nchunks;           // chunks of this view
    uint32_t sort_block_off;    // first depth-sort block of this view
    uint32_t nsort_blocks;
    uint32_t pad0;
    uint64_t hist_off;          // first radix-histogram entry of this view
    uint64_t cnt_off;           // first (chunk, tile) count entry of this view (chunk-major)
    uint64_t seg_off;           // first (segment, tile) partial-sum entry of this view
    uint64_t pix_off;           // first pixel of this view in per-pixel state arrays
    const float *xyz;
    const float *sh;
    const float *opacity;
    const float *radius;
    float *image;
    float *trans;
};

// Per-scene descriptor in device memory.
struct SceneDesc {
    int32_t n;
    int32_t sh_degree;
    uint32_t view_start;        // into the scene -> view index list
    uint32_t view_count;
    uint32_t block_off;         // first point-parallel block of this scene
    uint32_t pad0;
    const float *xyz;
    const float *sh;
    const float *opacity;
    const float *radius;
    float *dxyz;                // backward outputs (may be null)
    float *dsh;
    float *dopacity;
};

struct Thresholds {
    float lambda;      // -log2(alpha_min): candidate iff w - q >= -lambda
    float alpha_max;
    float t_min;
    float z_near;
    int32_t sh_frame;
    uint32_t max_splats;   // 0: no per-pixel cap
    int32_t kernel_norm;   // 1: w carries log2 (2 pi sx sy)^-1/2
};

// Splat record of one (view, point) item: 32 bytes.
struct __align__(16) SplatRec {
    float px, py, a, b;     // centre (pixels) and a = log2e / (2 sx^2), b = log2e / (2 sy^2)
    float w, cr, cg, cb;    // w = log2(o); colour
};

// Binning record of one item in depth order (32 bytes), written by the tile
// count and read by the emission: the item's tile rectangle, its id and
// everything the (splat, tile) test reads, so the emission reads its items
// contiguously instead of gathering two records per item by id.
struct __align__(16) BinRec {
    uint32_t rx, ry;        // tile rectangle (x0 | y0 << 16, x1 | y1 << 16)
    uint32_t g;             // item id
    float thr;              // w + lambda, the bound of the (splat, tile) test
    float px, py, a, b;     // centre and axis coefficients of the splat record
};

// Index of the segment containing x: largest s < n with starts[s] <= x.
__device__ __forceinline__ int find_segment(const uint32_t *starts, int n, uint32_t x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (starts[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Workgroups are dispatched to the 8 XCDs round-robin (block b -> XCD b % 8).
// This maps block b to a work index so that each XCD gets one contiguous range
// of work items (neighbouring items share data, which then stays in one L2).
// It is a bijection of [0, total).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t total) {
    const uint32_t q = total >> 3, r = total & 7u;
    const uint32_t x = b & 7u, i = b >> 3;
    return x * q + min(x, r) + i;
}

// Camera-space depth key, shared by the cull, the sort and the chain rule:
// Z32 = fmaf(R20, x, fmaf(R21, y, fmaf(R22, z, t2))).
__device__ __forceinline__ float depth_z(const float *R, const float *t, float x, float y, float z) {
    float acc = __fmaf_rn(R[8], z, t[2]);
    acc = __fmaf_rn(R[7], y, acc);
    return __fmaf_rn(R[6], x, acc);
}

// Exponent of the splat opacity: e = w - (a dx^2 + b dy^2); alpha = 2^e.
// Evaluated as (w - b dy^2) - a dx^2 with two FMAs: the row term w - b dy^2 is
// shared by the pixels of a row.  Written with explicit rounding so every
// kernel that re-evaluates a splat (forward, recompute, backward) takes
// bit-identical decisions.
__device__ __forceinline__ float splat_exponent(const SplatRec &s, float ux, float uy, float &dx, float &dy) {
    dx = __fsub_rn(s.px, ux);
    dy = __fsub_rn(s.py, uy);
    return __fmaf_rn(-s.a, __fmul_rn(dx, dx), __fmaf_rn(-s.b, __fmul_rn(dy, dy), s.w));
}

// Conservative test of whether any pixel centre of tile (tx, ty) can pass the
// candidate predicate a dx^2 + b dy^2 <= thr of a splat centred at (px, py):
// the quadratic form at the point of the tile's pixel-centre box closest to
// the centre is a lower bound for every pixel of the tile.  The count and emit
// kernels must take the same decision for every (splat, tile) pair (the count
// sizes each tile's list, the emission fills it), so the arithmetic is fixed:
// contraction is off and every operation rounds once.  (Left to the compiler,
// the two kernels fused different products into FMAs, and about one decision
// in 5e7 differed.)
__device__ __forceinline__ float box_form(float px, float py, float a, float b, float x0, float x1, float y0,
                                          float y1) {
#pragma clang fp contract(off)
    // the box's point nearest to the splat centre: px clamped to [x0, x1]
    // (med3 returns that same value, in one instruction)
    const float cx = __builtin_amdgcn_fmed3f(px, x0, x1);
    const float cy = __builtin_amdgcn_fmed3f(py, y0, y1);
    const float dx = cx - px, dy = cy - py;
    const float qx = (a * dx) * dx, qy = (b * dy) * dy;
    return qx + qy;
}

__device__ __forceinline__ bool splat_touches_tile(float px, float py, float a, float b, float thr, uint32_t tx,
                                                   uint32_t ty) {
#pragma clang fp contract(off)
    const float x0 = (float)(tx * kTile) + 0.5f, y0 = (float)(ty * kTile) + 0.5f;
    const float q = box_form(px, py, a, b, x0, x0 + (float)(kTile - 1), y0, y0 + (float)(kTile - 1));
    return q <= thr * (1.0f + 1.0f / 1024.0f) + 1.0e-6f;
}

// The same lower bound over the pixel centres [x0, x1] x [y0, y1], with a
// margin that covers the rounding of the per-pixel exponent of splat_exponent
// (a few ulps of |w| + lambda + q, below 1e-5 for |w| < 80): if the test fails,
// no pixel centre of the box passes e >= -lambda.  The forward uses it to skip
// records that cannot reach any of a wave's live pixels.
__device__ __forceinline__ bool splat_reaches_box(float px, float py, float a, float b, float thr, float x0, float x1,
                                                  float y0, float y1) {
#pragma clang fp contract(off)
    return box_form(px, py, a, b, x0, x1, y0, y1) <= thr * (1.0f + 1.0f / 1024.0f) + 1.0e-5f;
}

}  // namespace dpr

// Launchers (host side), one per stage.  All take the plan's stream.
namespace dpr {

struct Tables {                  // device pointers inside the plan workspace
    const ViewDesc *views;
    const SceneDesc *scenes;
    const uint32_t *scene_views;        // [n_views] view ids grouped by scene
    const uint32_t *scene_block_start;  // [n_scenes] first point block of each scene
    const uint32_t *sort_block_start;   // [n_views]
    const uint32_t *chunk_start;        // [n_views]
    const uint32_t *tile_start;         // [n_views]
    int32_t n_views, n_scenes;
    uint32_t max_view_tiles;            // largest tile count of any view
    uint32_t max_view_segs;             // largest column-scan segment count of any view
    uint32_t total_tiles;
};

hipError_t launch_project(const Tables &tb, const Thresholds &th, int sh_degree, uint32_t point_blocks,
                          SplatRec *rec, uint32_t *keys, uint32_t *vals, uint2 *rect,
                          hipStream_t st);

// Segmented (per view) stable LSD radix sort of 32-bit keys with 32-bit values.
// Scratch: hist[256 * sort_blocks + 1] u32, part[] u64 (scan partials).
hipError_t launch_depth_sort(const Tables &tb, uint32_t sort_blocks, uint32_t items,
                             uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                             uint32_t *hist, uint64_t *part, hipStream_t st);

// Exclusive scan of n u32 counts into out[0..n] (out[n] = total mod 2^32);
// the exact 64-bit total goes to *total64.  part: >= scan_partials(n) u64.
hipError_t launch_scan(const uint32_t *in, uint32_t *out, uint64_t n, uint64_t *part,
                       uint64_t *total64, hipStream_t st);
uint64_t scan_partials(uint64_t n);

// Binning.  cnt is chunk-major per view: cnt[cnt_off + c * tiles + t].
// Also writes bin[s], the binning record of sorted item s.
hipError_t launch_tile_count(const Tables &tb, uint32_t chunks, const uint32_t *order,
                             const uint2 *rect, const SplatRec *rec, float lambda, uint32_t *cnt, BinRec *bin,
                             hipStream_t st);
// In place: cnt[c][t] -> sum of cnt[c'][t] over c' < c; tile_total[tile] = column sum;
// tile_base = exclusive scan of tile_total (tiles + 1 entries, the last = pair
// count mod 2^32, the exact count in *total64); order = the tiles longest list
// first.  segs: scratch of sum over views of tiles * segments u32; bucket_cnt
// and block_sum: kOrderBuckets u32 and one u64 per order_count_blocks(tiles).
hipError_t launch_tile_colscan(const Tables &tb, uint32_t *cnt, uint32_t *segs, uint32_t *tile_total,
                               uint32_t *bucket_cnt, uint64_t *block_sum, uint32_t *tile_base, uint32_t *order,
                               uint64_t *total64, hipStream_t st);
// Also clears the 4 words at zero4 (the compositing counters that follow it).
// With more than pair_cap pairs in the plan (tile_base[total tiles]) it does nothing.
hipError_t launch_tile_emit(const Tables &tb, uint32_t chunks, const BinRec *bin, const uint32_t *pre,
                            const uint32_t *tile_base, uint32_t *pairs, uint32_t *zero4, uint32_t pair_cap,
                            hipStream_t st);

// Backward state of a tile list at the list positions s * kBwdSeg (s >= 1):
// per pixel (T, I) after the first s * kBwdSeg splats, 256 float4 per slot in
// row-major pixel order.  Slot of (tile t, s) = floor(tile_base[t] / kBwdSeg)
// + t + s: consecutive tiles' slot ranges never overlap, and every slot is
// below floor(pairs / kBwdSeg) + tiles + 1.
__host__ __device__ inline uint64_t ckpt_slot(uint32_t tile_base_t, uint32_t tile, uint32_t s) {
    return (uint64_t)(tile_base_t / (uint32_t)kBwdSeg) + tile + s;
}
inline uint64_t ckpt_slots(uint64_t pairs, uint64_t tiles) { return pairs / kBwdSeg + tiles + 2; }
inline uint64_t work_capacity(uint64_t pairs, uint64_t tiles) { return pairs / kBwdSeg + tiles + 1; }

struct CompositeArgs {
    const ViewDesc *views;
    const uint32_t *tile_start;
    int32_t n_views;
    uint32_t total_tiles;
    const SplatRec *rec;
    const uint32_t *pairs;
    const uint32_t *tile_base;  // [tiles + 1] first pair of each tile
    const uint32_t *tile_order; // [tiles] the order in which the forward takes the tiles, or null
    int write_views;            // 1: write image / trans / stats of each view
    uint32_t *stats;            // per-pixel blended count (or null)
    // backward state (all null for a forward that no backward will follow)
    uint32_t *nlast;            // per-pixel stop index
    float4 *fin;                // per-pixel final (T, I)
    float4 *ckpt;               // checkpoint slots (see ckpt_slot)
    uint2 *work;                // (tile, segment) backward work items
    uint32_t *counters;         // [0] persistent queue, [1] work items appended
    Thresholds th;
    // the pair capacity the forward workspace was laid out for: a launch whose
    // plan holds more pairs (tile_base[total_tiles]) does nothing
    uint32_t pair_cap = 0xFFFFFFFFu;
};
hipError_t launch_composite_fwd(const CompositeArgs &a, bool persistent, hipStream_t st);
// The forward takes the tiles longest pair list first: a tile's compositing
// time grows with the list positions it visits, and the kernel's end is set by
// the last long tile to start.  The length ranks that work only roughly (early
// termination), so the order is by bucket: the bit length of the length,
// longest first.  k_col_segscan counts each block's tiles per bucket;
// k_col_finish places them (the order of tiles within a bucket changes no
// result).
constexpr int kOrderBuckets = 33;            // bit lengths 32 .. 0
__device__ __forceinline__ uint32_t order_bucket(uint32_t len) { return len ? (uint32_t)__clz(len) : 32u; }
uint64_t order_count_blocks(uint64_t tiles);

struct BackwardArgs {
    CompositeArgs c;
    const float *const *dimage;     // device table [n_views] of dL/dimage pointers
    const float *const *dtrans;     // device table [n_views] (entries may be null) or null
    const uint32_t *nlast;
    const float4 *fin;
    const float4 *ckpt;
    const uint2 *work;
    const uint32_t *work_count;
    uint32_t *queue;
    float *grad;                    // [items][8] accumulators
};
hipError_t launch_composite_bwd(const BackwardArgs &a, hipStream_t st);

hipError_t launch_point_bwd(const Tables &tb, const Thresholds &th, int sh_degree, uint32_t point_blocks,
                            const float *grad, hipStream_t st);

// Stable LSD radix sort of n (key, value) pairs on the low `bits` bits of the
// keys, 8 bits per pass; the result is in the alt buffers when *in_alt.
// hist: radix_hist_words(n) + 1 words (the scan writes the total after the
// last one); part: scan_partials(hist words) + 1 words.
uint64_t radix_hist_words(uint64_t n);
hipError_t launch_radix_sort(uint32_t n, int bits, uint32_t *keys, uint32_t *vals, uint32_t *keys_alt,
                             uint32_t *vals_alt, uint32_t *hist, uint64_t *part, bool *in_alt, hipStream_t st);

// Hybrid coarse-to-fine update (hybrid.hip).
constexpr int kKnnMax = 32;               // largest K
constexpr uint32_t kKnnMaxGrid = 128;     // neighbour grid cells per axis, at most
constexpr uint32_t kHyBoxBlocks = 256;    // blocks of the bounding-box reduction
struct HyScratch {
    uint32_t *keys, *vals, *keys_alt, *vals_alt;   // [n] each
    uint32_t *hist;                               // radix_hist_words(n) + 1
    uint64_t *part;                               // scan_partials(max(n + 1, hist words)) + 1
    uint64_t *total64;
    uint32_t *flags, *seg, *starts;               // [n + 2] each
    uint32_t *cell_start;                         // [cells of the neighbour grid + 1]
    float *box_part, *box;                        // [6 kHyBoxBlocks], [6]
    int32_t *idx;                                 // [n K]
    float *d2;                                    // [n K]
};
uint32_t knn_grid_size(uint64_t m);
// Bytes of each HyScratch array for up to n points and K neighbours.
struct HyScratchBytes {
    uint64_t keys, vals, keys_alt, vals_alt, hist, part, total64, flags, seg, starts, cell_start, box_part, box, idx,
        d2;
};
HyScratchBytes hy_scratch_bytes(uint64_t n, int K);
hipError_t launch_knn(const float *xyz, uint32_t m, int K, int32_t *idx, float *d2, HyScratch &s, hipStream_t st);
hipError_t launch_voxel_reduce(const float *xyz, const float *sh, const float *op, const float *rad, uint32_t n,
                               int k3, uint32_t N, float *oxyz, float *osh, float *oop, float *orad, HyScratch &s,
                               uint64_t *m_host, hipStream_t st);
hipError_t launch_filter_generate(const float *xyz, const float *sh, const float *op, const float *rad, uint32_t m,
                                  int k3, int K, float eps, float *oxyz, float *osh, float *oop, float *orad,
                                  HyScratch &s, uint64_t *kept_host, uint64_t *count_host, hipStream_t st);

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t st);

// Visual hull / consistency check (hull.hip).
constexpr int32_t kHullMaxCams = 4096;
struct HullCam {                 // 96 bytes, one per camera, in the workspace
    float R[9], t[3], fx, fy, cx, cy;
    int32_t width, height;
    const uint8_t *mask;         // device, width x height, foreground where non-zero
    const uint32_t *bits;        // the mask packed one bit per pixel (row-major), in the workspace
    uint64_t word_off;           // first packed word of this camera
};
struct HullLayout {
    uint64_t cams, packed, bits, counts, offsets, part, total, bytes;
    uint64_t words;              // packed mask words over all cameras
};
struct HullJob {
    int32_t n_cams;
    const HullCam *cams;         // host table (uploaded into the workspace)
    uint64_t n;                  // candidates (sampling) or points (filter)
    const float *xyz;            // filter: points; sampling: null
    uint64_t seed;
    float lo[3], hi[3];
    uint8_t *keep;               // optional: CC per item
    float *out_xyz;              // optional: kept items (first `capacity`)
    uint64_t capacity;
    const float *sh, *opacity, *radius;       // filter: the other parameters
    float *out_sh, *out_opacity, *out_radius;
    int k3;
    bool sync;                   // wait for the kept count
};
uint64_t hull_blocks(uint64_t n);
// cams: host table (width, height used)
HullLayout hull_layout(uint64_t n, int32_t n_cams, const HullCam *cams);
hipError_t launch_hull(const HullJob &job, uint8_t *ws, uint64_t *kept_host, hipStream_t st);

// Video warm start: Chamfer distance, top-k SH transfer, Adam (chamfer.hip).
constexpr int kTopkMax = 32;
struct ChamferLayout {
    uint64_t key12, key21, acc, cnt, part1, part2, bytes;
};
ChamferLayout chamfer_layout(uint64_t n1, uint64_t n2);
hipError_t launch_chamfer(uint32_t n1, const float *s1, uint32_t n2, const float *s2, double *cd, float *grad2,
                          int32_t *nn12, int32_t *nn21, uint8_t *ws, hipStream_t st);
hipError_t launch_topk_sh(uint32_t n1, const float *s1, const float *sh1, uint32_t n2, const float *s2, int k3, int K,
                          float *out_sh, int32_t *idx, hipStream_t st);
hipError_t launch_adam(uint32_t n, float *p, const float *g, float *m, float *v, int t, float lr, float b1, float b2,
                       float eps, hipStream_t st);

// Eq. (8) loss over a batch of images (loss.hip).
struct LossImage {
    const float *render, *target;
    float *grad;
    int32_t width, height;
};
constexpr int kLossBatch = 16;     // images per launch (passed in the kernel arguments)
uint32_t loss_blocks(int32_t width, int32_t height);
// partial: per-block sums, as many as the largest batch of kLossBatch images needs
hipError_t launch_loss(const LossImage *img, int n, float lambda, float *partial, double *loss, hipStream_t st);
// Stream-ordered copy of a small host table (bytes % 4 == 0) through kernel arguments.
hipError_t upload_async(void *dst, const void *src, size_t bytes, hipStream_t st);
// One launch: a table of bytes % 4 == 0 copied as upload_async does, and the
// word ranges z0[0..n0), z1[0..n1) cleared (null ranges allowed).  Tables
// above kUploadZeroWords words take separate launches.
hipError_t upload_zero_async(void *dst, const void *src, size_t bytes, uint32_t *z0, uint64_t n0, uint32_t *z1,
                             uint64_t n1, hipStream_t st);
// Reads one 64-bit count that work queued on `st` produces: copies it into a
// pinned host word of the calling thread (allocated on the thread's first
// call and kept until the process ends), waits for the stream, stores it in *out.
hipError_t read_count(const uint64_t *dev, uint64_t *out, hipStream_t st);
// The same in two halves: the copy into the thread's pinned word and an event
// behind it, queued on `st`; then the wait for that event and the value.
hipError_t read_count_begin(const uint64_t *dev, hipStream_t st);
hipError_t read_count_end(uint64_t *out);

// Sets the thread's dpr_last_error message and returns `code`.
int set_last_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

}  // namespace dpr
