/*
 * dpr.h - C ABI of the MI355X differentiable point-splat renderer (libdpr.so).
 *
 * The renderer implements the differentiable splat rendering of
 * Zhang et al., "Differentiable Point-Based Radiance Fields for Efficient View
 * Synthesis" (SIGGRAPH Asia 2022):
 *   - projection of points P_i through a pinhole camera (R, t, M), Sec. 3.1 Eq. (1);
 *   - per-view colour from spherical harmonics of the view direction,
 *     Sec. 3.1 Eq. (2)-(4);
 *   - a Gaussian splat per point with front-to-back alpha blending over the
 *     points sorted by camera depth, Sec. 3.2 Eq. (5)-(7), restricted to
 *     points with non-negligible opacity near each pixel (end of Sec. 3.2);
 *   - gradients of a loss on the image with respect to positions, SH
 *     coefficients and opacities ("fully differentiable ... end-to-end",
 *     Sec. 3.3).
 *
 * Conventions (fixed by this library where the paper leaves them open):
 *   - x_cam = R * P + t with R row-major; pixel = (fx*x/z + cx, fy*y/z + cy);
 *     +x right, +y down, +z forward; pixel (x, y) is sampled at (x+0.5, y+0.5).
 *   - The splat of point i in a view has sigma_x = fx*r_i/Z, sigma_y = fy*r_i/Z
 *     (r_i = world radius, Z = camera depth) and
 *        alpha_i(u) = min(alpha_max, o_i * exp(-((px-ux)^2/sx^2 + (py-uy)^2/sy^2)/2));
 *     the 1/sqrt(2 pi r^2) factor of Eq. (5) is replaced by the per-point opacity o_i.
 *   - Point i is a candidate at pixel u iff o_i*G_i(u) >= alpha_min; compositing
 *     stops after the first blended splat that leaves T < t_min.
 *   - Depth order: ascending float32 key Z32 = fmaf(R20,x, fmaf(R21,y, fmaf(R22,z,t2))),
 *     ties by ascending point index; points with Z32 <= z_near are dropped.
 *   - Colour: real orthonormal SH, no Condon-Shortley phase, coefficient index
 *     k = l^2 + l + m, evaluated at v = x_cam/|x_cam| (sh_frame 0) or R^T v
 *     (sh_frame 1).  No activation or clamp; background 0 (the caller adds
 *     T * background).
 *
 * Memory: every pointer in the descriptors is DEVICE memory owned by the caller.
 * The library never allocates device memory: the caller provides three
 * workspaces whose sizes the library reports (plan, forward, backward).
 * All float arrays are float32, densely packed, 4-byte aligned; 16-byte
 * alignment of xyz/sh/images is recommended.
 *
 * Streams: a stream argument is a hipStream_t passed as void* (NULL = the
 * default stream).  Everything is asynchronous on that stream except
 * dpr_plan_forward and dpr_plan_forward_render, which wait once for the
 * number of (tile, splat) pairs.
 *
 * Errors: functions returning int return a dpr_status; a non-zero status
 * leaves a message in dpr_last_error() (thread-local).  The library never
 * aborts and never throws across this boundary.  Input VALUES (NaN/Inf) are
 * not validated; they propagate.
 *
 * Thread safety: a plan is used by one thread at a time; different plans are
 * independent.
 */
#ifndef DPR_H
#define DPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPR_ABI_VERSION 2

typedef enum dpr_status {
    DPR_OK = 0,
    DPR_ERR_INVALID_ARG = 1,  /* null required pointer, bad size/degree/threshold, bad scene index */
    DPR_ERR_WORKSPACE = 2,    /* a workspace is NULL or smaller than the reported size          */
    DPR_ERR_HIP = 3,          /* a HIP launch or runtime call failed; see dpr_last_error()       */
    DPR_ERR_UNSUPPORTED = 4,  /* sizes beyond the library's limits (e.g. >= 2^32 pairs)          */
    DPR_ERR_STATE = 5         /* calls out of order (e.g. backward before forward)               */
} dpr_status;

/* Pinhole camera of one view (Sec. 3.1 Eq. 1): M = [[fx,0,cx],[0,fy,cy],[0,0,1]]. */
typedef struct dpr_camera {
    float R[9];          /* world -> camera rotation, row-major                 */
    float t[3];          /* world -> camera translation                         */
    float fx, fy;        /* focal lengths in pixels, > 0                        */
    float cx, cy;        /* principal point in pixels                           */
    int32_t width;       /* image width in pixels, 1 .. 16384                   */
    int32_t height;      /* image height in pixels, 1 .. 16384                  */
} dpr_camera;

/* One point cloud (Sec. 3.1): positions P_i, SH coefficients H_i, opacity, radius. */
typedef struct dpr_scene {
    int64_t n;               /* number of points, 0 .. 2^31-1 (sum over views < 2^31) */
    int32_t sh_degree;       /* l_max, 0 .. 3; K = (l_max+1)^2 coefficients          */
    int32_t reserved;        /* must be 0                                            */
    const float *xyz;        /* [n][3]                                               */
    const float *sh;         /* [n][K][3]  (coefficient-major, RGB innermost)        */
    const float *opacity;    /* [n], o_i in (0, 1]                                   */
    const float *radius;     /* [n], world-space splat radius r_i > 0                */
} dpr_scene;

/* One rendered view of one scene. */
typedef struct dpr_view {
    int32_t scene;           /* index into the scene array                           */
    int32_t reserved;        /* must be 0                                            */
    dpr_camera cam;
    float *image;            /* [height][width][3] output (pre-background colour)    */
    float *trans;            /* [height][width] output: final transmittance T, or
                                NULL (then T is not written).                        */
} dpr_view;

enum { DPR_SH_FRAME_CAMERA = 0, DPR_SH_FRAME_WORLD = 1 };
enum { DPR_BWD_STORED = 0, DPR_BWD_RECOMPUTE = 1 };
enum {
    DPR_FLAG_TIMING = 1,      /* record HIP events around every stage (dpr_stage_times)    */
    DPR_FLAG_STATS = 2,       /* count blended splats per pixel (dpr_plan_info.stats_off)  */
    DPR_FLAG_PERSISTENT = 4,  /* forward compositing pops tiles from a work queue (the
                                 backward always pops (tile, segment) work items)           */
    DPR_FLAG_KERNEL_NORM = 8  /* keep Eq. (5)'s normalisation: alpha = min(alpha_max,
                                 o (2 pi sx sy)^-1/2 G), i.e. 1/sqrt(2 pi r^2) per the
                                 printed formula with r the screen sigma (per axis)         */
};

typedef struct dpr_params {
    float alpha_min;         /* candidate threshold on o*G, [0, 1); default 1e-5 (> 0 required) */
    float t_min;             /* early-stop transmittance, [0, 1); default 1e-5                  */
    float alpha_max;         /* alpha clamp, (0, 0.999]; default 0.99                           */
    float z_near;            /* near plane, > 0; default 0.01                                   */
    int32_t sh_frame;        /* DPR_SH_FRAME_*                                                  */
    int32_t bwd_mode;        /* DPR_BWD_*: the forward keeps the backward state in its
                                workspace (stored), or the backward composites again to
                                rebuild it (recompute: smaller forward workspace)             */
    int32_t flags;           /* DPR_FLAG_* bitmask                                              */
    int32_t max_splats;      /* > 0: a pixel blends at most this many splats, its first ones
                                in depth order (Sec. 3.3 uses n = 15); 0: no cap              */
    int32_t timing_stages;   /* with DPR_FLAG_TIMING: the stages to time, bit s = DPR_STAGE s;
                                0: every stage.  Each timed stage records two HIP events on
                                the stream, so timing only the stage of interest keeps the
                                others' launches back to back                                   */
} dpr_params;

typedef struct dpr_plan dpr_plan;   /* opaque, host-side */

/* Stage indices for dpr_stage_times. */
enum {
    DPR_STAGE_UPLOAD = 0, DPR_STAGE_PROJECT, DPR_STAGE_DEPTH_SORT, DPR_STAGE_TILE_COUNT,
    DPR_STAGE_TILE_SCAN, DPR_STAGE_EMIT, DPR_STAGE_COMPOSITE_FWD, DPR_STAGE_RECOMPUTE,
    DPR_STAGE_COMPOSITE_BWD, DPR_STAGE_POINT_BWD, DPR_STAGE_COUNT
};

/* Sizes and workspace offsets of a plan, for diagnostics and stage-level tests. */
typedef struct dpr_plan_info {
    int64_t items;           /* sum over views of the scene's point count (view-points) */
    int64_t pairs;           /* (tile, splat) pairs; valid after dpr_plan_forward       */
    int64_t tiles;           /* 16x16 screen tiles over all views                        */
    int64_t pixels;          /* pixels over all views                                    */
    int64_t chunks;          /* binning chunks over all views                            */
    int64_t plan_ws_bytes, fwd_ws_bytes, bwd_ws_bytes;
    /* byte offsets inside the plan workspace */
    int64_t rec_off;         /* [items] x 8 float: px, py, a, b, w, r, g, b   (see below) */
    int64_t key_off;         /* [items] u32 depth keys in sorted order: the key of item
                                order[j] (float bits of Z; 0xFFFFFFFF = dropped)          */
    int64_t order_off;       /* [items] u32 item ids, depth-sorted within each view      */
    int64_t rect_off;        /* [items] 2 x u32 tile rectangle (x0|y0<<16, x1|y1<<16)    */
    int64_t range_off;       /* [tiles + 1] u32: tile t's list is pairs[range[t] .. range[t+1]) */
    /* byte offsets inside the forward workspace */
    int64_t pairs_off;       /* [pairs] u32 item ids, grouped by tile, depth order within */
    int64_t nlast_off;       /* [pixels] u32 blend end (stored mode), -1 if absent: one
                                past the list position of the pixel's last blended splat,
                                0 if it blended none                                      */
    int64_t stats_off;       /* [pixels] u32 blended splats per pixel, -1 if absent       */
    int32_t tile_size;       /* 16                                                        */
    int32_t chunk_items;     /* items per binning chunk                                   */
} dpr_plan_info;
/* Record layout: a = log2(e)/(2 sx^2), b = log2(e)/(2 sy^2), w = log2(o), so that
 * alpha = min(alpha_max, 2^(w - a dx^2 - b dy^2)) with dx = px - ux, dy = py - uy.
 * Item id of point i in view v = sum of the point counts of the views before v + i. */

/* Version of this ABI (DPR_ABI_VERSION). */
int dpr_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char *dpr_last_error(void);

/* Bytes of the plan workspace for this set of scenes and views (0 on invalid
 * arguments; the reason is in dpr_last_error). */
size_t dpr_plan_ws_bytes(const dpr_scene *scenes, int32_t n_scenes,
                         const dpr_view *views, int32_t n_views);

/* Validates the arguments, creates a plan and runs projection + SH colour
 * (Eq. 1-4), the per-view depth sort (Sec. 3.2) and the tile counting of the
 * binning stage into plan_ws; waits once on `stream` for the pair count.
 * The descriptors are copied; the arrays they point to must stay valid and
 * unchanged until the last call that uses the plan.  plan_ws must stay alive
 * and untouched until the plan is freed.  On success *out owns the plan
 * (release with dpr_plan_free). */
int dpr_plan_forward(const dpr_scene *scenes, int32_t n_scenes,
                     const dpr_view *views, int32_t n_views, const dpr_params *params,
                     void *plan_ws, size_t plan_ws_bytes, void *stream, dpr_plan **out);

/* Bytes of the forward workspace, known after dpr_plan_forward: the per-tile
 * pair lists and, in stored mode, the state the backward reads (per pixel the
 * blend end and final (T, I); per tile a (T, I) checkpoint of every pixel each
 * 256 list positions; the backward's work items), up to 16 B per pair + 20 B
 * per pixel on top of the 4 B per pair of the lists. */
size_t dpr_workspace_bytes(const dpr_plan *plan);

/* Emits the per-tile depth-ordered splat lists and composites every view front
 * to back (Eq. 5-7), writing image and trans of each view.  `ws` must stay
 * alive and untouched until the last dpr_render_backward of this plan. */
int dpr_render_forward(dpr_plan *plan, void *ws, size_t ws_bytes, void *stream);

/* dpr_plan_forward and dpr_render_forward in one call, for a caller that keeps
 * a forward workspace from plan to plan (the rendering of Sec. 3.2, Eq. 5-7,
 * of the plan stage's splats).  The forward is queued right behind the plan
 * stage, before the wait for the pair count, laid out for as many pairs as
 * fwd_ws_bytes can hold; its kernels read the pair count on the device and do
 * nothing if the lists do not fit.  So the device goes on from the plan to the
 * forward without the host's round trip.
 *   *rendered = 1: the forward ran into fwd_ws, exactly as dpr_render_forward
 *                  would have; fwd_ws is this plan's forward workspace (for
 *                  dpr_render_backward) and dpr_plan_get_info reports its layout.
 *   *rendered = 0: fwd_ws was too small (dpr_workspace_bytes tells the size);
 *                  nothing was written to it or to the images.  The plan is
 *                  valid: call dpr_render_forward with a large enough buffer.
 * Arguments, ownership and errors otherwise as dpr_plan_forward; fwd_ws and
 * rendered must not be NULL (DPR_ERR_INVALID_ARG). */
int dpr_plan_forward_render(const dpr_scene *scenes, int32_t n_scenes,
                            const dpr_view *views, int32_t n_views, const dpr_params *params,
                            void *plan_ws, size_t plan_ws_bytes, void *fwd_ws, size_t fwd_ws_bytes,
                            void *stream, dpr_plan **out, int32_t *rendered);

/* Bytes of the backward scratch workspace (per-view-point gradient records,
 * plus, in recompute mode, the backward state that stored mode keeps in the
 * forward workspace).  Needed only during the call. */
size_t dpr_backward_ws_bytes(const dpr_plan *plan);

/* Reverse-mode gradients of a loss L through the forward of this plan.
 *   dL_dimage[v]  [H][W][3] gradient w.r.t. view v's image (required)
 *   dL_dtrans     NULL, or per view NULL / [H][W] gradient w.r.t. trans
 *   dL_dxyz[s]    [n][3]     } per scene, OVERWRITTEN with the sum over every
 *   dL_dsh[s]     [n][K][3]  } view of the scene; a NULL array pointer (or a NULL
 *   dL_dopacity[s][n]        } table) skips that output.
 * Candidate sets, depth order and the splats each pixel blends are held fixed (piecewise-constant
 * structure); clamped alphas pass no gradient to o or the position.  The
 * forward state is not modified, so backward may be called more than once.
 * `ws` must be the very buffer given to this plan's dpr_render_forward (it holds
 * the tile lists and, in stored mode, the backward state); any other pointer
 * returns DPR_ERR_STATE before device work, as does a call before the forward. */
int dpr_render_backward(dpr_plan *plan, const void *ws, size_t ws_bytes,
                        const float *const *dL_dimage, const float *const *dL_dtrans,
                        float *const *dL_dxyz, float *const *dL_dsh, float *const *dL_dopacity,
                        void *bwd_ws, size_t bwd_ws_bytes, void *stream);

/* Bytes of the device workspace dpr_loss_l2_tv needs for n_images images of
 * the given sizes (host arrays); 0 on invalid sizes (see dpr_last_error). */
size_t dpr_loss_ws_bytes(int32_t n_images, const int32_t *widths, const int32_t *heights);

/* The training loss of Eq. (8) (Sec. 3.3) and its gradient, for n_images
 * images in one pass:
 *   loss[v] = sum_{x,y,c} (R - I)^2
 *             + lambda (sum |R(x+1,y,c) - R(x,y,c)| + sum |R(x,y+1,c) - R(x,y,c)|)
 * i.e. squared L2 plus lambda times the anisotropic total variation (forward
 * differences between adjacent pixels, summed over channels; the paper uses
 * lambda = 0.01), and dL/dR with the subgradient of |d| at d = 0 taken as 0.
 *   render[v], target[v]  device [H][W][3] float32 (host array of pointers)
 *   dL_drender[v]         device [H][W][3] float32, OVERWRITTEN; may not alias
 *                         render[v] or target[v]
 *   widths, heights       host arrays
 *   loss                  device double[n_images], OVERWRITTEN; each image's sum
 *                         is reduced in a fixed order (deterministic)
 *   ws                    device workspace of dpr_loss_ws_bytes bytes, needed
 *                         until the work on `stream` has run
 * Asynchronous on `stream`.  Returns DPR_ERR_INVALID_ARG on NULL pointers,
 * aliasing outputs, sizes outside [1, 16384] or lambda < 0 / non-finite. */
int dpr_loss_l2_tv(int32_t n_images, const float *const *render, const float *const *target,
                   const int32_t *widths, const int32_t *heights, float lambda, float *const *dL_drender,
                   double *loss, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Hybrid coarse-to-fine update of the point cloud (Sec. 3.3, Alg. 1).
 * A point's parameters are its position, its SH coefficients [K][3]
 * (K = (sh_degree + 1)^2), its opacity and its radius; "average" means the
 * average of all of them.  All arrays are device float32, row-major.
 * Decisions read from float comparisons are taken in float32 with every
 * operation rounded on its own, so they are reproducible bit for bit:
 *   voxel/grid cell per axis: s = M / (hi - lo) over the points' bounding box
 *     (0 if hi == lo), cell = clamp(floor((p - lo) * s), 0, M - 1);
 *     key (iz M + iy) M + ix;
 *   neighbour order: the other points by d2 = (dx dx + dy dy) + dz dz with
 *     dx = x_j - x_i, ties by index;
 *   spread of a point's k = min(K, m - 1) neighbour distances d_q = sqrt(d2_q):
 *     mean = (sum d_q) / k, delta = sqrt(sum (d_q - mean)^2 / k) (sums in
 *     neighbour order); the point is removed if delta > eps (kept if k = 0).
 * Averages are accumulated in FP64 in a fixed order (ascending point index
 * within a voxel; neighbour order for a generated point).
 * ------------------------------------------------------------------------- */

/* Bytes of the device workspace of dpr_knn for m points (0 on bad sizes). */
size_t dpr_knn_ws_bytes(int64_t m, int32_t K);

/* The K nearest other points of every point (exact, K <= 32), by a uniform
 * grid search.  idx[m][K]: neighbour indices in neighbour order, -1 past
 * min(K, m - 1); d2[m][K]: their float32 squared distances (0 past the end).
 * Asynchronous on `stream`. */
int dpr_knn(int64_t m, const float *xyz, int32_t K, int32_t *idx, float *d2, void *ws, size_t ws_bytes,
            void *stream);

/* Bytes of the device workspace of dpr_hybrid_update (and, with K = 1, of
 * dpr_voxel_reduce) for n input points (0 on bad sizes). */
size_t dpr_hybrid_ws_bytes(int64_t n, int32_t sh_degree, int32_t K);

/* Step 1 of Alg. 1: the bounding box of the n points split into N^3 voxels
 * (1 <= N <= 1024), every non-empty voxel replaced by the average of its
 * points, written in ascending voxel key order to out_* (capacity n points);
 * *out_count (host) = number of voxels.  Synchronizes `stream` once (to learn
 * the count). */
int dpr_voxel_reduce(int64_t n, int32_t sh_degree, const float *xyz, const float *sh, const float *opacity,
                     const float *radius, int32_t N, float *out_xyz, float *out_sh, float *out_opacity,
                     float *out_radius, int64_t *out_count, void *ws, size_t ws_bytes, void *stream);

/* Alg. 1: voxel reduction (N), then on the reduced points outlier removal
 * (K nearest neighbours, threshold eps >= 0) and point generation (one new
 * point per kept point, the average of its K nearest kept neighbours, if it
 * has any).  Removal and generation are each decided against the set before
 * that step.  out_* (capacity 2 n points) receive the kept points, in voxel
 * order, followed by the generated ones in the same order.  out_counts (host
 * int64[3]) = {voxels, kept, output points}.  Synchronizes `stream` twice.
 * Inputs and outputs must not overlap. */
int dpr_hybrid_update(int64_t n, int32_t sh_degree, const float *xyz, const float *sh, const float *opacity,
                      const float *radius, int32_t N, int32_t K, float eps, float *out_xyz, float *out_sh,
                      float *out_opacity, float *out_radius, int64_t *out_counts, void *ws, size_t ws_bytes,
                      void *stream);

/* ---------------------------------------------------------------------------
 * Visual-hull initialisation and multi-view consistency filter (Sec. 3.1
 * "Initialization" and the appendix's consistency check CC: a point is kept
 * when it projects onto a foreground pixel of every camera's mask).
 * The pixel decision is taken in float32, each operation rounded once:
 *   X_c = fma(R_c0, x, fma(R_c1, y, fma(R_c2, z, t_c)))   (c = 0, 1, 2)
 *   px = fma(fx, X_0 / X_2, cx),  py = fma(fy, X_1 / X_2, cy)
 * P is inside mask i iff X_2 > 0, 0 <= px < width, 0 <= py < height and the
 * mask byte at (floor(py), floor(px)) is non-zero.
 * Sampling draws candidate j (j = 0 .. n-1) from Philox4x32-10 (Salmon et al.,
 * SC 2011) with counter (j mod 2^32, j div 2^32, 0, 0) and key (seed mod 2^32,
 * seed div 2^32): with its first three output words r, coordinate d is
 * fma((r_d >> 8) * 2^-24, hi_d - lo_d, lo_d) (hi_d - lo_d rounded once).
 * At most 4096 cameras per call; each mask must have its camera's image size.
 * ------------------------------------------------------------------------- */

/* Foreground mask of one camera: device bytes, row-major, width x height;
 * foreground where non-zero.  The caller owns it. */
typedef struct dpr_mask {
    const uint8_t *data;
    int32_t width, height;
} dpr_mask;

/* Bytes of the device workspace for n candidates or points and the n_cams
 * cameras cams (their image sizes; 0 on bad sizes).  The workspace holds the
 * masks packed to one bit per pixel. */
size_t dpr_hull_ws_bytes(int64_t n, int32_t n_cams, const dpr_camera *cams);

/* Rejection sampling of n candidates (0 <= n < 2^31) in the box [lo, hi] (host
 * float[3] each, lo < hi): the consistent ones, in candidate order, are written
 * to out_xyz (device float[capacity][3]; the first `capacity` of them);
 * *out_count (host) = the number of consistent candidates, which may exceed
 * capacity.  Synchronizes `stream` once. */
int dpr_hull_sample(int32_t n_cams, const dpr_camera *cams, const dpr_mask *masks, const float *lo, const float *hi,
                    uint64_t seed, int64_t n, float *out_xyz, int64_t capacity, int64_t *out_count, void *ws,
                    size_t ws_bytes, void *stream);

/* keep[j] = CC(P_j) (1 or 0) for n points (device float[n][3] -> device
 * uint8[n]).  Asynchronous on `stream`. */
int dpr_consistency(int64_t n, const float *xyz, int32_t n_cams, const dpr_camera *cams, const dpr_mask *masks,
                    uint8_t *keep, void *ws, size_t ws_bytes, void *stream);

/* The consistent points of a cloud (every parameter, input order) into out_*
 * (capacity n points; must not overlap the inputs); *out_count (host) = their
 * number.  Synchronizes `stream` once. */
int dpr_consistency_filter(int64_t n, int32_t sh_degree, const float *xyz, const float *sh, const float *opacity,
                           const float *radius, int32_t n_cams, const dpr_camera *cams, const dpr_mask *masks,
                           float *out_xyz, float *out_sh, float *out_opacity, float *out_radius, int64_t *out_count,
                           void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Video warm start (Sec. 3.4 "Video Synthesis"): the Chamfer distance of
 * Eq. (9) between the learned cloud S1 of one frame and the initial cloud S2
 * of the next, its gradient with respect to the positions of S2, an Adam step
 * on those positions, and the transfer to every S2 point of the mean SH
 * coefficients of its k nearest S1 points.
 * Squared distances in float32, each operation rounded once:
 * d2(x, y) = ((x0 - y0)^2 + (x1 - y1)^2) + (x2 - y2)^2; a nearest neighbour is
 * the point of smallest d2, ties to the lower index.  Brute force: the work
 * grows as n1 * n2 (meant for clouds of one frame, up to about 10^6 points).
 * ------------------------------------------------------------------------- */

/* Bytes of the device workspace of dpr_chamfer (0 on bad sizes). */
size_t dpr_chamfer_ws_bytes(int64_t n1, int64_t n2);

/* For clouds s1[n1][3], s2[n2][3] (device float32, 1 <= n < 2^31):
 *   *cd = (1/n1) sum_x d2(x, nn(x)) + (1/n2) sum_y d2(y, nn(y))   (Eq. 9; device
 *         double, FP64 sums; NULL to skip),
 *   grad2[j] = dCD/dy_j = (2/n2)(y_j - nn(y_j)) + (2/n1) sum_{x: nn(x) = y_j}
 *         (y_j - x)   (device float[n2][3], FP64 then rounded; NULL to skip),
 *   nn12[i], nn21[j]: nearest indices (device int32; NULL to skip).
 * Asynchronous on `stream`. */
int dpr_chamfer(int64_t n1, const float *s1, int64_t n2, const float *s2, double *cd, float *grad2, int32_t *nn12,
                int32_t *nn21, void *ws, size_t ws_bytes, void *stream);

/* out_sh2[j] = mean of sh1 over the k = min(K, n1) points of s1 with the
 * smallest (d2(y_j, x), index), FP64 sums in that order (1 <= K <= 32;
 * sh1/out_sh2: device float[n][(sh_degree + 1)^2][3]); idx[j][K] (device
 * int32, -1 past k; NULL to skip).  Asynchronous on `stream`. */
int dpr_topk_sh(int64_t n1, const float *s1, const float *sh1, int64_t n2, const float *s2, int32_t sh_degree,
                int32_t K, float *out_sh2, int32_t *idx, void *stream);

/* One Adam step (Kingma and Ba, ICLR 2015) on n values in float32, in place
 * on p, m, v (device), step t >= 1 with bias correction:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).  Asynchronous. */
int dpr_adam_step(int64_t n, float *p, const float *g, float *m, float *v, int32_t t, float lr, float beta1,
                  float beta2, float eps, void *stream);

/* Releases a plan (host memory and HIP events only).  NULL is ignored. */
void dpr_plan_free(dpr_plan *plan);

/* Fills *out with the plan's sizes and workspace offsets. */
int dpr_plan_get_info(const dpr_plan *plan, dpr_plan_info *out);

/* With DPR_FLAG_TIMING: milliseconds of each stage of the most recent call
 * that ran it, measured with HIP events on the plan's stream (-1 where the
 * stage did not run or is not in timing_stages).  Synchronizes on those events.  cap >= DPR_STAGE_COUNT. */
int dpr_stage_times(const dpr_plan *plan, float *ms, int32_t cap);

/* Convenience form of the single-scene, single-camera renderer:
 * render_forward(points, sh, opacity, radius, camera) -> image, transmittance.
 * Runs plan + forward in one workspace.  If ws_bytes is too small it returns
 * DPR_ERR_WORKSPACE and writes the required size to *ws_needed (which may take
 * running the plan stage, i.e. one wait on the stream).  ws may be NULL to query. */
int dpr_render_forward_1(const dpr_scene *scene, const dpr_camera *cam, const dpr_params *params,
                         float *image, float *trans, void *ws, size_t ws_bytes,
                         size_t *ws_needed, void *stream);

/* Bytes of the static device scratch of dpr_render_forward_1_noalloc (64 MiB). */
#define DPR_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): dpr_render_forward_1 with
 * its workspace in a static device array of DPR_NOALLOC_SCRATCH_BYTES instead
 * of a caller buffer.  It calls no hipMalloc/hipFree and creates no events.
 *   - Same arguments, results and kernels as dpr_render_forward_1 with
 *     ws/ws_bytes/ws_needed dropped; the caller still owns scene, image, trans.
 *   - bwd_mode is ignored (no backward state is kept: the plan ends with the
 *     call); DPR_FLAG_TIMING is refused with DPR_ERR_INVALID_ARG.
 *   - An input whose plan + forward workspace exceeds the scratch returns
 *     DPR_ERR_WORKSPACE with the size it needs (the plan stage may have run).
 *     About 300k points at 800x800 fit.
 *   - The scratch is per device: the first call on a device, with that device
 *     current, takes its address once; the device holds the array until the
 *     process ends.  The current device must own `stream` and the pointers.
 *   - Every call on one device uses the same array and nothing in it needs to
 *     start zeroed (the call clears its own counters).  Calls that overlap on
 *     one device (other threads or other streams) race on it: serialize them.
 *   - Like dpr_render_forward_1 it waits once on `stream` (for the pair count). */
int dpr_render_forward_1_noalloc(const dpr_scene *scene, const dpr_camera *cam, const dpr_params *params,
                                 float *image, float *trans, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DPR_H */
