// Host implementation of the C ABI declared in include/dpr.h: argument
// validation, workspace layout, stage sequencing on the caller's stream,
// error reporting and per-stage HIP-event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "dpr_internal.h"

using namespace dpr;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                             \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(DPR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

constexpr uint64_t kAlign = 256;
uint64_t align_up(uint64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Byte layout of a workspace: a list of (offset, size) regions.
struct Region {
    uint64_t off = 0, bytes = 0;
};
struct Layout {
    uint64_t total = 0;
    Region add(uint64_t bytes) {
        Region r;
        r.off = total;
        r.bytes = bytes;
        total = align_up(total + bytes);
        return r;
    }
};

struct Sizes {
    int32_t n_views = 0, n_scenes = 0;
    uint64_t items = 0, tiles = 0, pixels = 0, chunks = 0, cnt = 0, sort_blocks = 0, point_blocks = 0;
    uint64_t max_view_tiles = 0, max_view_segs = 0, segs = 0;
    int32_t sh_degree = 0;
};

struct PlanLayout {
    Region views, scenes, u32tab, rec, keys, vals, keys_alt, vals_alt, rect, bin, hist, part, cnt, segs, tile_total,
        tile_base, tile_order, bucket_cnt, block_sum;
    uint64_t total = 0;
};

PlanLayout plan_layout(const Sizes &s) {
    Layout L;
    PlanLayout p;
    p.views = L.add(sizeof(ViewDesc) * (uint64_t)s.n_views);
    p.scenes = L.add(sizeof(SceneDesc) * (uint64_t)s.n_scenes);
    // scene_views[V], scene_block_start[S], sort_block_start[V], chunk_start[V], tile_start[V]
    p.u32tab = L.add(sizeof(uint32_t) * (4ull * s.n_views + s.n_scenes));
    p.rec = L.add(sizeof(SplatRec) * s.items);
    p.keys = L.add(4 * s.items);
    p.vals = L.add(4 * s.items);
    p.keys_alt = L.add(4 * s.items);
    p.vals_alt = L.add(4 * s.items);
    p.rect = L.add(8 * s.items);
    p.bin = L.add(sizeof(BinRec) * s.items);
    const uint64_t nh = 256ull * s.sort_blocks;
    p.hist = L.add(4 * (nh + 1));
    const uint64_t np = std::max(scan_partials(nh), scan_partials(s.tiles)) + 2;
    p.part = L.add(8 * np);
    p.cnt = L.add(4 * s.cnt);
    p.segs = L.add(4 * s.segs);
    p.tile_total = L.add(4 * s.tiles);
    p.tile_base = L.add(4 * (s.tiles + 1));
    p.tile_order = L.add(4 * s.tiles);
    p.bucket_cnt = L.add(4ull * kOrderBuckets * order_count_blocks(s.tiles));
    p.block_sum = L.add(8ull * order_count_blocks(s.tiles));
    p.total = L.total;
    return p;
}

const int kLimitDim = 16384;

int check_params(const dpr_params *pr) {
    if (!pr) return fail(DPR_ERR_INVALID_ARG, "params is NULL");
    if (!(pr->alpha_min >= 0.f && pr->alpha_min < 1.f))
        return fail(DPR_ERR_INVALID_ARG, "alpha_min must be in [0, 1)");
    if (!(pr->t_min >= 0.f && pr->t_min < 1.f)) return fail(DPR_ERR_INVALID_ARG, "t_min must be in [0, 1)");
    if (!(pr->alpha_max > 0.f && pr->alpha_max <= 1.f))
        return fail(DPR_ERR_INVALID_ARG, "alpha_max must be in (0, 1]");
    if (!(pr->z_near > 0.f) || !std::isfinite(pr->z_near)) return fail(DPR_ERR_INVALID_ARG, "z_near must be > 0");
    if (pr->sh_frame != 0 && pr->sh_frame != 1) return fail(DPR_ERR_INVALID_ARG, "sh_frame must be 0 or 1");
    if (pr->bwd_mode != 0 && pr->bwd_mode != 1) return fail(DPR_ERR_INVALID_ARG, "bwd_mode must be 0 or 1");
    if (pr->flags & ~(DPR_FLAG_TIMING | DPR_FLAG_STATS | DPR_FLAG_PERSISTENT | DPR_FLAG_KERNEL_NORM))
        return fail(DPR_ERR_INVALID_ARG, "unknown flags 0x%x", pr->flags);
    if (pr->max_splats < 0) return fail(DPR_ERR_INVALID_ARG, "max_splats must be >= 0");
    if (pr->timing_stages & ~((1 << DPR_STAGE_COUNT) - 1))
        return fail(DPR_ERR_INVALID_ARG, "timing_stages 0x%x names no stage", pr->timing_stages);
    return DPR_OK;
}

int check_inputs(const dpr_scene *scenes, int32_t n_scenes, const dpr_view *views, int32_t n_views, Sizes *out) {
    if (n_scenes < 1 || !scenes) return fail(DPR_ERR_INVALID_ARG, "need at least one scene");
    if (n_views < 1 || !views) return fail(DPR_ERR_INVALID_ARG, "need at least one view");
    if (n_views > (1 << 20) || n_scenes > (1 << 20)) return fail(DPR_ERR_UNSUPPORTED, "too many views or scenes");
    Sizes s;
    s.n_views = n_views;
    s.n_scenes = n_scenes;
    s.sh_degree = scenes[0].sh_degree;
    for (int32_t i = 0; i < n_scenes; ++i) {
        const dpr_scene &sc = scenes[i];
        if (sc.n < 0 || sc.n > 0x7FFFFFFFll) return fail(DPR_ERR_INVALID_ARG, "scene %d: n out of range", i);
        if (sc.sh_degree < 0 || sc.sh_degree > 3)
            return fail(DPR_ERR_INVALID_ARG, "scene %d: sh_degree must be in [0, 3]", i);
        if (sc.sh_degree != s.sh_degree)
            return fail(DPR_ERR_UNSUPPORTED, "scene %d: all scenes of a plan must share sh_degree", i);
        if (sc.reserved != 0) return fail(DPR_ERR_INVALID_ARG, "scene %d: reserved must be 0", i);
        if (sc.n > 0 && (!sc.xyz || !sc.sh || !sc.opacity || !sc.radius))
            return fail(DPR_ERR_INVALID_ARG, "scene %d: NULL array", i);
        s.point_blocks += ((uint64_t)sc.n + 127) / 128;
    }
    for (int32_t v = 0; v < n_views; ++v) {
        const dpr_view &vw = views[v];
        if (vw.scene < 0 || vw.scene >= n_scenes) return fail(DPR_ERR_INVALID_ARG, "view %d: bad scene index", v);
        if (vw.reserved != 0) return fail(DPR_ERR_INVALID_ARG, "view %d: reserved must be 0", v);
        const dpr_camera &c = vw.cam;
        if (c.width < 1 || c.width > kLimitDim || c.height < 1 || c.height > kLimitDim)
            return fail(DPR_ERR_INVALID_ARG, "view %d: width/height must be in [1, %d]", v, kLimitDim);
        if (!(c.fx > 0.f) || !(c.fy > 0.f) || !std::isfinite(c.fx) || !std::isfinite(c.fy))
            return fail(DPR_ERR_INVALID_ARG, "view %d: fx, fy must be finite and > 0", v);
        if (!vw.image) return fail(DPR_ERR_INVALID_ARG, "view %d: image is NULL", v);
        const uint64_t n = (uint64_t)scenes[vw.scene].n;
        s.items += n;
        const uint64_t tx = ((uint64_t)c.width + kTile - 1) / kTile, ty = ((uint64_t)c.height + kTile - 1) / kTile;
        s.tiles += tx * ty;
        s.max_view_tiles = std::max(s.max_view_tiles, tx * ty);
        s.pixels += (uint64_t)c.width * (uint64_t)c.height;
        const uint64_t nch = (n + kChunkItems - 1) / kChunkItems;
        const uint64_t nseg = (nch + kSegChunks - 1) / kSegChunks;
        s.chunks += nch;
        s.cnt += tx * ty * nch;
        s.segs += tx * ty * nseg;
        s.max_view_segs = std::max(s.max_view_segs, nseg);
        s.sort_blocks += (n + kDepthSortTile - 1) / kDepthSortTile;
    }
    if (s.items >= 0x7FFFFFFFull) return fail(DPR_ERR_UNSUPPORTED, "total view-points must be < 2^31");
    if (s.tiles >= 0xFFFFFFFFull || s.cnt >= 0xFFFFFFFFull || s.chunks >= 0xFFFFFFFFull)
        return fail(DPR_ERR_UNSUPPORTED, "too many tiles");
    *out = s;
    return DPR_OK;
}

struct Events {
    hipEvent_t a[DPR_STAGE_COUNT] = {};
    hipEvent_t b[DPR_STAGE_COUNT] = {};
    bool ran[DPR_STAGE_COUNT] = {};
};

bool fault_injected(const char *what) {
    const char *f = getenv("DPR_FAULT");
    return f && strcmp(f, what) == 0;
}

}  // namespace

struct dpr_plan {
    Sizes sz;
    PlanLayout lay;
    dpr_params params;
    Thresholds th;
    std::vector<dpr_scene> scenes;
    std::vector<dpr_view> views;
    std::vector<ViewDesc> vdesc;
    std::vector<SceneDesc> sdesc;
    std::vector<uint32_t> u32tab;
    std::vector<uint32_t> up_img;   // the upload image of views, scenes and u32tab
    uint8_t *pws = nullptr;
    uint64_t pairs = 0;
    uint64_t fwd_pairs = 0;          // the pair count the forward workspace in use was laid out for
    int forward_done = 0;
    const void *fwd_ws = nullptr;
    Events ev;
    bool timing = false;
    uint32_t timed = 0;             // bit s: stage s records its events
    // backward host tables (kept alive while copies may be in flight)
    std::vector<uint64_t> bwd_tab;
    std::vector<SceneDesc> sdesc_bwd;
};

namespace {

Tables make_tables(const dpr_plan *p) {
    Tables tb;
    const uint32_t *u = reinterpret_cast<const uint32_t *>(p->pws + p->lay.u32tab.off);
    const int V = p->sz.n_views, S = p->sz.n_scenes;
    tb.views = reinterpret_cast<const ViewDesc *>(p->pws + p->lay.views.off);
    tb.scenes = reinterpret_cast<const SceneDesc *>(p->pws + p->lay.scenes.off);
    tb.scene_views = u;
    tb.scene_block_start = u + V;
    tb.sort_block_start = u + V + S;
    tb.chunk_start = u + 2 * V + S;
    tb.tile_start = u + 3 * V + S;
    tb.n_views = V;
    tb.n_scenes = S;
    tb.max_view_tiles = (uint32_t)p->sz.max_view_tiles;
    tb.max_view_segs = (uint32_t)p->sz.max_view_segs;
    tb.total_tiles = (uint32_t)p->sz.tiles;
    return tb;
}

struct StageScope {
    dpr_plan *p;
    int stage;
    hipStream_t st;
    StageScope(dpr_plan *p_, int s, hipStream_t st_) : p(p_), stage(s), st(st_) {
        if ((p->timed >> stage) & 1u) (void)hipEventRecord(p->ev.a[stage], st);   // timing only: not fatal
    }
    ~StageScope() {
        if ((p->timed >> stage) & 1u) {
            (void)hipEventRecord(p->ev.b[stage], st);
            p->ev.ran[stage] = true;
        }
    }
};

// Per-pixel and per-tile state a backward reads: stop index, final (T, I),
// (T, I) checkpoints every kBwdSeg list positions, and (tile, segment) work
// items.  Held in the forward workspace in stored mode and in the backward
// workspace in recompute mode.
struct BwdState {
    Region nlast, fin, ckpt, work;
};

BwdState add_bwd_state(Layout &L, const dpr_plan *p, bool on, uint64_t pairs) {
    BwdState s;
    s.nlast = L.add(on ? 4 * p->sz.pixels : 0);
    s.fin = L.add(on ? 16 * p->sz.pixels : 0);
    s.ckpt = L.add(on ? 16ull * kTilePix * ckpt_slots(pairs, p->sz.tiles) : 0);
    s.work = L.add(on ? 8 * work_capacity(pairs, p->sz.tiles) : 0);
    return s;
}

struct FwdLayout {
    Region pairs, stats, counters;
    BwdState st;
    uint64_t total = 0;
};

// The forward workspace laid out for `pairs` (tile, splat) pairs: a workspace
// laid out for more pairs than the plan has serves it as well.
FwdLayout fwd_layout_for(const dpr_plan *p, uint64_t pairs) {
    Layout L;
    FwdLayout f;
    f.pairs = L.add(4 * pairs);
    f.st = add_bwd_state(L, p, p->params.bwd_mode == DPR_BWD_STORED, pairs);
    f.stats = L.add((p->params.flags & DPR_FLAG_STATS) ? 4 * p->sz.pixels : 0);
    f.counters = L.add(16);
    f.total = L.total;
    return f;
}

// The layout of the forward workspace in use.
FwdLayout fwd_layout(const dpr_plan *p) { return fwd_layout_for(p, p->fwd_pairs); }

// The most pairs a forward workspace of `bytes` can hold (its size grows with
// the pair count), or -1 if it cannot hold the plan's per-pixel state at all.
int64_t pairs_that_fit(const dpr_plan *p, uint64_t bytes) {
    if (fwd_layout_for(p, 0).total > bytes) return -1;
    uint64_t lo = 0, hi = 0xFFFFFFFEull;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        if (fwd_layout_for(p, mid).total <= bytes) lo = mid;
        else hi = mid - 1;
    }
    return (int64_t)lo;
}

struct BwdLayout {
    Region tabs, sgrad, grad, counters;
    BwdState st;
    uint64_t total = 0;
};

BwdLayout bwd_layout(const dpr_plan *p) {
    Layout L;
    BwdLayout b;
    b.tabs = L.add(8ull * 2 * p->sz.n_views);
    b.sgrad = L.add(sizeof(SceneDesc) * (uint64_t)p->sz.n_scenes);
    b.grad = L.add(32ull * p->sz.items);
    b.st = add_bwd_state(L, p, p->params.bwd_mode == DPR_BWD_RECOMPUTE, p->pairs);
    b.counters = L.add(16);
    b.total = L.total;
    return b;
}

// Points the composite arguments at a backward state region.
void set_bwd_state(CompositeArgs &a, uint8_t *base, const BwdState &s) {
    a.nlast = reinterpret_cast<uint32_t *>(base + s.nlast.off);
    a.fin = reinterpret_cast<float4 *>(base + s.fin.off);
    a.ckpt = reinterpret_cast<float4 *>(base + s.ckpt.off);
    a.work = reinterpret_cast<uint2 *>(base + s.work.off);
}

CompositeArgs composite_args(const dpr_plan *p, const void *ws) {
    const Tables tb = make_tables(p);
    const FwdLayout f = fwd_layout(p);
    const uint8_t *w = static_cast<const uint8_t *>(ws);
    CompositeArgs a;
    a.views = tb.views;
    a.tile_start = tb.tile_start;
    a.n_views = tb.n_views;
    a.total_tiles = (uint32_t)p->sz.tiles;
    a.rec = reinterpret_cast<const SplatRec *>(p->pws + p->lay.rec.off);
    a.pairs = reinterpret_cast<const uint32_t *>(w + f.pairs.off);
    a.tile_base = reinterpret_cast<const uint32_t *>(p->pws + p->lay.tile_base.off);
    a.tile_order = reinterpret_cast<const uint32_t *>(p->pws + p->lay.tile_order.off);
    a.write_views = 0;
    a.stats = nullptr;
    a.nlast = nullptr;
    a.fin = nullptr;
    a.ckpt = nullptr;
    a.work = nullptr;
    a.counters = nullptr;
    a.th = p->th;
    return a;
}

// Workspace of dpr_loss_l2_tv: per-block sums of the largest batch of images.
struct LossLayout {
    Region partial;
    uint64_t total = 0;
};

int loss_layout(int32_t n, const int32_t *widths, const int32_t *heights, LossLayout *out) {
    if (n < 1 || n > (1 << 20)) return fail(DPR_ERR_INVALID_ARG, "n_images must be in [1, 2^20]");
    if (!widths || !heights) return fail(DPR_ERR_INVALID_ARG, "widths / heights is NULL");
    uint64_t most = 0, batch = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (widths[v] < 1 || heights[v] < 1 || widths[v] > kLimitDim || heights[v] > kLimitDim)
            return fail(DPR_ERR_INVALID_ARG, "image %d: size %dx%d outside [1, %d]", v, widths[v], heights[v],
                        kLimitDim);
        if (v % kLossBatch == 0) batch = 0;
        batch += loss_blocks(widths[v], heights[v]);
        most = std::max(most, batch);
    }
    if (most >= 0xFFFFFFFFull) return fail(DPR_ERR_UNSUPPORTED, "too many pixels in one batch");
    Layout L;
    out->partial = L.add(4 * most);
    out->total = L.total;
    return DPR_OK;
}

// Scratch of the hybrid update / neighbour search for up to n points.
struct HyLayout {
    Region keys, vals, keys_alt, vals_alt, hist, part, total, flags, seg, starts, cell_start, box_part, box, idx, d2,
        red;
    uint64_t total_bytes = 0;
};

HyLayout hy_layout(uint64_t n, int K, int k3, bool reduced_cloud) {
    Layout L;
    HyLayout h;
    const HyScratchBytes b = hy_scratch_bytes(n, K);
    h.keys = L.add(b.keys);
    h.vals = L.add(b.vals);
    h.keys_alt = L.add(b.keys_alt);
    h.vals_alt = L.add(b.vals_alt);
    h.hist = L.add(b.hist);
    h.part = L.add(b.part);
    h.total = L.add(b.total64);
    h.flags = L.add(b.flags);
    h.seg = L.add(b.seg);
    h.starts = L.add(b.starts);
    h.cell_start = L.add(b.cell_start);
    h.box_part = L.add(b.box_part);
    h.box = L.add(b.box);
    h.idx = L.add(b.idx);
    h.d2 = L.add(b.d2);
    h.red = L.add(reduced_cloud ? 4 * n * (uint64_t)(5 + k3) : 0);
    h.total_bytes = L.total;
    return h;
}

HyScratch hy_scratch(uint8_t *w, const HyLayout &h) {
    HyScratch s;
    s.keys = reinterpret_cast<uint32_t *>(w + h.keys.off);
    s.vals = reinterpret_cast<uint32_t *>(w + h.vals.off);
    s.keys_alt = reinterpret_cast<uint32_t *>(w + h.keys_alt.off);
    s.vals_alt = reinterpret_cast<uint32_t *>(w + h.vals_alt.off);
    s.hist = reinterpret_cast<uint32_t *>(w + h.hist.off);
    s.part = reinterpret_cast<uint64_t *>(w + h.part.off);
    s.total64 = reinterpret_cast<uint64_t *>(w + h.total.off);
    s.flags = reinterpret_cast<uint32_t *>(w + h.flags.off);
    s.seg = reinterpret_cast<uint32_t *>(w + h.seg.off);
    s.starts = reinterpret_cast<uint32_t *>(w + h.starts.off);
    s.cell_start = reinterpret_cast<uint32_t *>(w + h.cell_start.off);
    s.box_part = reinterpret_cast<float *>(w + h.box_part.off);
    s.box = reinterpret_cast<float *>(w + h.box.off);
    s.idx = reinterpret_cast<int32_t *>(w + h.idx.off);
    s.d2 = reinterpret_cast<float *>(w + h.d2.off);
    return s;
}

// Camera / mask table of the consistency check; 0 or an error code.
int hull_table(int32_t n_cams, const dpr_camera *cams, const dpr_mask *masks, std::vector<HullCam> &out) {
    if (n_cams < 1 || n_cams > kHullMaxCams) return fail(DPR_ERR_INVALID_ARG, "n_cams must be in [1, %d]", kHullMaxCams);
    if (!cams || !masks) return fail(DPR_ERR_INVALID_ARG, "cams or masks is NULL");
    out.resize((size_t)n_cams);
    for (int32_t i = 0; i < n_cams; ++i) {
        const dpr_camera &c = cams[i];
        if (c.width < 1 || c.width > kLimitDim || c.height < 1 || c.height > kLimitDim)
            return fail(DPR_ERR_INVALID_ARG, "camera %d: width/height must be in [1, %d]", i, kLimitDim);
        if (!(c.fx > 0.f) || !(c.fy > 0.f) || !std::isfinite(c.fx) || !std::isfinite(c.fy))
            return fail(DPR_ERR_INVALID_ARG, "camera %d: fx, fy must be finite and > 0", i);
        if (!masks[i].data) return fail(DPR_ERR_INVALID_ARG, "mask %d is NULL", i);
        if (masks[i].width != c.width || masks[i].height != c.height)
            return fail(DPR_ERR_INVALID_ARG, "mask %d is %dx%d, its camera's image %dx%d", i, masks[i].width,
                        masks[i].height, c.width, c.height);
        HullCam &h = out[(size_t)i];
        memcpy(h.R, c.R, sizeof(h.R));
        memcpy(h.t, c.t, sizeof(h.t));
        h.fx = c.fx; h.fy = c.fy; h.cx = c.cx; h.cy = c.cy;
        h.width = c.width; h.height = c.height;
        h.mask = masks[i].data;
    }
    return DPR_OK;
}

int check_hybrid_args(int64_t n, int32_t sh_degree, int32_t K) {
    if (n < 1 || n > (int64_t)0x7FFFFFFF) return fail(DPR_ERR_INVALID_ARG, "point count must be in [1, 2^31 - 1]");
    if (sh_degree < 0 || sh_degree > 3) return fail(DPR_ERR_INVALID_ARG, "sh_degree must be in [0, 3]");
    if (K < 1 || K > kKnnMax) return fail(DPR_ERR_INVALID_ARG, "K must be in [1, %d]", kKnnMax);
    return DPR_OK;
}

}  // namespace

int dpr::set_last_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

extern "C" {

int dpr_version(void) { return DPR_ABI_VERSION; }

const char *dpr_last_error(void) { return g_err.c_str(); }

size_t dpr_plan_ws_bytes(const dpr_scene *scenes, int32_t n_scenes, const dpr_view *views, int32_t n_views) {
    Sizes s;
    if (check_inputs(scenes, n_scenes, views, n_views, &s) != DPR_OK) return 0;
    return (size_t)plan_layout(s).total;
}

namespace {
int launch_forward(dpr_plan *p, void *ws, uint64_t layout_pairs, uint32_t pair_cap, hipStream_t st);
int64_t pairs_that_fit(const dpr_plan *p, uint64_t bytes);

// The plan stage; with fwd_ws, also the forward into it, queued before the
// wait for the pair count (the kernels check the count against what fwd_ws
// can hold and do nothing if it does not fit); *rendered tells which.
int plan_forward_impl(const dpr_scene *scenes, int32_t n_scenes, const dpr_view *views, int32_t n_views,
                      const dpr_params *params, void *plan_ws, size_t plan_ws_bytes, void *fwd_ws,
                      size_t fwd_ws_bytes, void *stream, dpr_plan **out, int32_t *rendered) {
    g_err.clear();
    if (!out) return fail(DPR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (rendered) *rendered = 0;
    int rc = check_params(params);
    if (rc) return rc;
    Sizes s;
    rc = check_inputs(scenes, n_scenes, views, n_views, &s);
    if (rc) return rc;
    const PlanLayout lay = plan_layout(s);
    if (!plan_ws || plan_ws_bytes < lay.total)
        return fail(DPR_ERR_WORKSPACE, "plan workspace needs %llu bytes, got %llu", (unsigned long long)lay.total,
                    (unsigned long long)plan_ws_bytes);
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");

    dpr_plan *p = new dpr_plan();
    p->sz = s;
    p->lay = lay;
    p->params = *params;
    p->th.lambda = params->alpha_min > 0.f ? -log2f(params->alpha_min) : INFINITY;
    p->th.alpha_max = params->alpha_max;
    p->th.t_min = params->t_min;
    p->th.z_near = params->z_near;
    p->th.sh_frame = params->sh_frame;
    p->th.max_splats = (uint32_t)params->max_splats;
    p->th.kernel_norm = (params->flags & DPR_FLAG_KERNEL_NORM) ? 1 : 0;
    p->scenes.assign(scenes, scenes + n_scenes);
    p->views.assign(views, views + n_views);
    p->pws = static_cast<uint8_t *>(plan_ws);
    p->timing = (params->flags & DPR_FLAG_TIMING) != 0;
    p->timed = !p->timing ? 0u
                          : (params->timing_stages ? (uint32_t)params->timing_stages : (1u << DPR_STAGE_COUNT) - 1u);
    hipStream_t st = static_cast<hipStream_t>(stream);

    auto cleanup_fail = [&](int code) {
        dpr_plan_free(p);
        return code;
    };
    if (p->timing) {
        for (int i = 0; i < DPR_STAGE_COUNT; ++i) {
            if (!((p->timed >> i) & 1u)) continue;
            if (hipEventCreate(&p->ev.a[i]) != hipSuccess || hipEventCreate(&p->ev.b[i]) != hipSuccess)
                return cleanup_fail(fail(DPR_ERR_HIP, "hipEventCreate failed"));
        }
    }

    // host tables
    const int V = n_views, S = n_scenes;
    p->vdesc.resize(V);
    p->sdesc.resize(S);
    p->u32tab.assign(4 * (size_t)V + S, 0u);
    uint32_t *scene_views = p->u32tab.data();
    uint32_t *scene_block_start = scene_views + V;
    uint32_t *sort_block_start = scene_block_start + S;
    uint32_t *chunk_start = sort_block_start + V;
    uint32_t *tile_start = chunk_start + V;
    {
        std::vector<uint32_t> count(S, 0);
        for (int v = 0; v < V; ++v) count[views[v].scene]++;
        uint32_t acc = 0, blk = 0;
        for (int sidx = 0; sidx < S; ++sidx) {
            SceneDesc &d = p->sdesc[sidx];
            memset(&d, 0, sizeof(d));
            d.n = (int32_t)scenes[sidx].n;
            d.sh_degree = scenes[sidx].sh_degree;
            d.view_start = acc;
            d.view_count = 0;
            d.block_off = blk;
            d.xyz = scenes[sidx].xyz;
            d.sh = scenes[sidx].sh;
            d.opacity = scenes[sidx].opacity;
            d.radius = scenes[sidx].radius;
            scene_block_start[sidx] = blk;
            blk += (uint32_t)((d.n + 127) / 128);
            acc += count[sidx];
        }
        for (int v = 0; v < V; ++v) {
            SceneDesc &d = p->sdesc[views[v].scene];
            scene_views[d.view_start + d.view_count++] = (uint32_t)v;
        }
    }
    {
        uint64_t item = 0, tile = 0, chunk = 0, sblk = 0, hist = 0, cnt = 0, seg = 0, pix = 0;
        for (int v = 0; v < V; ++v) {
            const dpr_view &vw = views[v];
            ViewDesc &d = p->vdesc[v];
            memset(&d, 0, sizeof(d));
            memcpy(d.R, vw.cam.R, sizeof(d.R));
            memcpy(d.t, vw.cam.t, sizeof(d.t));
            d.fx = vw.cam.fx; d.fy = vw.cam.fy; d.cx = vw.cam.cx; d.cy = vw.cam.cy;
            d.width = vw.cam.width;
            d.height = vw.cam.height;
            d.tiles_x = (d.width + kTile - 1) / kTile;
            d.tiles_y = (d.height + kTile - 1) / kTile;
            d.scene = vw.scene;
            const dpr_scene &sc = scenes[vw.scene];
            d.sh_degree = sc.sh_degree;
            d.n = (int32_t)sc.n;
            d.item_off = (uint32_t)item;
            d.tile_off = (uint32_t)tile;
            d.chunk_off = (uint32_t)chunk;
            d.nchunks = (uint32_t)(((uint64_t)sc.n + kChunkItems - 1) / kChunkItems);
            d.sort_block_off = (uint32_t)sblk;
            d.nsort_blocks = (uint32_t)(((uint64_t)sc.n + kDepthSortTile - 1) / kDepthSortTile);
            d.hist_off = hist;
            d.cnt_off = cnt;
            d.seg_off = seg;
            d.pix_off = pix;
            d.xyz = sc.xyz; d.sh = sc.sh; d.opacity = sc.opacity; d.radius = sc.radius;
            d.image = vw.image;
            d.trans = vw.trans;
            sort_block_start[v] = d.sort_block_off;
            chunk_start[v] = d.chunk_off;
            tile_start[v] = d.tile_off;
            const uint64_t nt = (uint64_t)d.tiles_x * d.tiles_y;
            item += (uint64_t)sc.n;
            tile += nt;
            chunk += d.nchunks;
            sblk += d.nsort_blocks;
            hist += 256ull * d.nsort_blocks;
            cnt += nt * d.nchunks;
            seg += nt * ((d.nchunks + kSegChunks - 1) / kSegChunks);
            pix += (uint64_t)d.width * d.height;
        }
    }

    uint8_t *w = p->pws;
    const Tables tb = make_tables(p);
    SplatRec *rec = reinterpret_cast<SplatRec *>(w + lay.rec.off);
    uint32_t *keys = reinterpret_cast<uint32_t *>(w + lay.keys.off);
    uint32_t *vals = reinterpret_cast<uint32_t *>(w + lay.vals.off);
    uint32_t *keys_alt = reinterpret_cast<uint32_t *>(w + lay.keys_alt.off);
    uint32_t *vals_alt = reinterpret_cast<uint32_t *>(w + lay.vals_alt.off);
    uint2 *rect = reinterpret_cast<uint2 *>(w + lay.rect.off);
    uint32_t *hist = reinterpret_cast<uint32_t *>(w + lay.hist.off);
    uint64_t *part = reinterpret_cast<uint64_t *>(w + lay.part.off);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(w + lay.cnt.off);
    uint32_t *segs = reinterpret_cast<uint32_t *>(w + lay.segs.off);
    uint32_t *tile_total = reinterpret_cast<uint32_t *>(w + lay.tile_total.off);
    uint32_t *tile_base = reinterpret_cast<uint32_t *>(w + lay.tile_base.off);
    const uint64_t np = lay.part.bytes / 8;
    uint64_t *total64 = part + np - 1;

#define STAGE_TRY(expr)                                                                           \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return cleanup_fail(fail(DPR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)));       \
    } while (0)

    {
        StageScope sc_(p, DPR_STAGE_UPLOAD, st);
        // the three tables are the first regions of the layout: one image of them
        const uint64_t img = lay.u32tab.off + 4 * p->u32tab.size() - lay.views.off;
        p->up_img.assign((size_t)(img / 4), 0u);
        uint8_t *h = reinterpret_cast<uint8_t *>(p->up_img.data());
        memcpy(h + (lay.views.off - lay.views.off), p->vdesc.data(), sizeof(ViewDesc) * V);
        memcpy(h + (lay.scenes.off - lay.views.off), p->sdesc.data(), sizeof(SceneDesc) * S);
        memcpy(h + (lay.u32tab.off - lay.views.off), p->u32tab.data(), 4 * p->u32tab.size());
        STAGE_TRY(upload_async(w + lay.views.off, h, img, st));
    }
    {
        StageScope sc_(p, DPR_STAGE_PROJECT, st);
        STAGE_TRY(launch_project(tb, p->th, s.sh_degree, (uint32_t)s.point_blocks, rec, keys, vals, rect, st));
    }
    {
        StageScope sc_(p, DPR_STAGE_DEPTH_SORT, st);
        STAGE_TRY(launch_depth_sort(tb, (uint32_t)s.sort_blocks, (uint32_t)s.items, keys, vals, keys_alt, vals_alt,
                                    hist, part, st));
    }
    {
        StageScope sc_(p, DPR_STAGE_TILE_COUNT, st);
        STAGE_TRY(launch_tile_count(tb, (uint32_t)s.chunks, vals, rect, rec, p->th.lambda, cnt,
                                    reinterpret_cast<BinRec *>(w + lay.bin.off), st));
    }
    {
        StageScope sc_(p, DPR_STAGE_TILE_SCAN, st);
        uint32_t *bucket_cnt = reinterpret_cast<uint32_t *>(w + lay.bucket_cnt.off);
        uint64_t *block_sum = reinterpret_cast<uint64_t *>(w + lay.block_sum.off);
        STAGE_TRY(launch_tile_colscan(tb, cnt, segs, tile_total, bucket_cnt, block_sum, tile_base,
                                      reinterpret_cast<uint32_t *>(w + lay.tile_order.off), total64, st));
    }
    if (!fwd_ws) {
        STAGE_TRY(read_count(total64, &p->pairs, st));
    } else {
        STAGE_TRY(read_count_begin(total64, st));
        const int64_t cap = pairs_that_fit(p, fwd_ws_bytes);
        if (cap >= 0) {
            const int rc2 = launch_forward(p, fwd_ws, (uint64_t)cap, (uint32_t)cap, st);
            if (rc2) return cleanup_fail(rc2);
        }
        STAGE_TRY(read_count_end(&p->pairs));
        if (cap >= 0 && p->pairs <= (uint64_t)cap) {
            p->forward_done = 1;
            p->fwd_ws = fwd_ws;
            if (rendered) *rendered = 1;
        }
    }
    if (!p->forward_done) p->fwd_pairs = p->pairs;
    if (p->pairs >= 0xFFFFFFFFull)
        return cleanup_fail(fail(DPR_ERR_UNSUPPORTED, "%llu (tile, splat) pairs exceed 2^32 - 1",
                                 (unsigned long long)p->pairs));
#undef STAGE_TRY
    *out = p;
    return DPR_OK;
}

}  // namespace

int dpr_plan_forward(const dpr_scene *scenes, int32_t n_scenes, const dpr_view *views, int32_t n_views,
                     const dpr_params *params, void *plan_ws, size_t plan_ws_bytes, void *stream,
                     dpr_plan **out) {
    return plan_forward_impl(scenes, n_scenes, views, n_views, params, plan_ws, plan_ws_bytes, nullptr, 0, stream,
                             out, nullptr);
}

int dpr_plan_forward_render(const dpr_scene *scenes, int32_t n_scenes, const dpr_view *views, int32_t n_views,
                            const dpr_params *params, void *plan_ws, size_t plan_ws_bytes, void *fwd_ws,
                            size_t fwd_ws_bytes, void *stream, dpr_plan **out, int32_t *rendered) {
    if (!rendered) return fail(DPR_ERR_INVALID_ARG, "rendered is NULL");
    if (!fwd_ws) return fail(DPR_ERR_INVALID_ARG, "fwd_ws is NULL (dpr_plan_forward plans without a forward)");
    return plan_forward_impl(scenes, n_scenes, views, n_views, params, plan_ws, plan_ws_bytes, fwd_ws, fwd_ws_bytes,
                             stream, out, rendered);
}

size_t dpr_workspace_bytes(const dpr_plan *plan) {
    if (!plan) return 0;
    return (size_t)fwd_layout_for(plan, plan->pairs).total;
}

size_t dpr_backward_ws_bytes(const dpr_plan *plan) {
    if (!plan) return 0;
    return (size_t)bwd_layout(plan).total;
}

namespace {

// Emission and compositing into `ws`, laid out for layout_pairs pairs; the
// kernels do nothing if the plan holds more than pair_cap pairs.
int launch_forward(dpr_plan *p, void *ws, uint64_t layout_pairs, uint32_t pair_cap, hipStream_t st) {
    p->fwd_pairs = layout_pairs;
    const FwdLayout f = fwd_layout(p);
    uint8_t *w = static_cast<uint8_t *>(ws);
    const Tables tb = make_tables(p);
    const PlanLayout &lay = p->lay;
    {
        StageScope sc_(p, DPR_STAGE_EMIT, st);
        HIP_TRY(launch_tile_emit(tb, (uint32_t)p->sz.chunks, reinterpret_cast<const BinRec *>(p->pws + lay.bin.off),
                                 reinterpret_cast<const uint32_t *>(p->pws + lay.cnt.off),
                                 reinterpret_cast<const uint32_t *>(p->pws + lay.tile_base.off),
                                 reinterpret_cast<uint32_t *>(w + f.pairs.off),
                                 reinterpret_cast<uint32_t *>(w + f.counters.off), pair_cap, st));
    }
    CompositeArgs a = composite_args(p, ws);
    a.pair_cap = pair_cap;
    a.write_views = 1;
    a.stats = f.stats.bytes ? reinterpret_cast<uint32_t *>(w + f.stats.off) : nullptr;
    if (p->params.bwd_mode == DPR_BWD_STORED) set_bwd_state(a, w, f.st);
    a.counters = reinterpret_cast<uint32_t *>(w + f.counters.off);
    const bool persistent = (p->params.flags & DPR_FLAG_PERSISTENT) != 0;
    {
        StageScope sc_(p, DPR_STAGE_COMPOSITE_FWD, st);   // the counters were cleared by the emission
        HIP_TRY(launch_composite_fwd(a, persistent, st));
    }
    return DPR_OK;
}

}  // namespace

int dpr_render_forward(dpr_plan *p, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!p) return fail(DPR_ERR_INVALID_ARG, "plan is NULL");
    const uint64_t need = fwd_layout_for(p, p->pairs).total;
    if (!ws || ws_bytes < need)
        return fail(DPR_ERR_WORKSPACE, "forward workspace needs %llu bytes, got %llu", (unsigned long long)need,
                    (unsigned long long)ws_bytes);
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    p->forward_done = 0;
    const int rc = launch_forward(p, ws, p->pairs, 0xFFFFFFFFu, static_cast<hipStream_t>(stream));
    if (rc) return rc;
    p->forward_done = 1;
    p->fwd_ws = ws;
    return DPR_OK;
}

int dpr_render_backward(dpr_plan *p, const void *ws, size_t ws_bytes, const float *const *dL_dimage,
                        const float *const *dL_dtrans, float *const *dL_dxyz, float *const *dL_dsh,
                        float *const *dL_dopacity, void *bwd_ws, size_t bwd_ws_bytes, void *stream) {
    g_err.clear();
    if (!p) return fail(DPR_ERR_INVALID_ARG, "plan is NULL");
    if (!p->forward_done) return fail(DPR_ERR_STATE, "dpr_render_backward before dpr_render_forward");
    const FwdLayout f = fwd_layout(p);
    if (!ws || ws_bytes < f.total) return fail(DPR_ERR_WORKSPACE, "forward workspace too small");
    // the tile lists (and in stored mode the backward state) live in the
    // workspace the forward wrote; any other buffer holds item ids and work
    // items of some other plan
    if (ws != p->fwd_ws)
        return fail(DPR_ERR_STATE, "dpr_render_backward needs the workspace of this plan's dpr_render_forward");
    const BwdLayout bl = bwd_layout(p);
    if (!bwd_ws || bwd_ws_bytes < bl.total)
        return fail(DPR_ERR_WORKSPACE, "backward workspace needs %llu bytes, got %llu",
                    (unsigned long long)bl.total, (unsigned long long)bwd_ws_bytes);
    if (p->params.alpha_max > 0.999f)
        return fail(DPR_ERR_INVALID_ARG, "backward needs alpha_max <= 0.999 (T is recovered by division)");
    if (!dL_dimage) return fail(DPR_ERR_INVALID_ARG, "dL_dimage is NULL");
    const int V = p->sz.n_views, S = p->sz.n_scenes;
    const bool recompute = p->params.bwd_mode == DPR_BWD_RECOMPUTE;
    for (int v = 0; v < V; ++v)
        if (!dL_dimage[v]) return fail(DPR_ERR_INVALID_ARG, "dL_dimage[%d] is NULL", v);
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *bw = static_cast<uint8_t *>(bwd_ws);
    const uint8_t *w = static_cast<const uint8_t *>(ws);

    // pointer tables: dimage[V], dtrans[V]; scene descriptors with gradient outputs
    p->bwd_tab.assign(2 * (size_t)V, 0ull);
    for (int v = 0; v < V; ++v) {
        p->bwd_tab[v] = (uint64_t)(uintptr_t)dL_dimage[v];
        p->bwd_tab[V + v] = dL_dtrans ? (uint64_t)(uintptr_t)dL_dtrans[v] : 0ull;
    }
    p->sdesc_bwd = p->sdesc;
    for (int s = 0; s < S; ++s) {
        p->sdesc_bwd[s].dxyz = dL_dxyz ? dL_dxyz[s] : nullptr;
        p->sdesc_bwd[s].dsh = dL_dsh ? dL_dsh[s] : nullptr;
        p->sdesc_bwd[s].dopacity = dL_dopacity ? dL_dopacity[s] : nullptr;
    }
    // pointer tables and gradient scene descriptors (adjacent regions: one
    // image), with the counters and the gradient accumulators cleared in the
    // same launch
    {
        const uint64_t img = bl.sgrad.off + sizeof(SceneDesc) * S - bl.tabs.off;
        p->up_img.assign((size_t)(img / 4), 0u);
        uint8_t *h = reinterpret_cast<uint8_t *>(p->up_img.data());
        memcpy(h, p->bwd_tab.data(), 8 * p->bwd_tab.size());
        memcpy(h + (bl.sgrad.off - bl.tabs.off), p->sdesc_bwd.data(), sizeof(SceneDesc) * S);
        HIP_TRY(upload_zero_async(bw + bl.tabs.off, h, img, reinterpret_cast<uint32_t *>(bw + bl.counters.off), 4,
                                  reinterpret_cast<uint32_t *>(bw + bl.grad.off), 8ull * p->sz.items, st));
    }

    CompositeArgs a = composite_args(p, ws);
    const bool persistent = (p->params.flags & DPR_FLAG_PERSISTENT) != 0;
    uint32_t *counters = reinterpret_cast<uint32_t *>(bw + bl.counters.off);   // [0] recompute queue, [1] work
    BackwardArgs b;                                                                // items, [2] backward queue
    b.dimage = reinterpret_cast<const float *const *>(bw + bl.tabs.off);
    b.dtrans = dL_dtrans ? reinterpret_cast<const float *const *>(bw + bl.tabs.off + 8ull * V) : nullptr;
    b.grad = reinterpret_cast<float *>(bw + bl.grad.off);
    if (recompute) {
        // the forward again, writing only the backward state (to the backward workspace)
        set_bwd_state(a, bw, bl.st);
        a.counters = counters;
        StageScope sc_(p, DPR_STAGE_RECOMPUTE, st);
        HIP_TRY(launch_composite_fwd(a, persistent, st));
        b.work_count = counters + 1;
    } else {
        set_bwd_state(a, const_cast<uint8_t *>(w), f.st);
        b.work_count = reinterpret_cast<const uint32_t *>(w + f.counters.off) + 1;
    }
    b.nlast = a.nlast;
    b.fin = a.fin;
    b.ckpt = a.ckpt;
    b.work = a.work;
    b.queue = counters + 2;
    a.nlast = nullptr;
    a.fin = nullptr;
    a.ckpt = nullptr;
    a.work = nullptr;
    a.counters = nullptr;
    b.c = a;
    {
        StageScope sc_(p, DPR_STAGE_COMPOSITE_BWD, st);
        HIP_TRY(launch_composite_bwd(b, st));
    }
    {
        Tables tb = make_tables(p);
        tb.scenes = reinterpret_cast<const SceneDesc *>(bw + bl.sgrad.off);
        StageScope sc_(p, DPR_STAGE_POINT_BWD, st);
        HIP_TRY(launch_point_bwd(tb, p->th, p->sz.sh_degree, (uint32_t)p->sz.point_blocks, b.grad, st));
    }
    return DPR_OK;
}

void dpr_plan_free(dpr_plan *p) {
    if (!p) return;
    for (int i = 0; i < DPR_STAGE_COUNT; ++i) {
        if (p->ev.a[i]) (void)hipEventDestroy(p->ev.a[i]);
        if (p->ev.b[i]) (void)hipEventDestroy(p->ev.b[i]);
    }
    delete p;
}

int dpr_plan_get_info(const dpr_plan *p, dpr_plan_info *out) {
    if (!p || !out) return fail(DPR_ERR_INVALID_ARG, "NULL argument");
    memset(out, 0, sizeof(*out));
    const FwdLayout f = fwd_layout(p);
    out->items = (int64_t)p->sz.items;
    out->pairs = (int64_t)p->pairs;
    out->tiles = (int64_t)p->sz.tiles;
    out->pixels = (int64_t)p->sz.pixels;
    out->chunks = (int64_t)p->sz.chunks;
    out->plan_ws_bytes = (int64_t)p->lay.total;
    out->fwd_ws_bytes = (int64_t)f.total;
    out->bwd_ws_bytes = (int64_t)bwd_layout(p).total;
    out->rec_off = (int64_t)p->lay.rec.off;
    out->key_off = (int64_t)p->lay.keys.off;
    out->order_off = (int64_t)p->lay.vals.off;
    out->rect_off = (int64_t)p->lay.rect.off;
    out->range_off = (int64_t)p->lay.tile_base.off;
    out->pairs_off = (int64_t)f.pairs.off;
    out->nlast_off = f.st.nlast.bytes ? (int64_t)f.st.nlast.off : -1;
    out->stats_off = f.stats.bytes ? (int64_t)f.stats.off : -1;
    out->tile_size = kTile;
    out->chunk_items = kChunkItems;
    return DPR_OK;
}

int dpr_stage_times(const dpr_plan *p, float *ms, int32_t cap) {
    if (!p || !ms || cap < DPR_STAGE_COUNT) return fail(DPR_ERR_INVALID_ARG, "bad arguments");
    for (int i = 0; i < DPR_STAGE_COUNT; ++i) ms[i] = -1.f;
    if (!p->timing) return fail(DPR_ERR_STATE, "plan was created without DPR_FLAG_TIMING");
    for (int i = 0; i < DPR_STAGE_COUNT; ++i) {
        if (!p->ev.ran[i]) continue;
        HIP_TRY(hipEventSynchronize(p->ev.b[i]));
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, p->ev.a[i], p->ev.b[i]));
        ms[i] = t;
    }
    return DPR_OK;
}

int dpr_render_forward_1(const dpr_scene *scene, const dpr_camera *cam, const dpr_params *params, float *image,
                         float *trans, void *ws, size_t ws_bytes, size_t *ws_needed, void *stream) {
    g_err.clear();
    if (!scene || !cam) return fail(DPR_ERR_INVALID_ARG, "scene or camera is NULL");
    dpr_view view;
    memset(&view, 0, sizeof(view));
    view.scene = 0;
    view.cam = *cam;
    view.image = image;
    view.trans = trans;
    const size_t pb = dpr_plan_ws_bytes(scene, 1, &view, 1);
    if (pb == 0) {
        int rc = check_params(params);
        if (rc) return rc;
        Sizes s;
        return check_inputs(scene, 1, &view, 1, &s);
    }
    const size_t pb_al = (size_t)align_up(pb);
    if (ws_needed) *ws_needed = pb_al;
    if (!ws || ws_bytes < pb_al) return fail(DPR_ERR_WORKSPACE, "workspace needs at least %zu bytes", pb_al);
    dpr_plan *p = nullptr;
    int rc = dpr_plan_forward(scene, 1, &view, 1, params, ws, pb, stream, &p);
    if (rc) return rc;
    const size_t need = pb_al + dpr_workspace_bytes(p);
    if (ws_needed) *ws_needed = need;
    if (ws_bytes < need) {
        dpr_plan_free(p);
        return fail(DPR_ERR_WORKSPACE, "workspace needs %zu bytes", need);
    }
    rc = dpr_render_forward(p, static_cast<uint8_t *>(ws) + pb_al, ws_bytes - pb_al, stream);
    dpr_plan_free(p);
    return rc;
}

size_t dpr_loss_ws_bytes(int32_t n_images, const int32_t *widths, const int32_t *heights) {
    LossLayout L;
    if (loss_layout(n_images, widths, heights, &L) != DPR_OK) return 0;
    return (size_t)L.total;
}

int dpr_loss_l2_tv(int32_t n_images, const float *const *render, const float *const *target, const int32_t *widths,
                   const int32_t *heights, float lambda, float *const *dL_drender, double *loss, void *ws,
                   size_t ws_bytes, void *stream) {
    g_err.clear();
    LossLayout lay;
    int rc = loss_layout(n_images, widths, heights, &lay);
    if (rc) return rc;
    if (!render || !target || !dL_drender || !loss)
        return fail(DPR_ERR_INVALID_ARG, "render / target / dL_drender / loss is NULL");
    if (!(lambda >= 0.f) || !std::isfinite(lambda)) return fail(DPR_ERR_INVALID_ARG, "lambda must be finite, >= 0");
    if (!ws || ws_bytes < lay.total)
        return fail(DPR_ERR_WORKSPACE, "loss workspace needs %llu bytes, got %llu", (unsigned long long)lay.total,
                    (unsigned long long)ws_bytes);
    std::vector<LossImage> tab((size_t)n_images);
    for (int32_t v = 0; v < n_images; ++v) {
        if (!render[v] || !target[v] || !dL_drender[v])
            return fail(DPR_ERR_INVALID_ARG, "image %d: NULL pointer", v);
        if (dL_drender[v] == render[v] || dL_drender[v] == target[v])
            return fail(DPR_ERR_INVALID_ARG, "image %d: dL_drender aliases an input", v);
        tab[v].render = render[v];
        tab[v].target = target[v];
        tab[v].grad = dL_drender[v];
        tab[v].width = widths[v];
        tab[v].height = heights[v];
    }
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *w = static_cast<uint8_t *>(ws);
    HIP_TRY(launch_loss(tab.data(), n_images, lambda, reinterpret_cast<float *>(w + lay.partial.off), loss, st));
    return DPR_OK;
}

size_t dpr_knn_ws_bytes(int64_t m, int32_t K) {
    if (check_hybrid_args(m, 0, K) != DPR_OK) return 0;
    return (size_t)hy_layout((uint64_t)m, K, 0, false).total_bytes;
}

int dpr_knn(int64_t m, const float *xyz, int32_t K, int32_t *idx, float *d2, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    int rc = check_hybrid_args(m, 0, K);
    if (rc) return rc;
    if (!xyz || !idx || !d2) return fail(DPR_ERR_INVALID_ARG, "xyz / idx / d2 is NULL");
    const HyLayout h = hy_layout((uint64_t)m, K, 0, false);
    if (!ws || ws_bytes < h.total_bytes)
        return fail(DPR_ERR_WORKSPACE, "workspace needs %llu bytes", (unsigned long long)h.total_bytes);
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    HyScratch sc = hy_scratch(static_cast<uint8_t *>(ws), h);
    HIP_TRY(launch_knn(xyz, (uint32_t)m, K, idx, d2, sc, static_cast<hipStream_t>(stream)));
    return DPR_OK;
}

size_t dpr_hybrid_ws_bytes(int64_t n, int32_t sh_degree, int32_t K) {
    if (check_hybrid_args(n, sh_degree, K) != DPR_OK) return 0;
    const int k3 = 3 * (sh_degree + 1) * (sh_degree + 1);
    return (size_t)hy_layout((uint64_t)n, K, k3, true).total_bytes;
}

int dpr_voxel_reduce(int64_t n, int32_t sh_degree, const float *xyz, const float *sh, const float *opacity,
                     const float *radius, int32_t N, float *out_xyz, float *out_sh, float *out_opacity,
                     float *out_radius, int64_t *out_count, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    int rc = check_hybrid_args(n, sh_degree, 1);
    if (rc) return rc;
    if (N < 1 || N > 1024) return fail(DPR_ERR_INVALID_ARG, "N must be in [1, 1024]");
    if (!xyz || !sh || !opacity || !radius || !out_xyz || !out_sh || !out_opacity || !out_radius || !out_count)
        return fail(DPR_ERR_INVALID_ARG, "NULL array");
    const int k3 = 3 * (sh_degree + 1) * (sh_degree + 1);
    const HyLayout h = hy_layout((uint64_t)n, 1, k3, true);
    if (!ws || ws_bytes < h.total_bytes)
        return fail(DPR_ERR_WORKSPACE, "workspace needs %llu bytes", (unsigned long long)h.total_bytes);
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    HyScratch sc = hy_scratch(static_cast<uint8_t *>(ws), h);
    uint64_t m = 0;
    HIP_TRY(launch_voxel_reduce(xyz, sh, opacity, radius, (uint32_t)n, k3, (uint32_t)N, out_xyz, out_sh,
                                out_opacity, out_radius, sc, &m, static_cast<hipStream_t>(stream)));
    *out_count = (int64_t)m;
    return DPR_OK;
}

int dpr_hybrid_update(int64_t n, int32_t sh_degree, const float *xyz, const float *sh, const float *opacity,
                      const float *radius, int32_t N, int32_t K, float eps, float *out_xyz, float *out_sh,
                      float *out_opacity, float *out_radius, int64_t *out_counts, void *ws, size_t ws_bytes,
                      void *stream) {
    g_err.clear();
    int rc = check_hybrid_args(n, sh_degree, K);
    if (rc) return rc;
    if (N < 1 || N > 1024) return fail(DPR_ERR_INVALID_ARG, "N must be in [1, 1024]");
    if (!(eps >= 0.f) || !std::isfinite(eps)) return fail(DPR_ERR_INVALID_ARG, "eps must be finite, >= 0");
    if (!xyz || !sh || !opacity || !radius || !out_xyz || !out_sh || !out_opacity || !out_radius || !out_counts)
        return fail(DPR_ERR_INVALID_ARG, "NULL array");
    const int k3 = 3 * (sh_degree + 1) * (sh_degree + 1);
    const HyLayout h = hy_layout((uint64_t)n, K, k3, true);
    if (!ws || ws_bytes < h.total_bytes)
        return fail(DPR_ERR_WORKSPACE, "workspace needs %llu bytes", (unsigned long long)h.total_bytes);
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *w = static_cast<uint8_t *>(ws);
    HyScratch sc = hy_scratch(w, h);
    float *red = reinterpret_cast<float *>(w + h.red.off);
    float *rxyz = red, *rsh = red + 3 * (size_t)n, *rop = rsh + (size_t)k3 * n, *rrad = rop + n;
    uint64_t m = 0, kept = 0, count = 0;
    HIP_TRY(launch_voxel_reduce(xyz, sh, opacity, radius, (uint32_t)n, k3, (uint32_t)N, rxyz, rsh, rop, rrad, sc,
                                &m, st));
    HIP_TRY(launch_filter_generate(rxyz, rsh, rop, rrad, (uint32_t)m, k3, K, eps, out_xyz, out_sh, out_opacity,
                                   out_radius, sc, &kept, &count, st));
    out_counts[0] = (int64_t)m;
    out_counts[1] = (int64_t)kept;
    out_counts[2] = (int64_t)count;
    return DPR_OK;
}

size_t dpr_hull_ws_bytes(int64_t n, int32_t n_cams, const dpr_camera *cams) {
    if (n < 0 || n > (int64_t)0x7FFFFFFF || n_cams < 1 || n_cams > kHullMaxCams || !cams) return 0;
    std::vector<HullCam> tab((size_t)n_cams);
    for (int32_t i = 0; i < n_cams; ++i) {
        if (cams[i].width < 1 || cams[i].width > kLimitDim || cams[i].height < 1 || cams[i].height > kLimitDim)
            return 0;
        tab[(size_t)i].width = cams[i].width;
        tab[(size_t)i].height = cams[i].height;
    }
    return (size_t)hull_layout((uint64_t)n, n_cams, tab.data()).bytes;
}

int dpr_hull_sample(int32_t n_cams, const dpr_camera *cams, const dpr_mask *masks, const float *lo, const float *hi,
                    uint64_t seed, int64_t n, float *out_xyz, int64_t capacity, int64_t *out_count, void *ws,
                    size_t ws_bytes, void *stream) {
    g_err.clear();
    if (n < 0 || n > (int64_t)0x7FFFFFFF) return fail(DPR_ERR_INVALID_ARG, "n must be in [0, 2^31 - 1]");
    if (capacity < 0) return fail(DPR_ERR_INVALID_ARG, "capacity must be >= 0");
    if (!lo || !hi || !out_count || (capacity > 0 && !out_xyz)) return fail(DPR_ERR_INVALID_ARG, "NULL argument");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(lo[d]) || !std::isfinite(hi[d]) || !(lo[d] < hi[d]))
            return fail(DPR_ERR_INVALID_ARG, "the box needs finite lo < hi on every axis");
    std::vector<HullCam> tab;
    int rc = hull_table(n_cams, cams, masks, tab);
    if (rc) return rc;
    const HullLayout L = hull_layout((uint64_t)n, n_cams, tab.data());
    if (!ws || ws_bytes < L.bytes) return fail(DPR_ERR_WORKSPACE, "workspace needs %llu bytes", (unsigned long long)L.bytes);
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    HullJob job = {};
    job.n_cams = n_cams;
    job.cams = tab.data();
    job.n = (uint64_t)n;
    job.seed = seed;
    for (int d = 0; d < 3; ++d) { job.lo[d] = lo[d]; job.hi[d] = hi[d]; }
    job.out_xyz = out_xyz;
    job.capacity = (uint64_t)capacity;
    job.sync = true;
    uint64_t kept = 0;
    HIP_TRY(launch_hull(job, static_cast<uint8_t *>(ws), &kept, static_cast<hipStream_t>(stream)));
    *out_count = (int64_t)kept;
    return DPR_OK;
}

int dpr_consistency(int64_t n, const float *xyz, int32_t n_cams, const dpr_camera *cams, const dpr_mask *masks,
                    uint8_t *keep, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (n < 0 || n > (int64_t)0x7FFFFFFF) return fail(DPR_ERR_INVALID_ARG, "n must be in [0, 2^31 - 1]");
    if (n > 0 && (!xyz || !keep)) return fail(DPR_ERR_INVALID_ARG, "xyz or keep is NULL");
    std::vector<HullCam> tab;
    int rc = hull_table(n_cams, cams, masks, tab);
    if (rc) return rc;
    const HullLayout L = hull_layout((uint64_t)n, n_cams, tab.data());
    if (!ws || ws_bytes < L.bytes) return fail(DPR_ERR_WORKSPACE, "workspace needs %llu bytes", (unsigned long long)L.bytes);
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    HullJob job = {};
    job.n_cams = n_cams;
    job.cams = tab.data();
    job.n = (uint64_t)n;
    job.xyz = xyz;
    job.keep = keep;
    job.sync = false;
    uint64_t kept = 0;
    HIP_TRY(launch_hull(job, static_cast<uint8_t *>(ws), &kept, static_cast<hipStream_t>(stream)));
    return DPR_OK;
}

int dpr_consistency_filter(int64_t n, int32_t sh_degree, const float *xyz, const float *sh, const float *opacity,
                           const float *radius, int32_t n_cams, const dpr_camera *cams, const dpr_mask *masks,
                           float *out_xyz, float *out_sh, float *out_opacity, float *out_radius, int64_t *out_count,
                           void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (n < 0 || n > (int64_t)0x7FFFFFFF) return fail(DPR_ERR_INVALID_ARG, "n must be in [0, 2^31 - 1]");
    if (sh_degree < 0 || sh_degree > 3) return fail(DPR_ERR_INVALID_ARG, "sh_degree must be in [0, 3]");
    if (!out_count || (n > 0 && (!xyz || !sh || !opacity || !radius || !out_xyz || !out_sh || !out_opacity ||
                                 !out_radius)))
        return fail(DPR_ERR_INVALID_ARG, "NULL array");
    std::vector<HullCam> tab;
    int rc = hull_table(n_cams, cams, masks, tab);
    if (rc) return rc;
    const HullLayout L = hull_layout((uint64_t)n, n_cams, tab.data());
    if (!ws || ws_bytes < L.bytes) return fail(DPR_ERR_WORKSPACE, "workspace needs %llu bytes", (unsigned long long)L.bytes);
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    HullJob job = {};
    job.n_cams = n_cams;
    job.cams = tab.data();
    job.n = (uint64_t)n;
    job.xyz = xyz;
    job.out_xyz = out_xyz;
    job.capacity = (uint64_t)n;
    job.sh = sh; job.opacity = opacity; job.radius = radius;
    job.out_sh = out_sh; job.out_opacity = out_opacity; job.out_radius = out_radius;
    job.k3 = 3 * (sh_degree + 1) * (sh_degree + 1);
    job.sync = true;
    uint64_t kept = 0;
    HIP_TRY(launch_hull(job, static_cast<uint8_t *>(ws), &kept, static_cast<hipStream_t>(stream)));
    *out_count = (int64_t)kept;
    return DPR_OK;
}

size_t dpr_chamfer_ws_bytes(int64_t n1, int64_t n2) {
    if (n1 < 1 || n2 < 1 || n1 > (int64_t)0x7FFFFFFF || n2 > (int64_t)0x7FFFFFFF) return 0;
    return (size_t)chamfer_layout((uint64_t)n1, (uint64_t)n2).bytes;
}

int dpr_chamfer(int64_t n1, const float *s1, int64_t n2, const float *s2, double *cd, float *grad2, int32_t *nn12,
                int32_t *nn21, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (n1 < 1 || n2 < 1 || n1 > (int64_t)0x7FFFFFFF || n2 > (int64_t)0x7FFFFFFF)
        return fail(DPR_ERR_INVALID_ARG, "point counts must be in [1, 2^31 - 1]");
    if (!s1 || !s2) return fail(DPR_ERR_INVALID_ARG, "s1 or s2 is NULL");
    const ChamferLayout L = chamfer_layout((uint64_t)n1, (uint64_t)n2);
    if (!ws || ws_bytes < L.bytes) return fail(DPR_ERR_WORKSPACE, "workspace needs %llu bytes", (unsigned long long)L.bytes);
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    HIP_TRY(launch_chamfer((uint32_t)n1, s1, (uint32_t)n2, s2, cd, grad2, nn12, nn21, static_cast<uint8_t *>(ws),
                           static_cast<hipStream_t>(stream)));
    return DPR_OK;
}

int dpr_topk_sh(int64_t n1, const float *s1, const float *sh1, int64_t n2, const float *s2, int32_t sh_degree,
                int32_t K, float *out_sh2, int32_t *idx, void *stream) {
    g_err.clear();
    if (n1 < 1 || n2 < 0 || n1 > (int64_t)0x7FFFFFFF || n2 > (int64_t)0x7FFFFFFF)
        return fail(DPR_ERR_INVALID_ARG, "point counts must be n1 in [1, 2^31 - 1], n2 in [0, 2^31 - 1]");
    if (sh_degree < 0 || sh_degree > 3) return fail(DPR_ERR_INVALID_ARG, "sh_degree must be in [0, 3]");
    if (K < 1 || K > kTopkMax) return fail(DPR_ERR_INVALID_ARG, "K must be in [1, %d]", kTopkMax);
    if (!s1 || !sh1 || (n2 > 0 && (!s2 || !out_sh2))) return fail(DPR_ERR_INVALID_ARG, "NULL array");
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    HIP_TRY(launch_topk_sh((uint32_t)n1, s1, sh1, (uint32_t)n2, s2, 3 * (sh_degree + 1) * (sh_degree + 1), K, out_sh2,
                           idx, static_cast<hipStream_t>(stream)));
    return DPR_OK;
}

int dpr_adam_step(int64_t n, float *p, const float *g, float *m, float *v, int32_t t, float lr, float beta1,
                  float beta2, float eps, void *stream) {
    g_err.clear();
    if (n < 0 || n > (int64_t)0xFFFFFFFF) return fail(DPR_ERR_INVALID_ARG, "n must be in [0, 2^32 - 1]");
    if (t < 1) return fail(DPR_ERR_INVALID_ARG, "t must be >= 1");
    if (!(lr >= 0.f) || !std::isfinite(lr) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f) || !std::isfinite(eps))
        return fail(DPR_ERR_INVALID_ARG, "need lr >= 0, 0 <= beta1, beta2 < 1, eps > 0 (all finite)");
    if (n > 0 && (!p || !g || !m || !v)) return fail(DPR_ERR_INVALID_ARG, "NULL array");
    if (fault_injected("launch")) return fail(DPR_ERR_HIP, "injected launch failure (DPR_FAULT=launch)");
    HIP_TRY(launch_adam((uint32_t)n, p, g, m, v, t, lr, beta1, beta2, eps, static_cast<hipStream_t>(stream)));
    return DPR_OK;
}

}  // extern "C"
