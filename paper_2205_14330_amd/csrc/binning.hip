// Screen-tile binning of the depth-sorted splats (only points near a pixel
// with non-negligible opacity are considered: end of Sec. 3.2).
//
// Instead of sorting (tile, depth) pairs, the depth-sorted item list of each
// view is cut into chunks of kChunkItems consecutive items and binned with a
// stable counting scatter:
//   count  : per chunk, an LDS histogram of how many of its splats touch each
//            tile, written as one coalesced row cnt[view][chunk][tile];
//   colscan: per tile, an exclusive scan down the chunk column (in place) and
//            the column total; an exclusive scan of the totals (tile_base)
//            gives every tile's list range [tile_base[t], tile_base[t + 1]);
//   emit   : per chunk, one wave walks the items in depth order and appends
//            each to every tile it touches through an LDS cursor per tile,
//            starting at tile_base[t] + cnt[chunk][t].
// Within a tile the lists come out in chunk order, and inside a chunk in item
// order, i.e. exactly ascending (depth, point index): the front-to-back order
// of Eq. (6)-(7).  The only pass over all pairs is the 4-byte write of emit.
#include "dpr_internal.h"

namespace dpr {

constexpr int kCountThreads = 256;
constexpr int kEmitLanes = 64;
constexpr int kColThreads = 256;

struct ChunkInfo {
    uint32_t c;          // chunk index within the view
    uint32_t beg, end;   // sorted-item range
    uint32_t ntiles;
    int32_t tiles_x;
    uint32_t tile_off;
    uint64_t row;        // first count entry of this chunk's row
};

__device__ __forceinline__ ChunkInfo chunk_info(const Tables &tb) {
    const int v = find_segment(tb.chunk_start, tb.n_views, blockIdx.x);
    const ViewDesc &vd = tb.views[v];
    ChunkInfo ci;
    ci.c = blockIdx.x - vd.chunk_off;
    ci.beg = vd.item_off + ci.c * (uint32_t)kChunkItems;
    ci.end = min(ci.beg + (uint32_t)kChunkItems, vd.item_off + (uint32_t)vd.n);
    ci.tiles_x = vd.tiles_x;
    ci.ntiles = (uint32_t)vd.tiles_x * (uint32_t)vd.tiles_y;
    ci.tile_off = vd.tile_off;
    ci.row = vd.cnt_off + (uint64_t)ci.c * ci.ntiles;
    return ci;
}

__global__ __launch_bounds__(kCountThreads) void k_tile_count(Tables tb, const uint32_t *order, const uint2 *rect,
                                                               const SplatRec *rec, float lambda, uint32_t *cnt,
                                                               uint32_t band_tiles) {
    extern __shared__ uint32_t s_h[];
    const ChunkInfo ci = chunk_info(tb);
    for (uint32_t band = 0; band < ci.ntiles; band += band_tiles) {
        const uint32_t bend = min(band + band_tiles, ci.ntiles);
        for (uint32_t t = threadIdx.x; t < bend - band; t += kCountThreads) s_h[t] = 0;
        __syncthreads();
        for (uint32_t s = ci.beg + threadIdx.x; s < ci.end; s += kCountThreads) {
            const uint32_t g = order[s];
            const uint2 rc = rect[g];
            const uint32_t x0 = rc.x & 0xFFFFu, y0 = rc.x >> 16, x1 = rc.y & 0xFFFFu, y1 = rc.y >> 16;
            if (x1 <= x0 || y1 <= y0) continue;
            const float4 r0 = reinterpret_cast<const float4 *>(rec + g)[0];
            const float thr = reinterpret_cast<const float4 *>(rec + g)[1].x + lambda;
            for (uint32_t ty = y0; ty < y1; ++ty) {
                const uint32_t rowb = ty * (uint32_t)ci.tiles_x;
                if (rowb + x1 <= band || rowb + x0 >= bend) continue;
                for (uint32_t tx = x0; tx < x1; ++tx) {
                    const uint32_t t = rowb + tx;
                    if (t >= band && t < bend && splat_touches_tile(r0.x, r0.y, r0.z, r0.w, thr, tx, ty))
                        atomicAdd(&s_h[t - band], 1u);
                }
            }
        }
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < bend - band; t += kCountThreads) cnt[ci.row + band + t] = s_h[t];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// column scan: grid (tiles / 256, segments); segment s covers chunks
// [s * kSegChunks, (s + 1) * kSegChunks) of every tile column.
// ---------------------------------------------------------------------------
struct ColCtx {
    bool ok;
    uint32_t t, ntiles, nchunks, nseg;
    uint64_t cnt_off, seg_off;
    uint32_t gtile;
};

__device__ __forceinline__ ColCtx col_ctx(const Tables &tb) {
    ColCtx c;
    c.gtile = blockIdx.x * kColThreads + threadIdx.x;
    c.ok = c.gtile < tb.total_tiles;
    if (!c.ok) return c;
    const int v = find_segment(tb.tile_start, tb.n_views, c.gtile);
    const ViewDesc &vd = tb.views[v];
    c.t = c.gtile - vd.tile_off;
    c.ntiles = (uint32_t)vd.tiles_x * (uint32_t)vd.tiles_y;
    c.nchunks = vd.nchunks;
    c.nseg = (vd.nchunks + kSegChunks - 1) / kSegChunks;
    c.cnt_off = vd.cnt_off;
    c.seg_off = vd.seg_off;
    return c;
}

__global__ __launch_bounds__(kColThreads) void k_col_segsum(Tables tb, const uint32_t *cnt, uint32_t *segs) {
    const ColCtx c = col_ctx(tb);
    const uint32_t s = blockIdx.y;
    if (!c.ok || s >= c.nseg) return;
    const uint32_t c0 = s * kSegChunks, c1 = min(c0 + (uint32_t)kSegChunks, c.nchunks);
    uint32_t sum = 0;
#pragma unroll 4
    for (uint32_t k = c0; k < c1; ++k) sum += cnt[c.cnt_off + (uint64_t)k * c.ntiles + c.t];
    segs[c.seg_off + (uint64_t)s * c.ntiles + c.t] = sum;
}

// Also counts the block's tiles per order bucket (bucket_cnt[block][kOrderBuckets]).
__global__ __launch_bounds__(kColThreads) void k_col_segscan(Tables tb, uint32_t *segs, uint32_t *tile_total,
                                                             uint32_t *bucket_cnt) {
    __shared__ uint32_t s_b[kOrderBuckets];
    if (threadIdx.x < (uint32_t)kOrderBuckets) s_b[threadIdx.x] = 0;
    __syncthreads();
    const ColCtx c = col_ctx(tb);
    if (c.ok) {
        uint32_t run = 0;
        for (uint32_t s = 0; s < c.nseg; ++s) {
            uint32_t *p = segs + c.seg_off + (uint64_t)s * c.ntiles + c.t;
            const uint32_t v = *p;
            *p = run;
            run += v;
        }
        tile_total[c.gtile] = run;
        atomicAdd(&s_b[order_bucket(run)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < (uint32_t)kOrderBuckets)
        bucket_cnt[(uint64_t)blockIdx.x * kOrderBuckets + threadIdx.x] = s_b[threadIdx.x];
}

uint64_t order_count_blocks(uint64_t tiles) { return (tiles + kColThreads - 1) / kColThreads; }

// Same blocks of kColThreads tiles as k_col_segscan.  Bucket b starts after
// every tile of the longer buckets and after bucket b's tiles of the earlier
// blocks; inside a block the tiles of a bucket take its slots by LDS atomics.
__global__ __launch_bounds__(kColThreads) void k_tile_order(const uint32_t *len, uint32_t n, const uint32_t *bucket_cnt,
                                                            uint32_t nblk, uint32_t *order) {
    __shared__ uint32_t s_tot[kOrderBuckets], s_before[kOrderBuckets], s_base[kOrderBuckets];
    const uint32_t tid = threadIdx.x;
    if (tid < (uint32_t)kOrderBuckets) {
        uint32_t tot = 0, before = 0;
#pragma unroll 8
        for (uint32_t i = 0; i < nblk; ++i) {
            const uint32_t v = bucket_cnt[(uint64_t)i * kOrderBuckets + tid];
            tot += v;
            before += i < blockIdx.x ? v : 0u;
        }
        s_tot[tid] = tot;
        s_before[tid] = before;
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int b = 0; b < kOrderBuckets; ++b) {
            s_base[b] = run + s_before[b];
            run += s_tot[b];
        }
    }
    __syncthreads();
    const uint32_t t = blockIdx.x * kColThreads + tid;
    if (t < n) order[atomicAdd(&s_base[order_bucket(len[t])], 1u)] = t;
}

hipError_t launch_tile_order(const uint32_t *len, uint32_t n, const uint32_t *bucket_cnt, uint32_t *order,
                             hipStream_t st) {
    if (n == 0) return hipSuccess;
    const uint32_t nblk = (uint32_t)order_count_blocks(n);
    hipLaunchKernelGGL(k_tile_order, dim3(nblk), dim3(kColThreads), 0, st, len, n, bucket_cnt, nblk, order);
    return hipGetLastError();
}

__global__ __launch_bounds__(kColThreads) void k_col_down(Tables tb, uint32_t *cnt, const uint32_t *segs) {
    const ColCtx c = col_ctx(tb);
    const uint32_t s = blockIdx.y;
    if (!c.ok || s >= c.nseg) return;
    const uint32_t c0 = s * kSegChunks, c1 = min(c0 + (uint32_t)kSegChunks, c.nchunks);
    uint32_t run = segs[c.seg_off + (uint64_t)s * c.ntiles + c.t];
    for (uint32_t k = c0; k < c1; ++k) {
        uint32_t *p = cnt + c.cnt_off + (uint64_t)k * c.ntiles + c.t;
        const uint32_t v = *p;
        *p = run;
        run += v;
    }
}

hipError_t launch_tile_colscan(const Tables &tb, uint32_t *cnt, uint32_t *segs, uint32_t *tile_total,
                               uint32_t *bucket_cnt, hipStream_t st) {
    if (tb.total_tiles == 0) return hipSuccess;
    const uint32_t bx = (tb.total_tiles + kColThreads - 1) / kColThreads;
    const uint32_t ns = tb.max_view_segs > 0 ? tb.max_view_segs : 1;
    hipLaunchKernelGGL(k_col_segsum, dim3(bx, ns), dim3(kColThreads), 0, st, tb, cnt, segs);
    hipLaunchKernelGGL(k_col_segscan, dim3(bx), dim3(kColThreads), 0, st, tb, segs, tile_total, bucket_cnt);
    hipLaunchKernelGGL(k_col_down, dim3(bx, ns), dim3(kColThreads), 0, st, tb, cnt, segs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// emit
// ---------------------------------------------------------------------------
struct EmitItem {
    uint32_t g, x0, y0, w, n;
    float inv_w;
    float px, py, a, b, thr;
};

// The items of a batch of 64 are staged in LDS, one per lane, and each is read
// back as an LDS broadcast: its fields then sit in VGPRs, and the arithmetic of
// the tile test issues at the VGPR-operand rate (an SGPR operand, as left by a
// readlane, costs about twice as much per instruction).
struct EmitStage {
    float4 shape;      // px, py, a, b
    float4 misc;       // thr, 1 / w, g (bits), x0 | y0 << 16 (bits)
    uint2 wn;          // w, n
};

__device__ __forceinline__ void stage_item(EmitStage &st, uint32_t g, uint32_t ra, uint32_t rb, const float4 &shape,
                                           float thr) {
    const uint32_t x0 = ra & 0xFFFFu, y0 = ra >> 16;
    const uint32_t x1 = rb & 0xFFFFu, y1 = rb >> 16;
    const uint32_t w = x1 > x0 ? x1 - x0 : 0u;
    const uint32_t h = y1 > y0 ? y1 - y0 : 0u;
    st.shape = shape;
    st.misc = make_float4(thr, w ? __builtin_amdgcn_rcpf((float)w) : 0.f, __uint_as_float(g), __uint_as_float(ra));
    st.wn = make_uint2(w, w * h);
}

__device__ __forceinline__ EmitItem emit_item(const EmitStage *stage, uint32_t j) {
    const EmitStage &st = stage[j];
    const float4 shape = st.shape, misc = st.misc;
    const uint2 wn = st.wn;
    EmitItem it;
    it.px = shape.x;
    it.py = shape.y;
    it.a = shape.z;
    it.b = shape.w;
    it.thr = misc.x;
    it.inv_w = misc.y;
    it.g = __float_as_uint(misc.z);
    const uint32_t ra = __float_as_uint(misc.w);
    it.x0 = ra & 0xFFFFu;
    it.y0 = ra >> 16;
    it.w = wn.x;
    it.n = wn.y;
    return it;
}

// Appends one item to all its tiles (any rectangle size); cell k of the
// rectangle is row floor((k + 0.5) / w), exact for k < 2^20 and w <= 1024.
__device__ __forceinline__ void emit_one(const EmitItem &it, uint32_t lane, uint32_t tiles_x, uint32_t band,
                                         uint32_t bend, uint32_t *s_pos, uint32_t *pairs) {
    for (uint32_t k = lane; k < it.n; k += kEmitLanes) {
        const uint32_t r = (uint32_t)(((float)k + 0.5f) * it.inv_w);
        const uint32_t cx = it.x0 + k - r * it.w, cy = it.y0 + r;
        const uint32_t tt = cy * tiles_x + cx;
        if (tt >= band && tt < bend && splat_touches_tile(it.px, it.py, it.a, it.b, it.thr, cx, cy))
            pairs[atomicAdd(&s_pos[tt - band], 1u)] = it.g;
    }
}

// One wave per chunk.  Items are appended strictly in depth order; four items
// are interleaved so that their LDS cursor updates are in flight together
// (LDS operations of one wave complete in program order, so a tile touched by
// two of them still receives them in order).
__global__ __launch_bounds__(kEmitLanes) void k_tile_emit(Tables tb, const uint32_t *order, const uint2 *rect,
                                                           const SplatRec *rec, float lambda, const uint32_t *pre,
                                                           const uint32_t *tile_base, uint32_t *pairs,
                                                           uint32_t band_tiles) {
    extern __shared__ uint32_t s_pos[];    // [band_tiles]
    __shared__ EmitStage s_stage[kEmitLanes];
    const ChunkInfo ci = chunk_info(tb);
    const uint32_t lane = threadIdx.x;
    const uint32_t tx = (uint32_t)ci.tiles_x;
    for (uint32_t band = 0; band < ci.ntiles; band += band_tiles) {
        const uint32_t bend = min(band + band_tiles, ci.ntiles);
        const uint32_t nb_t = bend - band;
        for (uint32_t t = lane; t < nb_t; t += kEmitLanes)
            s_pos[t] = tile_base[ci.tile_off + band + t] + pre[ci.row + band + t];
        __syncthreads();
        for (uint32_t s0 = ci.beg; s0 < ci.end; s0 += kEmitLanes) {
            const uint32_t my = s0 + lane;
            uint32_t g = 0;
            uint2 rc = make_uint2(0u, 0u);
            float4 shape = make_float4(0.f, 0.f, 0.f, 0.f);
            float thr = -1.f;
            if (my < ci.end) {
                g = order[my];
                rc = rect[g];
                shape = reinterpret_cast<const float4 *>(rec + g)[0];
                thr = reinterpret_cast<const float4 *>(rec + g)[1].x + lambda;
            }
            __syncthreads();                 // the previous batch's broadcasts are done (one wave: cheap)
            stage_item(s_stage[lane], g, rc.x, rc.y, shape, thr);
            __syncthreads();
            const uint32_t nb = min((uint32_t)kEmitLanes, ci.end - s0);
            uint32_t j = 0;
            for (; j + 4 <= nb; j += 4) {
                EmitItem it[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) it[q] = emit_item(s_stage, j + q);
                const uint32_t nmax = max(max(it[0].n, it[1].n), max(it[2].n, it[3].n));
                if (nmax <= (uint32_t)kEmitLanes) {
                    uint32_t t[4], p[4];
                    bool on[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        on[q] = false;
                        t[q] = 0;
                        if (lane < it[q].n) {
                            const uint32_t r = (uint32_t)(((float)lane + 0.5f) * it[q].inv_w);
                            const uint32_t cx = it[q].x0 + lane - r * it[q].w, cy = it[q].y0 + r;
                            const uint32_t tt = cy * tx + cx;
                            on[q] = tt >= band && tt < bend &&
                                    splat_touches_tile(it[q].px, it[q].py, it[q].a, it[q].b, it[q].thr, cx, cy);
                            t[q] = tt - band;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (on[q]) p[q] = atomicAdd(&s_pos[t[q]], 1u);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (on[q]) pairs[p[q]] = it[q].g;
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) emit_one(it[q], lane, tx, band, bend, s_pos, pairs);
                }
            }
            for (; j < nb; ++j) emit_one(emit_item(s_stage, j), lane, tx, band, bend, s_pos, pairs);
        }
        __syncthreads();
    }
}

static uint32_t band_for(const Tables &tb) {
    return tb.max_view_tiles < (uint32_t)kBandTiles ? tb.max_view_tiles : (uint32_t)kBandTiles;
}

hipError_t launch_tile_count(const Tables &tb, uint32_t chunks, const uint32_t *order,
                             const uint2 *rect, const SplatRec *rec, float lambda, uint32_t *cnt, hipStream_t st) {
    if (chunks == 0) return hipSuccess;
    const uint32_t band = band_for(tb);
    hipLaunchKernelGGL(k_tile_count, dim3(chunks), dim3(kCountThreads), (size_t)band * 4, st, tb, order, rect, rec,
                       lambda, cnt, band);
    return hipGetLastError();
}

hipError_t launch_tile_emit(const Tables &tb, uint32_t chunks, const uint32_t *order,
                            const uint2 *rect, const SplatRec *rec, float lambda, const uint32_t *pre,
                            const uint32_t *tile_base, uint32_t *pairs, hipStream_t st) {
    if (chunks == 0) return hipSuccess;
    const uint32_t band = band_for(tb);
    hipLaunchKernelGGL(k_tile_emit, dim3(chunks), dim3(kEmitLanes), (size_t)band * 4, st, tb, order, rect, rec,
                       lambda, pre, tile_base, pairs, band);
    return hipGetLastError();
}

}  // namespace dpr
