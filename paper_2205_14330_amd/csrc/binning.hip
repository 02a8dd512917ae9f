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
//   emit   : per chunk, an LDS bitmap per tile of which of the chunk's items
//            touch it, read back in item order: each tile's run of the chunk
//            is written contiguously at tile_base[t] + cnt[chunk][t].
// Within a tile the lists come out in chunk order, and inside a chunk in item
// order, i.e. exactly ascending (depth, point index): the front-to-back order
// of Eq. (6)-(7).  The only pass over all pairs is the 4-byte write of emit.
#include "dpr_internal.h"

namespace dpr {

constexpr int kCountThreads = 256;
constexpr int kColThreads = 256;

struct ChunkInfo {
    uint32_t c;          // chunk index within the view
    uint32_t beg, end;   // sorted-item range
    uint32_t ntiles;
    int32_t tiles_x;
    uint32_t tile_off;
    uint64_t row;        // first count entry of this chunk's row
};

// Chunk of work index b (a block index, or a remapped one).
__device__ __forceinline__ ChunkInfo chunk_info(const Tables &tb, uint32_t b) {
    const int v = find_segment(tb.chunk_start, tb.n_views, b);
    const ViewDesc &vd = tb.views[v];
    ChunkInfo ci;
    ci.c = b - vd.chunk_off;
    ci.beg = vd.item_off + ci.c * (uint32_t)kChunkItems;
    ci.end = min(ci.beg + (uint32_t)kChunkItems, vd.item_off + (uint32_t)vd.n);
    ci.tiles_x = vd.tiles_x;
    ci.ntiles = (uint32_t)vd.tiles_x * (uint32_t)vd.tiles_y;
    ci.tile_off = vd.tile_off;
    ci.row = vd.cnt_off + (uint64_t)ci.c * ci.ntiles;
    return ci;
}

constexpr int kCountPer = kChunkItems / kCountThreads;    // items per count thread
static_assert(kChunkItems % kCountThreads == 0, "whole items per count thread");

// The thread's items are gathered once (ids, rectangles, then the splat
// records of the non-empty ones, each step's loads all in flight together),
// their binning records written in depth order, then binned band by band
// from registers.
__global__ __launch_bounds__(kCountThreads) void k_tile_count(Tables tb, const uint32_t *order, const uint2 *rect,
                                                               const SplatRec *rec, float lambda, uint32_t *cnt,
                                                               BinRec *bin, uint32_t band_tiles) {
    extern __shared__ uint32_t s_h[];
    const ChunkInfo ci = chunk_info(tb, blockIdx.x);
    uint32_t g[kCountPer];
    uint2 rc[kCountPer];
    float4 r0[kCountPer];
    float thr[kCountPer];
#pragma unroll
    for (int k = 0; k < kCountPer; ++k) {
        const uint32_t s = ci.beg + threadIdx.x + (uint32_t)k * kCountThreads;
        g[k] = s < ci.end ? order[s] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kCountPer; ++k) {
        const uint32_t s = ci.beg + threadIdx.x + (uint32_t)k * kCountThreads;
        rc[k] = s < ci.end ? rect[g[k]] : make_uint2(0u, 0u);     // outside the chunk: an empty rectangle
    }
#pragma unroll
    for (int k = 0; k < kCountPer; ++k) {
        r0[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        thr[k] = 0.f;
        if ((rc[k].y & 0xFFFFu) > (rc[k].x & 0xFFFFu) && (rc[k].y >> 16) > (rc[k].x >> 16)) {
            r0[k] = reinterpret_cast<const float4 *>(rec + g[k])[0];
            thr[k] = reinterpret_cast<const float4 *>(rec + g[k])[1].x + lambda;
        }
    }
#pragma unroll
    for (int k = 0; k < kCountPer; ++k) {
        const uint32_t s = ci.beg + threadIdx.x + (uint32_t)k * kCountThreads;
        if (s < ci.end) {
            uint4 *dst = reinterpret_cast<uint4 *>(bin + s);
            dst[0] = make_uint4(rc[k].x, rc[k].y, g[k], __float_as_uint(thr[k]));
            dst[1] = make_uint4(__float_as_uint(r0[k].x), __float_as_uint(r0[k].y), __float_as_uint(r0[k].z),
                                __float_as_uint(r0[k].w));
        }
    }
    for (uint32_t band = 0; band < ci.ntiles; band += band_tiles) {
        const uint32_t bend = min(band + band_tiles, ci.ntiles);
        for (uint32_t t = threadIdx.x; t < bend - band; t += kCountThreads) s_h[t] = 0;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kCountPer; ++k) {
            const uint32_t x0 = rc[k].x & 0xFFFFu, y0 = rc[k].x >> 16, x1 = rc[k].y & 0xFFFFu, y1 = rc[k].y >> 16;
            for (uint32_t ty = y0; ty < y1; ++ty) {
                const uint32_t rowb = ty * (uint32_t)ci.tiles_x;
                if (rowb + x1 <= band || rowb + x0 >= bend) continue;
                for (uint32_t tx = x0; tx < x1; ++tx) {
                    const uint32_t t = rowb + tx;
                    if (t >= band && t < bend && splat_touches_tile(r0[k].x, r0[k].y, r0[k].z, r0[k].w, thr[k], tx, ty))
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

// Also counts the block's tiles per order bucket (bucket_cnt[block][kOrderBuckets])
// and sums its tiles' totals (block_sum[block]).
__global__ __launch_bounds__(kColThreads) void k_col_segscan(Tables tb, uint32_t *segs, uint32_t *tile_total,
                                                             uint32_t *bucket_cnt, uint64_t *block_sum) {
    __shared__ uint32_t s_b[kOrderBuckets];
    __shared__ uint64_t s_w[kColThreads / 64];
    if (threadIdx.x < (uint32_t)kOrderBuckets) s_b[threadIdx.x] = 0;
    __syncthreads();
    const ColCtx c = col_ctx(tb);
    uint64_t mine = 0;
    if (c.ok) {
        // 16 segment sums loaded before any is overwritten (the loads then
        // wait once per batch, not once per segment)
        uint32_t run = 0;
        for (uint32_t s0 = 0; s0 < c.nseg; s0 += 16u) {
            uint32_t *const p = segs + c.seg_off + (uint64_t)s0 * c.ntiles + c.t;
            uint32_t v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v[u] = s0 + u < c.nseg ? p[(uint64_t)u * c.ntiles] : 0u;
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (s0 + u < c.nseg) {
                    p[(uint64_t)u * c.ntiles] = run;
                    run += v[u];
                }
        }
        tile_total[c.gtile] = run;
        atomicAdd(&s_b[order_bucket(run)], 1u);
        mine = run;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) mine += __shfl_xor(mine, d, 64);
    if ((threadIdx.x & 63u) == 0) s_w[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x < (uint32_t)kOrderBuckets)
        bucket_cnt[(uint64_t)blockIdx.x * kOrderBuckets + threadIdx.x] = s_b[threadIdx.x];
    if (threadIdx.x == 0) {
        uint64_t t = 0;
#pragma unroll
        for (int w = 0; w < kColThreads / 64; ++w) t += s_w[w];
        block_sum[blockIdx.x] = t;
    }
}

uint64_t order_count_blocks(uint64_t tiles) { return (tiles + kColThreads - 1) / kColThreads; }

// The column down-sweep (grid (tile blocks, segments): segment s covers chunks
// [s kSegChunks, (s + 1) kSegChunks) of every tile column), and in the blocks
// of segment 0 also, over the same blocks of kColThreads tiles as
// k_col_segscan:
//   tile_base: the exclusive scan of the tile totals (the block's base is the
//              sum of the earlier blocks' sums; the last block writes the
//              total after the last tile and the 64-bit pair count);
//   order    : the tiles longest list first.  Bucket b starts after every tile
//              of the longer buckets and after bucket b's tiles of the earlier
//              blocks; inside a block the tiles of a bucket take its slots by
//              LDS atomics.
__global__ __launch_bounds__(kColThreads) void k_col_finish(Tables tb, uint32_t *cnt, const uint32_t *segs,
                                                            const uint32_t *tile_total, const uint64_t *block_sum,
                                                            const uint32_t *bucket_cnt, uint32_t nblk,
                                                            uint32_t *tile_base, uint32_t *order,
                                                            uint64_t *total64) {
    {
        const ColCtx c = col_ctx(tb);
        const uint32_t s = blockIdx.y;
        if (c.ok && s < c.nseg) {
            const uint32_t c0 = s * kSegChunks, c1 = min(c0 + (uint32_t)kSegChunks, c.nchunks);
            uint32_t run = segs[c.seg_off + (uint64_t)s * c.ntiles + c.t];
            // the segment's counts loaded before any is overwritten
            uint32_t *const p = cnt + c.cnt_off + (uint64_t)c0 * c.ntiles + c.t;
            uint32_t v[kSegChunks];
#pragma unroll
            for (int u = 0; u < kSegChunks; ++u) v[u] = c0 + u < c1 ? p[(uint64_t)u * c.ntiles] : 0u;
#pragma unroll
            for (int u = 0; u < kSegChunks; ++u)
                if (c0 + u < c1) {
                    p[(uint64_t)u * c.ntiles] = run;
                    run += v[u];
                }
        }
    }
    if (blockIdx.y != 0) return;
    __shared__ uint64_t s_w[kColThreads / 64];
    __shared__ uint32_t s_tot[kOrderBuckets], s_before[kOrderBuckets], s_base[kOrderBuckets];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t n = tb.total_tiles;
    const uint32_t t = blockIdx.x * kColThreads + tid;
    const uint32_t len = t < n ? tile_total[t] : 0u;
    // block base: the earlier blocks' sums
    uint64_t pre = 0;
    for (uint32_t b = tid; b < blockIdx.x; b += kColThreads) pre += block_sum[b];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) pre += __shfl_xor(pre, d, 64);
    if (lane == 0) s_w[wave] = pre;
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
    uint64_t base = 0;
#pragma unroll
    for (int w = 0; w < kColThreads / 64; ++w) base += s_w[w];
    if (tid == 0) {
        uint32_t run = 0;
        for (int b = 0; b < kOrderBuckets; ++b) {
            s_base[b] = run + s_before[b];
            run += s_tot[b];
        }
    }
    __syncthreads();                          // every thread has read s_w
    // exclusive scan of the block's lengths
    uint64_t incl = len;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(incl, d, 64);
        if (lane >= (uint32_t)d) incl += y;
    }
    if (lane == 63) s_w[wave] = incl;
    __syncthreads();
    uint64_t wbase = 0, btot = 0;
#pragma unroll
    for (int w = 0; w < kColThreads / 64; ++w) {
        const uint64_t v = s_w[w];
        wbase += (uint32_t)w < wave ? v : 0u;
        btot += v;
    }
    if (t < n) {
        tile_base[t] = (uint32_t)(base + wbase + incl - len);
        order[atomicAdd(&s_base[order_bucket(len)], 1u)] = t;
    }
    if (blockIdx.x == gridDim.x - 1 && tid == 0) {
        tile_base[n] = (uint32_t)(base + btot);
        *total64 = base + btot;
    }
}

hipError_t launch_tile_colscan(const Tables &tb, uint32_t *cnt, uint32_t *segs, uint32_t *tile_total,
                               uint32_t *bucket_cnt, uint64_t *block_sum, uint32_t *tile_base, uint32_t *order,
                               uint64_t *total64, hipStream_t st) {
    if (tb.total_tiles == 0) {
        hipError_t e = launch_fill_u32(tile_base, 0u, 1, st);
        if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<uint32_t *>(total64), 0u, 2, st);
        return e;
    }
    const uint32_t bx = (tb.total_tiles + kColThreads - 1) / kColThreads;
    const uint32_t ns = tb.max_view_segs > 0 ? tb.max_view_segs : 1;
    hipLaunchKernelGGL(k_col_segsum, dim3(bx, ns), dim3(kColThreads), 0, st, tb, cnt, segs);
    hipLaunchKernelGGL(k_col_segscan, dim3(bx), dim3(kColThreads), 0, st, tb, segs, tile_total, bucket_cnt,
                       block_sum);
    hipLaunchKernelGGL(k_col_finish, dim3(bx, ns), dim3(kColThreads), 0, st, tb, cnt, segs, tile_total, block_sum,
                       bucket_cnt, bx, tile_base, order, total64);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// emit
// ---------------------------------------------------------------------------
// One workgroup per chunk.  The chunk's items are staged in LDS, and the
// view's tiles are taken in bands: a rectangle of whole tile rows (as many as
// fit kEmitBand tiles), or of a part of one row on views wider than kEmitBand
// tiles.  Per band:
//   mark : each thread takes items (i = tid, tid + kEmitThreads, ...) and sets
//          bit i of the bitmap of every tile of the band it touches, and the
//          bit of that bitmap word in the tile's word summary (LDS atomic OR:
//          the order of the updates does not matter, a bit's place is the
//          item's place in the chunk);
//   write: each thread takes a tile and walks the non-empty words of its
//          bitmap in bit order, so the tile's segment comes out in item order,
//          stored by one lane in consecutive instructions at
//          tile_base[t] + cnt[chunk][t] (loaded while the band is marked); it
//          clears the words it reads, so the next band starts clear.
// Every (item, tile) decision is splat_touches_tile, as in the count, so each
// segment has exactly the length the count reserved.
// Block b runs on XCD b % 8 (round-robin dispatch).  The emission maps the
// blocks so that each XCD takes stripes of kEmitStripe consecutive chunks: the
// runs that consecutive chunks write into one tile list are adjacent, so most
// 128-byte lines of the lists are completed inside one XCD's L2 before they
// are written back (about half the written bytes of the identity map), while
// the stripes of all XCDs still advance through the views together (one
// contiguous range per XCD left the XCDs unevenly loaded).  A bijection of
// [0, total): the blocks past the last whole group of 8 stripes map to
// themselves.
constexpr uint32_t kEmitStripe = 16;
__device__ __forceinline__ uint32_t emit_chunk_of_block(uint32_t b, uint32_t total) {
    const uint32_t full = total / (8u * kEmitStripe) * (8u * kEmitStripe);
    if (b >= full) return b;
    const uint32_t x = b & 7u, i = b >> 3;
    return ((i / kEmitStripe) * 8u + x) * kEmitStripe + i % kEmitStripe;
}

constexpr int kEmitThreads = 512;
constexpr int kEmitBand = 512;                 // tiles per band (at most)
constexpr int kEmitWords = kChunkItems / 32;   // bitmap words per tile
constexpr int kEmitTilesPerThread = (kEmitBand + kEmitThreads - 1) / kEmitThreads;
static_assert(kChunkItems % 32 == 0 && kEmitWords <= 32, "whole bitmap words, one summary word");
static_assert(kEmitThreads == kChunkItems, "one item per emission thread");

__global__ __launch_bounds__(kEmitThreads) void k_tile_emit(Tables tb, const BinRec *bin, const uint32_t *pre,
                                                             const uint32_t *tile_base, uint32_t *pairs,
                                                             uint32_t *zero4, uint32_t pair_cap) {
    // word w of band tile b at s_bits[w * kEmitBand + b]: the write phase's
    // lanes (consecutive tiles) read consecutive words
    __shared__ uint32_t s_bits[kEmitWords * kEmitBand];
    __shared__ uint32_t s_sum[kEmitBand];
    __shared__ uint32_t s_g[kChunkItems];
    if (tile_base[tb.total_tiles] > pair_cap) return;     // the pair lists do not fit the workspace
    const ChunkInfo ci = chunk_info(tb, emit_chunk_of_block(blockIdx.x, gridDim.x));
    const uint32_t tid = threadIdx.x;
    const uint32_t n = ci.end - ci.beg;
    if (blockIdx.x == 0 && tid < 4u) zero4[tid] = 0u;
    // thread i holds item i of the chunk (its binning record, read contiguously)
    const uint32_t i = tid;
    uint4 ra = make_uint4(0u, 0u, 0u, 0u), rb = ra;
    if (i < n) {
        const uint4 *src = reinterpret_cast<const uint4 *>(bin + ci.beg + i);
        ra = src[0];
        rb = src[1];
        s_g[i] = ra.z;
    }
    const float thr = __uint_as_float(ra.w);
    const float spx = __uint_as_float(rb.x), spy = __uint_as_float(rb.y);
    const float sa = __uint_as_float(rb.z), sb = __uint_as_float(rb.w);
    {
        // the bitmaps start clear; the write phase clears the words it reads
        uint4 *const z = reinterpret_cast<uint4 *>(s_bits);
        for (uint32_t k = tid; k < (uint32_t)(kEmitWords * kEmitBand / 4); k += kEmitThreads)
            z[k] = make_uint4(0u, 0u, 0u, 0u);
        for (uint32_t k = tid; k < (uint32_t)kEmitBand; k += kEmitThreads) s_sum[k] = 0u;
    }
    const uint32_t TX = (uint32_t)ci.tiles_x, TY = TX ? ci.ntiles / TX : 0u;
    const uint32_t bw = min(TX, (uint32_t)kEmitBand), bh = (uint32_t)kEmitBand / max(bw, 1u);
    for (uint32_t r0 = 0; r0 < TY; r0 += bh) {
        for (uint32_t c0 = 0; c0 < TX; c0 += bw) {
            const uint32_t r1 = min(r0 + bh, TY), c1 = min(c0 + bw, TX);
            const uint32_t bwid = c1 - c0, nt = bwid * (r1 - r0);
            // the band's segment starts, in flight while the band is marked
            uint32_t pos[kEmitTilesPerThread];
#pragma unroll
            for (int q = 0; q < kEmitTilesPerThread; ++q) {
                const uint32_t lt = tid + (uint32_t)q * kEmitThreads;
                pos[q] = 0;
                if (lt < nt) {
                    const uint32_t rr = lt / bwid, t = (r0 + rr) * TX + c0 + (lt - rr * bwid);
                    pos[q] = tile_base[ci.tile_off + t] + pre[ci.row + t];
                }
            }
            __syncthreads();              // the bitmaps are clear; the staged items are published
            {
                // an item outside the chunk has an empty rectangle
                const uint32_t x0 = max(ra.x & 0xFFFFu, c0), y0 = max(ra.x >> 16, r0);
                const uint32_t x1 = min(ra.y & 0xFFFFu, c1), y1 = min(ra.y >> 16, r1);
                const uint32_t bit = 1u << (i & 31u), word = i >> 5, wbit = 1u << word;
                uint32_t *const bits = s_bits + word * (uint32_t)kEmitBand;
                for (uint32_t ty = y0; ty < y1; ++ty) {
                    const uint32_t rowb = (ty - r0) * bw - c0;
                    for (uint32_t cx = x0; cx < x1; ++cx) {
                        if (splat_touches_tile(spx, spy, sa, sb, thr, cx, ty)) {
                            atomicOr(&bits[rowb + cx], bit);
                            atomicOr(&s_sum[rowb + cx], wbit);
                        }
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < kEmitTilesPerThread; ++q) {
                const uint32_t lt = tid + (uint32_t)q * kEmitThreads;
                if (lt >= nt) continue;
                const uint32_t rr = lt / bwid, b = rr * bw + (lt - rr * bwid);
                uint32_t p = pos[q];
                uint32_t words = s_sum[b];
                s_sum[b] = 0u;
                while (words) {
                    const uint32_t w = (uint32_t)__builtin_ctz(words);
                    words &= words - 1u;
                    uint32_t m = s_bits[w * (uint32_t)kEmitBand + b];
                    s_bits[w * (uint32_t)kEmitBand + b] = 0u;
                    while (m) {
                        const uint32_t k = (uint32_t)__builtin_ctz(m);
                        m &= m - 1u;
                        pairs[p++] = s_g[w * 32u + k];
                    }
                }
            }
            __syncthreads();              // the bitmaps are read before the next band clears them
        }
    }
}

static uint32_t band_for(const Tables &tb) {
    return tb.max_view_tiles < (uint32_t)kBandTiles ? tb.max_view_tiles : (uint32_t)kBandTiles;
}

hipError_t launch_tile_count(const Tables &tb, uint32_t chunks, const uint32_t *order,
                             const uint2 *rect, const SplatRec *rec, float lambda, uint32_t *cnt, BinRec *bin,
                             hipStream_t st) {
    if (chunks == 0) return hipSuccess;
    const uint32_t band = band_for(tb);
    hipLaunchKernelGGL(k_tile_count, dim3(chunks), dim3(kCountThreads), (size_t)band * 4, st, tb, order, rect, rec,
                       lambda, cnt, bin, band);
    return hipGetLastError();
}

hipError_t launch_tile_emit(const Tables &tb, uint32_t chunks, const BinRec *bin, const uint32_t *pre,
                            const uint32_t *tile_base, uint32_t *pairs, uint32_t *zero4, uint32_t pair_cap,
                            hipStream_t st) {
    if (chunks == 0) return launch_fill_u32(zero4, 0u, 4, st);     // no items: no pairs
    hipLaunchKernelGGL(k_tile_emit, dim3(chunks), dim3(kEmitThreads), 0, st, tb, bin, pre, tile_base, pairs, zero4,
                       pair_cap);
    return hipGetLastError();
}

}  // namespace dpr
