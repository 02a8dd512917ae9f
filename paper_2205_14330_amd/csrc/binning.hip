// Screen-tile binning of the depth-sorted splats (only points near a pixel
// with non-negligible opacity are considered: end of Sec. 3.2).
//
// Instead of sorting (tile, depth) pairs, the depth-sorted item list of each
// view is cut into chunks of kChunkItems consecutive items and binned with a
// stable counting scatter:
//   count: per chunk, an LDS histogram of how many of its splats touch each
//          tile, stored tile-major as cnt[view][tile][chunk];
//   scan : one exclusive scan over all counts gives, for every (tile, chunk),
//          the first output slot; tile t's list is [scan(t, 0), scan(t+1, 0));
//   emit : per chunk, items are walked in depth order and appended to each
//          tile they touch through an LDS cursor per tile.
// Within a tile the lists come out in chunk order, and inside a chunk in item
// order, i.e. exactly ascending (depth, point index): the front-to-back order
// of Eq. (6)-(7).  The only pass over all pairs is the 4-byte write of emit.
#include "dpr_internal.h"

namespace dpr {

constexpr int kCountThreads = 256;
constexpr int kEmitThreads = 256;     // 4 waves; wave w owns tile rows with (row & 3) == w

struct ChunkInfo {
    uint32_t c;          // chunk index within the view
    uint32_t beg, end;   // sorted-item range
    uint32_t nchunks;
    int32_t tiles_x, tiles_y;
    uint64_t cnt_off;
};

__device__ __forceinline__ ChunkInfo chunk_info(const Tables &tb) {
    const int v = find_segment(tb.chunk_start, tb.n_views, blockIdx.x);
    const ViewDesc &vd = tb.views[v];
    ChunkInfo ci;
    ci.c = blockIdx.x - vd.chunk_off;
    ci.beg = vd.item_off + ci.c * (uint32_t)kChunkItems;
    ci.end = min(ci.beg + (uint32_t)kChunkItems, vd.item_off + (uint32_t)vd.n);
    ci.nchunks = vd.nchunks;
    ci.tiles_x = vd.tiles_x;
    ci.tiles_y = vd.tiles_y;
    ci.cnt_off = vd.cnt_off;
    return ci;
}

__global__ __launch_bounds__(kCountThreads) void k_tile_count(Tables tb, const uint32_t *order, const uint2 *rect,
                                                               uint32_t *cnt) {
    __shared__ uint32_t s_h[kBandTiles];
    const ChunkInfo ci = chunk_info(tb);
    const uint32_t ntiles = (uint32_t)ci.tiles_x * (uint32_t)ci.tiles_y;
    for (uint32_t band = 0; band < ntiles; band += kBandTiles) {
        const uint32_t bend = min(band + (uint32_t)kBandTiles, ntiles);
        for (uint32_t t = threadIdx.x; t < bend - band; t += kCountThreads) s_h[t] = 0;
        __syncthreads();
        for (uint32_t s = ci.beg + threadIdx.x; s < ci.end; s += kCountThreads) {
            const uint2 rc = rect[order[s]];
            const uint32_t x0 = rc.x & 0xFFFFu, y0 = rc.x >> 16, x1 = rc.y & 0xFFFFu, y1 = rc.y >> 16;
            for (uint32_t ty = y0; ty < y1; ++ty) {
                const uint32_t rowb = ty * (uint32_t)ci.tiles_x;
                if (rowb + x1 <= band || rowb + x0 >= bend) continue;
                for (uint32_t tx = x0; tx < x1; ++tx) {
                    const uint32_t t = rowb + tx;
                    if (t >= band && t < bend) atomicAdd(&s_h[t - band], 1u);
                }
            }
        }
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < bend - band; t += kCountThreads)
            cnt[ci.cnt_off + (uint64_t)(band + t) * ci.nchunks + ci.c] = s_h[t];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kEmitThreads) void k_tile_emit(Tables tb, const uint32_t *order, const uint2 *rect,
                                                             const uint32_t *range, uint32_t *pairs) {
    __shared__ uint32_t s_pos[kBandTiles];
    const ChunkInfo ci = chunk_info(tb);
    const uint32_t ntiles = (uint32_t)ci.tiles_x * (uint32_t)ci.tiles_y;
    const int lane = __lane_id();
    const uint32_t wave = threadIdx.x >> 6;
    for (uint32_t band = 0; band < ntiles; band += kBandTiles) {
        const uint32_t bend = min(band + (uint32_t)kBandTiles, ntiles);
        for (uint32_t t = threadIdx.x; t < bend - band; t += kEmitThreads)
            s_pos[t] = range[ci.cnt_off + (uint64_t)(band + t) * ci.nchunks + ci.c];
        __syncthreads();
        // every wave walks the whole chunk in depth order; it only appends to
        // the tile rows it owns, so no two waves touch the same cursor
        for (uint32_t s0 = ci.beg; s0 < ci.end; s0 += 64) {
            const uint32_t my = s0 + (uint32_t)lane;
            uint32_t g = 0;
            uint2 rc = make_uint2(0u, 0u);
            if (my < ci.end) {
                g = order[my];
                rc = rect[g];
            }
            const uint32_t nb = min(64u, ci.end - s0);
            for (uint32_t j = 0; j < nb; ++j) {
                const uint32_t gj = __builtin_amdgcn_readlane(g, j);
                const uint32_t ra = __builtin_amdgcn_readlane(rc.x, j);
                const uint32_t rb = __builtin_amdgcn_readlane(rc.y, j);
                const uint32_t x0 = ra & 0xFFFFu, y0 = ra >> 16, x1 = rb & 0xFFFFu, y1 = rb >> 16;
                if (x1 <= x0 || y1 <= y0) continue;
                const uint32_t first = y0 + ((wave - (y0 & 3u)) & 3u);   // first row == wave (mod 4)
                if (first >= y1) continue;
                const uint32_t rows = (y1 - first + 3u) >> 2;
                const uint32_t width = x1 - x0;
                const uint32_t n = rows * width;
                const float inv_w = 1.0f / (float)width;
                for (uint32_t k = (uint32_t)lane; k < n; k += 64u) {
                    const uint32_t rr = (uint32_t)(((float)k + 0.5f) * inv_w);
                    const uint32_t cc = k - rr * width;
                    const uint32_t t = (first + 4u * rr) * (uint32_t)ci.tiles_x + x0 + cc;
                    if (t >= band && t < bend) {
                        const uint32_t p = atomicAdd(&s_pos[t - band], 1u);
                        pairs[p] = gj;
                    }
                }
            }
        }
        __syncthreads();
    }
}

hipError_t launch_tile_count(const Tables &tb, uint32_t chunks, const uint32_t *order,
                             const uint2 *rect, uint32_t *cnt, hipStream_t st) {
    if (chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_count, dim3(chunks), dim3(kCountThreads), 0, st, tb, order, rect, cnt);
    return hipGetLastError();
}

hipError_t launch_tile_emit(const Tables &tb, uint32_t chunks, const uint32_t *order,
                            const uint2 *rect, const uint32_t *range, uint32_t *pairs,
                            hipStream_t st) {
    if (chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_emit, dim3(chunks), dim3(kEmitThreads), 0, st, tb, order, rect, range, pairs);
    return hipGetLastError();
}

}  // namespace dpr
