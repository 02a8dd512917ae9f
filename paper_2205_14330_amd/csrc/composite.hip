// Per-tile front-to-back compositing (Sec. 3.2, Eq. 5-7) and its reverse-mode
// derivative.
//
// Forward: one workgroup of 2 waves per 16x16 tile; wave w owns the 16x8
// half w, two horizontally adjacent pixels per lane.  Each wave walks the
// tile's depth-ordered list on its own, in chunks of 128 positions: the splat
// records are gathered into registers one chunk ahead; at a chunk's start the
// records that may reach one of the wave's live pixels are kept in LDS, and
// read back as broadcasts in unrolled groups of 16 (compile-time offsets),
// each 32-byte record one record ahead of its use.  The blend is branch-free
// per pixel.  A pixel stops after the first blended
// splat that leaves T < t_min; a wave leaves the list once its 128 pixels have
// stopped.
//
// Backward: one wave per (tile, segment) work item; each lane owns a 2x2
// pixel quad so that the per-splat reduction is shared by 256 pixels.  A
// segment is 256 list positions; the forward left at each segment boundary a
// checkpoint of every pixel's (T, I), so the segments of one long list are
// processed independently and in parallel (the longest tiles no longer set
// the kernel's duration).  A segment is walked in reverse from its end (or the
// furthest blend end in it), recovering T_i = T_{i+1} / (1 - alpha_i)
// (alpha <= alpha_max < 1), carrying D = dL/dI . B + dL/dT T_final with B the
// colour blended behind (B = I_final - I_checkpoint at a segment end), and
// folding each (pixel, splat) contribution into 7 per-lane partial sums.  A
// chunk of 64 records is gathered one per lane, written to LDS and read back
// as broadcasts, one record ahead of its use, in unrolled groups of 16.  T is
// recovered with one reciprocal per lane and splat, of the product of the
// quad's four (1 - alpha).  Each lane stages its 7 sums of up to 4 splats in
// LDS, and each flush completes the 28 sums over the 64 lanes and adds them to
// the per-item gradient records with one float atomic each.
#include "dpr_internal.h"

#include <cstring>

namespace dpr {

constexpr int kCompLanes = 64;
constexpr int kQuad = 4;          // pixels per lane

// Keeps a wave-uniform value in a VGPR.  A VALU instruction that reads an SGPR
// issues at about half the rate of one whose operands are VGPRs, inline
// constants or literals (measured on gfx950: ~4 against ~2 clocks per wave64
// add), so the loop-invariant thresholds of the inner loops are copied to
// VGPRs once.  The empty asm hides the value's uniformity from the compiler,
// which would otherwise fold it back into SGPR operands.
template <typename V>
__device__ __forceinline__ V in_vgpr(V x) {
    asm volatile("" : "+v"(x));
    return x;
}

struct TileCtx {
    uint32_t start, end;       // list range in pairs[]
    int v;                     // view
    int x0, y0;                // top-left pixel of this lane's quad
};

// Backward layout: lane owns the 2x2 quad at (2 (lane & 7), 2 (lane >> 3)).
__device__ __forceinline__ TileCtx tile_ctx(const CompositeArgs &a, uint32_t tile) {
    TileCtx c;
    c.v = find_segment(a.tile_start, a.n_views, tile);
    const ViewDesc &vd = a.views[c.v];
    const uint32_t lt = tile - vd.tile_off;
    const uint32_t ty = lt / (uint32_t)vd.tiles_x;
    const uint32_t tx = lt - ty * (uint32_t)vd.tiles_x;
    const int lane = threadIdx.x & 63;
    c.x0 = (int)(tx * kTile) + 2 * (lane & 7);
    c.y0 = (int)(ty * kTile) + 2 * (lane >> 3);
    c.start = a.tile_base[tile];
    c.end = a.tile_base[tile + 1];
    return c;
}

// alpha = min(alpha_max, 2^e); the clamp (and only it) blocks the gradient to e.
// The exponent never exceeds the record's w (its quadratic form is >= 0), so a
// splat whose peak 2^w stays below alpha_max clamps no pixel; w_noclamp puts
// that test a margin of 2^-1e-5 (about 58 float ulps) inside alpha_max, far
// above the error of exp2 and log2.  The forward flags each staged chunk that
// holds a record with w above it and applies the clamp to every record of a
// flagged chunk only (a no-op for the others), so the common chunk pays no
// per-record test; the backward tests w per record, on a path of its own.
__device__ __forceinline__ float no_clamp_w(float alpha_max) { return __log2f(alpha_max) - 1e-5f; }

// Record k of the pair list, or an inert record past the end.
__device__ __forceinline__ void load_rec(const CompositeArgs &a, uint32_t k, uint32_t end, float4 &r0, float4 &r1,
                                         uint32_t &id) {
    if (k < end) {
        id = a.pairs[k];
        const float4 *src = reinterpret_cast<const float4 *>(a.rec + id);
        r0 = src[0];
        r1 = src[1];
    } else {
        id = 0;
        r0 = make_float4(0.f, 0.f, 0.f, 0.f);
        r1 = make_float4(-INFINITY, 0.f, 0.f, 0.f);
    }
}

// next tile for persistent waves
__device__ __forceinline__ uint32_t pop_tile(uint32_t *queue) {
    uint32_t t = 0;
    if (threadIdx.x == 0) t = atomicAdd(queue, 1u) + gridDim.x;
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// Two waves per tile: wave w owns rows [8w, 8w + 8), each lane a horizontal
// pixel pair.  The waves walk the tile's list independently, kFwdChunk list
// positions at a time.  Each lane gathers kFwdPerLane records of the next
// chunk into registers while the current chunk is blended (the ids one chunk
// further ahead, so the record loads never wait for them).  At the start of a
// chunk the wave takes the bounding box of its live pixels from two ballots
// and keeps, in LDS and in list order, only the records that may reach a pixel
// centre of that box (splat_reaches_box, conservative).  A skipped record
// cannot blend a live pixel, and a pixel that has stopped blends nothing more,
// so the result is the walk over every record.  The kept records are padded
// with inert ones (w = -inf) to whole groups of kFwdGroup, and each group is
// walked fully unrolled, so every LDS read of a record has a compile-time
// offset and the walk has no per-record loop control; each record is read one
// record ahead of its use.  A record that no pixel of the wave blends skips
// the blend after its exponents.
constexpr int kFwdPx = 2;                 // pixels per lane
constexpr int kFwdThreads = 128;
constexpr int kFwdChunk = 128;            // list positions per chunk
constexpr int kFwdPerLane = kFwdChunk / 64;
constexpr int kFwdGroup = 16;             // kept records per unrolled group
static_assert(kFwdChunk % kFwdGroup == 0, "whole groups fit the staged chunk");

// A pixel is live while T >= t_min: T only decreases, by T alpha <= T, and
// the pixel stops right after the blend that takes it below t_min, so the
// test is exactly the stop rule.  Pixels outside the image start at T = -1.
//
// With backward state requested (a.nlast non-null) the kernel also writes,
// per pixel, its blend end (one past the list position of the last splat it
// blended, 0 if none: no later splat changes the pixel) and the final (T, I);
// at every list position s * kBwdSeg its wave reaches, the (T, I) checkpoint
// of each of the wave's pixels (a pixel that blends past that position keeps
// its wave walking, so every checkpoint the backward reads is written); and
// it appends the tile's backward work items (tile, s) for
// s < ceil(max blend end / kBwdSeg).  Within a group a pixel keeps the
// group-relative index of its last blended record (a compile-time constant
// of the unrolled walk), folded into the chunk's kept-record index after the
// group; the list position is formed once per chunk.
static_assert(kBwdSeg % kFwdChunk == 0, "backward segments are whole forward chunks");

// The 8 bits of a 64-lane mask folded over its 8 groups of 8 lanes: bit c is
// set if lane 8r + c is set for some r.
__device__ __forceinline__ uint32_t fold_columns(uint64_t m) {
    m |= m >> 32;
    m |= m >> 16;
    m |= m >> 8;
    return (uint32_t)m & 0xFFu;
}

// COUNT: the kernel counts each pixel's blended splats, for the per-pixel
// statistics and for the cap th.max_splats: a pixel also stops after blending
// that many (then it is live while T >= t_min and fewer than max_splats splats
// were blended).  Without a cap the count never reaches cap = 2^32 - 1.
// STATE: backward state is requested (a.nlast non-null); without it the
// kernel keeps no blend ends.
template <bool PERSISTENT, bool COUNT, bool STATE>
__global__ __launch_bounds__(kFwdThreads) void k_composite(CompositeArgs a) {
    constexpr int PX = kFwdPx, kThreads = kFwdThreads, kChunk = kFwdChunk, kPer = kFwdPerLane;
    // per wave: the kept records of the current chunk (padded to whole groups)
    // and the chunk position of each kept record
    __shared__ float4 s_r0[2][kChunk], s_r1[2][kChunk];
    __shared__ uint32_t s_j[2][kChunk];
    __shared__ uint32_t s_next, s_max[2], s_work;
    const float lambda = a.th.lambda;
    const float neg_lambda = in_vgpr(-lambda);
    const float alpha_max = a.th.alpha_max;
    const float w_noclamp = in_vgpr(no_clamp_w(alpha_max));
    const float t_min = in_vgpr(a.th.t_min);
    const uint32_t cap = in_vgpr(a.th.max_splats > 0 ? a.th.max_splats : 0xFFFFFFFFu);
    if (a.tile_base[a.total_tiles] > a.pair_cap) return;   // the pair lists do not fit the workspace
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // block (or popped) index -> tile: through the longest-first order when there is one
    for (uint32_t idx = blockIdx.x; idx < a.total_tiles;) {
        const uint32_t tile = a.tile_order ? a.tile_order[idx] : (PERSISTENT ? idx : xcd_remap(idx, a.total_tiles));
        const int v = find_segment(a.tile_start, a.n_views, tile);
        const ViewDesc &vd = a.views[v];
        const uint32_t lt = tile - vd.tile_off;
        const uint32_t ty = lt / (uint32_t)vd.tiles_x;
        const uint32_t tx = lt - ty * (uint32_t)vd.tiles_x;
        const uint32_t start = a.tile_base[tile], end = a.tile_base[tile + 1];
        const int lx = 2 * (lane & 7), ly = 8 * wave + (lane >> 3);     // in-tile position of pixel 0
        const int x0 = (int)(tx * kTile) + lx, y0 = (int)(ty * kTile) + ly;
        // pixel centres of the wave's first column and row
        const float cx0 = (float)(tx * kTile) + 0.5f, cy0 = (float)(ty * kTile + 8 * wave) + 0.5f;
        float ux[PX], uy[PX], T[PX], I0[PX], I1[PX], I2[PX];
        uint32_t nlast[PX], nblend[PX];
        int last[PX];                     // index of the last blended kept record of this chunk, or -1
#pragma unroll
        for (int p = 0; p < PX; ++p) {
            const int px = x0 + p, py = y0;
            ux[p] = (float)px + 0.5f;
            uy[p] = (float)py + 0.5f;
            T[p] = (px < vd.width && py < vd.height) ? 1.f : -1.f;
            I0[p] = I1[p] = I2[p] = 0.f;
            nlast[p] = 0; nblend[p] = 0; last[p] = -1;
        }
        // records of the chunk at `base` (registers), ids of the chunk after it
        float4 n0[kPer], n1[kPer];
        uint32_t nid[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const uint32_t k = start + q * 64 + lane;
            n0[q] = make_float4(0.f, 0.f, 0.f, 0.f);
            n1[q] = make_float4(-INFINITY, 0.f, 0.f, 0.f);
            if (k < end) {
                const float4 *src = reinterpret_cast<const float4 *>(a.rec + a.pairs[k]);
                n0[q] = src[0];
                n1[q] = src[1];
            }
            nid[q] = (k + kChunk < end) ? a.pairs[k + kChunk] : 0u;
        }
        for (uint32_t base = start; base < end; base += kChunk) {
            bool live[PX];
#pragma unroll
            for (int p = 0; p < PX; ++p) live[p] = T[p] >= t_min && (!COUNT || nblend[p] < cap);
            const uint64_t m0 = __ballot(live[0]), m1 = __ballot(live[1]);
            if ((m0 | m1) == 0ull) break;
            if (STATE && a.ckpt && base > start && (base - start) % (uint32_t)kBwdSeg == 0) {
                float4 *dst = a.ckpt + ckpt_slot(start, tile, (base - start) / (uint32_t)kBwdSeg) * kTilePix +
                              ly * kTile + lx;
#pragma unroll
                for (int p = 0; p < PX; ++p) dst[p] = make_float4(T[p], I0[p], I1[p], I2[p]);
            }
            // the live pixels' box: rows from the first and last live lane
            // (row = lane / 8), columns from the folded masks of the even
            // (pixel 0) and odd (pixel 1) columns
            const uint64_t m = m0 | m1;
            const int r_lo = __builtin_ctzll(m) >> 3, r_hi = (63 - __builtin_clzll(m)) >> 3;
            const uint32_t c0 = fold_columns(m0), c1 = fold_columns(m1);
            int x_lo = 2 * kTile, x_hi = -1;
            if (c0) { x_lo = 2 * __builtin_ctz(c0); x_hi = 2 * (31 - __builtin_clz(c0)); }
            if (c1) { x_lo = min(x_lo, 2 * __builtin_ctz(c1) + 1); x_hi = max(x_hi, 2 * (31 - __builtin_clz(c1)) + 1); }
            const float bx0 = cx0 + (float)x_lo, bx1 = cx0 + (float)x_hi;
            const float by0 = cy0 + (float)r_lo, by1 = cy0 + (float)r_hi;
            // keep the records that may reach the box, in list order
            int kept = 0;
            bool near = false;
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const uint32_t j = (uint32_t)(q * 64 + lane);
                const bool keep = base + j < end &&
                                  splat_reaches_box(n0[q].x, n0[q].y, n0[q].z, n0[q].w, n1[q].x + lambda, bx0, bx1,
                                                    by0, by1);
                const uint64_t km = __ballot(keep);
                if (keep) {
                    const int pos = kept + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
                    s_r0[wave][pos] = n0[q];
                    s_r1[wave][pos] = n1[q];
                    if (STATE) s_j[wave][pos] = j;
                    near = near || n1[q].x > w_noclamp;
                }
                kept += __builtin_popcountll(km);
            }
            // the chunk flag: may any kept record reach the alpha_max clamp
            const bool chunk_clamp = __ballot(near) != 0ull;
            // inert records (w = -inf: no pixel passes e >= -lambda) up to a whole group
            {
                const int kp = (kept + kFwdGroup - 1) & ~(kFwdGroup - 1);
                if (lane < kp - kept) {
                    s_r0[wave][kept + lane] = make_float4(0.f, 0.f, 0.f, 0.f);
                    s_r1[wave][kept + lane] = make_float4(-INFINITY, 0.f, 0.f, 0.f);
                }
            }
            // the next chunk's records, and the ids of the one after it
#pragma unroll
            for (int q = 0; q < kPer; ++q) {
                const uint32_t k = base + kChunk + q * 64 + lane;
                if (k < end) {
                    const float4 *src = reinterpret_cast<const float4 *>(a.rec + nid[q]);
                    n0[q] = src[0];
                    n1[q] = src[1];
                }
                if (k + kChunk < end) nid[q] = a.pairs[k + kChunk];
            }
            // the kept records are written before any lane of the wave reads them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            for (int j0 = 0; j0 < kept; j0 += kFwdGroup) {
                if (j0 > 0) {
                    bool any_live = false;
#pragma unroll
                    for (int p = 0; p < PX; ++p) any_live = any_live || (T[p] >= t_min && (!COUNT || nblend[p] < cap));
                    if (__ballot(any_live) == 0ull) break;
                }
                int lrel[PX];
#pragma unroll
                for (int p = 0; p < PX; ++p) lrel[p] = -1;
                auto blend = [&](const float4 &r0, const float4 &r1, int jr) {
                    SplatRec s;
                    s.px = r0.x; s.py = r0.y; s.a = r0.z; s.b = r0.w;
                    s.w = r1.x;
                    s.cr = r1.y; s.cg = r1.z; s.cb = r1.w;
                    float alpha[PX], e[PX];
                    bool hit[PX];
                    bool any = false;
#pragma unroll
                    for (int p = 0; p < PX; ++p) {
                        float dx, dy;
                        e[p] = splat_exponent(s, ux[p], uy[p], dx, dy);
                        hit[p] = (T[p] >= t_min) & (!COUNT || nblend[p] < cap) & (e[p] >= neg_lambda);
                        any = any || hit[p];
                    }
                    if (__ballot(any) == 0ull) return;
#pragma unroll
                    for (int p = 0; p < PX; ++p) alpha[p] = hit[p] ? __builtin_amdgcn_exp2f(e[p]) : 0.f;
                    if (__builtin_expect(chunk_clamp, 0)) {
                        const float am = in_vgpr(alpha_max);
#pragma unroll
                        for (int p = 0; p < PX; ++p)
                            if (alpha[p] > am) alpha[p] = am;
                    }
#pragma unroll
                    for (int p = 0; p < PX; ++p) {
                        const float Ta = T[p] * alpha[p];
                        I0[p] = fmaf(Ta, s.cr, I0[p]);
                        I1[p] = fmaf(Ta, s.cg, I1[p]);
                        I2[p] = fmaf(Ta, s.cb, I2[p]);
                        if (COUNT) nblend[p] += hit[p] ? 1u : 0u;
                        T[p] = T[p] - Ta;
                        if (STATE && hit[p]) lrel[p] = jr;
                    }
                };
                const float4 *q0 = s_r0[wave] + j0, *q1 = s_r1[wave] + j0;
                float4 a0 = q0[0], a1 = q1[0];
#pragma unroll
                for (int j = 0; j < kFwdGroup; ++j) {
                    float4 c0 = a0, c1 = a1;
                    if (j + 1 < kFwdGroup) { c0 = q0[j + 1]; c1 = q1[j + 1]; }
                    blend(a0, a1, j);
                    a0 = c0; a1 = c1;
                }
#pragma unroll
                for (int p = 0; p < PX; ++p)
                    if (STATE && lrel[p] >= 0) last[p] = j0 + lrel[p];
            }
#pragma unroll
            for (int p = 0; p < PX; ++p)
                if (STATE && last[p] >= 0) {
                    nlast[p] = base - start + s_j[wave][last[p]] + 1u;
                    last[p] = -1;
                }
            // this chunk's kept records are read before the next chunk's are written
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        uint32_t mymax = 0;
#pragma unroll
        for (int p = 0; p < PX; ++p) {
            const int px = x0 + p, py = y0;
            if (px >= vd.width || py >= vd.height) continue;
            const uint64_t lpix = (uint64_t)py * (uint64_t)vd.width + (uint64_t)px;
            const uint64_t pix = vd.pix_off + lpix;
            if (a.write_views) {
                float *img = vd.image + 3 * lpix;
                img[0] = I0[p]; img[1] = I1[p]; img[2] = I2[p];
                if (vd.trans) vd.trans[lpix] = T[p];
                if (COUNT && a.stats) a.stats[pix] = nblend[p];
            }
            if (STATE) {
                a.nlast[pix] = nlast[p];
                a.fin[pix] = make_float4(T[p], I0[p], I1[p], I2[p]);
                mymax = max(mymax, nlast[p]);
            }
        }
        if (STATE) {
            // the tile's backward work items: one per kBwdSeg positions below its largest blend end
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) mymax = max(mymax, (uint32_t)__shfl_xor((int)mymax, d, 64));
            if (lane == 0) s_max[wave] = mymax;
            __syncthreads();
            const uint32_t nseg = (max(s_max[0], s_max[1]) + (uint32_t)kBwdSeg - 1) / (uint32_t)kBwdSeg;
            if (tid == 0) s_work = nseg ? atomicAdd(a.counters + 1, nseg) : 0u;
            __syncthreads();
            for (uint32_t i = tid; i < nseg; i += kThreads) a.work[s_work + i] = make_uint2(tile, i);
        }
        if (!PERSISTENT) break;
        __syncthreads();
        if (tid == 0) s_next = atomicAdd(a.counters, 1u) + gridDim.x;
        __syncthreads();
        idx = s_next;
    }
}


// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// The value of the lane given by a quad-permute pattern.  ds_swizzle in quad
// mode (offset bit 15 set; two bits per destination lane of the quad) runs on
// the LDS pipe; a DPP-modified add costs about twice a plain one on the VALU.
template <int PATTERN>
__device__ __forceinline__ float swizzle(float v) {
    return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x8000 | PATTERN));
}

// Staging of per-splat partial sums: slot k holds, for one splat, each lane's
// 7 sums (over its 4 pixels) column by column, the 64 lanes of a column in
// consecutive words (one conflict-free store per column), columns
// kColStride = 68 words apart.  No cross-lane operation runs per splat: a
// lane-pair swizzle per sum cost more (7 LDS-pipe operations and a wait per
// splat) than the longer flush sums.  4 slots keep the kernel's LDS within
// 16 waves per CU.
constexpr int kSlots = 4;
constexpr int kCols = 7;
constexpr int kColStride = 68;
constexpr int kSlotStride = kCols * kColStride;

// Completes the sums of the first nslots slots and adds them to the gradient
// records: lane L sums half h = L & 1 (32 lanes' values, eight 16-byte reads)
// of column c = (L >> 1) & 7 < 7 of slot k = L >> 4, one swizzle adds the other
// half, and the lane with h = 0 issues the atomic.  Columns 0-2 are quantities
// 0-2 and columns 3-6 quantities 4-7 (quantity 3 is unused).  Slot k's item id
// is s_ids[(slotj >> 7k) & 127]: the wave-uniform slotj holds, per slot, the
// parity of the chunk its splat came from (which half of the double-buffered
// s_ids holds that chunk's ids) and the splat's index in the chunk.
__device__ __forceinline__ void flush_slots(const float *s_part, const uint32_t *s_ids, uint32_t slotj, int nslots,
                                            float *grad, int lane) {
    const int k = lane >> 4, c = (lane >> 1) & 7, h = lane & 1;
    const bool act = k < nslots && c < kCols;
    float sum = 0.f;
    if (act) {
        const float4 *src = reinterpret_cast<const float4 *>(s_part + k * kSlotStride + c * kColStride + 32 * h);
        float4 t = src[0];
#pragma unroll
        for (int o = 1; o < 8; ++o) {
            const float4 u = src[o];
            t.x += u.x; t.y += u.y; t.z += u.z; t.w += u.w;
        }
        sum = (t.x + t.y) + (t.z + t.w);
    }
    sum += swizzle<0xB1>(sum);
    if (act && h == 0) {
        const uint32_t gid = s_ids[(slotj >> (7 * k)) & 127u];
        atomicAdd(grad + 8 * (size_t)gid + (c < 3 ? c : c + 1), sum);
    }
}

// Persistent: each wave pops (tile, segment) work items until the list is
// exhausted.  Segment s covers list positions [s kBwdSeg, (s + 1) kBwdSeg); a
// pixel still live after the segment starts from the checkpoint there, any
// other pixel from its final state.
__global__ __launch_bounds__(kCompLanes) void k_composite_bwd(BackwardArgs b) {
    __shared__ __align__(16) float s_part[kSlots * kSlotStride];
    __shared__ uint32_t s_ids[2 * kCompLanes];
    // the current chunk: record j at s_rec[2j], s_rec[2j + 1]
    __shared__ float4 s_rec[2 * kCompLanes];
    const CompositeArgs &a = b.c;
    const float neg_lambda = in_vgpr(-a.th.lambda);
    const float alpha_max = a.th.alpha_max;
    const float w_noclamp = in_vgpr(no_clamp_w(alpha_max));
    const int lane = threadIdx.x;
    float *const my_part = s_part + lane;
    const uint32_t nwork = *b.work_count;

    for (uint32_t w = blockIdx.x; w < nwork;) {
        const uint2 item = b.work[w];
        const uint32_t tile = item.x;
        const uint32_t seg_beg = item.y * (uint32_t)kBwdSeg, seg_end = seg_beg + (uint32_t)kBwdSeg;
        const TileCtx c = tile_ctx(a, tile);
        const ViewDesc &vd = a.views[c.v];
        const float4 *ck = b.ckpt + ckpt_slot(c.start, tile, item.y + 1) * kTilePix;
        // per pixel: T (recovered front-to-back transmittance), dL/dI, and
        // D = dL/dI . B + dL/dT * T_final with B = sum over the blended splats
        // behind of T_k alpha_k c_k, so that dL/dalpha_i = T_i (dL/dI . c_i) - D / (1 - alpha_i).
        // The walk keeps E = D / T_after (T_after: the transmittance behind
        // splat i, T_i (1 - alpha_i)) instead of D: then dL/dalpha_i =
        // T_i (dL/dI . c_i - E) and, one splat further forward,
        // E <- E + alpha_i (dL/dI . c_i - E), a convex step for alpha in [0, 1].
        float ux[kQuad], uy[kQuad], T[kQuad], gI0[kQuad], gI1[kQuad], gI2[kQuad], D[kQuad];
        uint32_t nl[kQuad];
        uint32_t mymax = 0;
#pragma unroll
        for (int p = 0; p < kQuad; ++p) {
            const int px = c.x0 + (p & 1), py = c.y0 + (p >> 1);
            ux[p] = (float)px + 0.5f;
            uy[p] = (float)py + 0.5f;
            nl[p] = 0; T[p] = 1.f; gI0[p] = gI1[p] = gI2[p] = 0.f; D[p] = 0.f;
            if (px < vd.width && py < vd.height) {
                const uint64_t lpix = (uint64_t)py * (uint64_t)vd.width + (uint64_t)px;
                const uint64_t pix = vd.pix_off + lpix;
                nl[p] = b.nlast[pix];
                const float4 f = b.fin[pix];
                const float *gi = b.dimage[c.v] + 3 * lpix;
                gI0[p] = gi[0]; gI1[p] = gi[1]; gI2[p] = gi[2];
                const float gT = (b.dtrans && b.dtrans[c.v]) ? b.dtrans[c.v][lpix] : 0.f;
                if (nl[p] > seg_end) {
                    // blends past this segment: B = I_final - (I after the first seg_end splats)
                    const float4 k = ck[(py - (c.y0 & ~(kTile - 1))) * kTile + (px - (c.x0 & ~(kTile - 1)))];
                    T[p] = k.x;
                    D[p] = fmaf(gI0[p], f.y - k.y, fmaf(gI1[p], f.z - k.z, fmaf(gI2[p], f.w - k.w, gT * f.x)));
                } else {
                    T[p] = f.x;
                    D[p] = gT * f.x;                                        // dL/dT * T_final
                }
                mymax = max(mymax, min(nl[p], seg_end));
            }
            D[p] = D[p] / T[p];      // E; T > 0 (a product of factors 1 - alpha >= 1 - alpha_max)
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) mymax = max(mymax, (uint32_t)__shfl_xor((int)mymax, d, 64));
        const uint32_t maxn = (uint32_t)__builtin_amdgcn_readfirstlane((int)mymax);

        // chunks back to front: [cbeg, cbeg + 64) aligned to the segment start
        int nslots = 0;
        uint32_t slotj = 0, slot_par = 0;    // slot k: bits [7k, 7k + 7) = chunk parity * 64 + record
        if (maxn > seg_beg) {
            const uint32_t sbeg = c.start + seg_beg;
            uint32_t cbeg = sbeg + ((maxn - seg_beg - 1) / kCompLanes) * kCompLanes;
            const uint32_t lend = c.start + maxn;
            float4 n0, n1;
            uint32_t nid;
            load_rec(a, cbeg + lane, lend, n0, n1, nid);
            // Pixel p may have blended the record at list position cbeg - start + j
            // only if that position is below nl[p], i.e. iff j < lim[p] =
            // nl[p] - (cbeg - start) for the current chunk; lim grows by 64 per
            // chunk back.  Within a group of 16 records from g0 the test is
            // jj < limg[p] = lim[p] - g0 with jj = j - g0 a compile-time constant.
            int lim[kQuad], limg[kQuad];
#pragma unroll
            for (int p = 0; p < kQuad; ++p) lim[p] = (int)nl[p] - (int)(cbeg - c.start);
            int par = 0;
            while (true) {
                if (slot_par & (1u << par)) {    // pending slots name ids about to be overwritten
                    __syncthreads();
                    flush_slots(s_part, s_ids, slotj, nslots, b.grad, lane);
                    nslots = 0; slotj = 0; slot_par = 0;
                }
                __syncthreads();                 // the previous chunk's broadcasts are done
                s_rec[2 * lane] = n0;
                s_rec[2 * lane + 1] = n1;
                s_ids[par * kCompLanes + lane] = nid;
                __syncthreads();
                const bool more = cbeg > sbeg;
                if (more) load_rec(a, cbeg - kCompLanes + lane, lend, n0, n1, nid);
                const int cnt = (int)min((uint32_t)kCompLanes, lend - cbeg);
                // one (pixel, splat) record of the walk: record j = g0 + jj of the chunk
                auto splat = [&](const float4 &f0, const float4 &f1, int jj, int j) {
                    SplatRec s;
                    s.px = f0.x; s.py = f0.y; s.a = f0.z; s.b = f0.w;
                    s.w = f1.x;
                    float gw[kQuad], Ta[kQuad], e[kQuad], g[kQuad], alpha[kQuad];
                    float dx0 = 0.f, dy0 = 0.f;
                    bool hit[kQuad];
                    bool any = false;
#pragma unroll
                    for (int p = 0; p < kQuad; ++p) {
                        float dx, dy;
                        e[p] = splat_exponent(s, ux[p], uy[p], dx, dy);
                        if (p == 0) { dx0 = dx; dy0 = dy; }
                        hit[p] = (jj < limg[p]) & (e[p] >= neg_lambda);
                        any = any || hit[p];
                    }
                    // a splat that no pixel of the tile blended changes nothing below
                    // (alpha = 0 for every pixel makes every update an exact no-op)
                    if (__ballot(any) == 0ull) return;
                    s.cr = f1.y; s.cg = f1.z; s.cb = f1.w;
#pragma unroll
                    for (int p = 0; p < kQuad; ++p) {
                        g[p] = __builtin_amdgcn_exp2f(e[p]);
                        // a pixel that did not blend this splat gets alpha = 0, so
                        // 1/(1 - alpha) = 1 and every update below is an exact no-op for it
                        alpha[p] = hit[p] ? g[p] : 0.f;
                    }
                    // the alpha_max clamp, which also blocks the gradient to e, is rare:
                    // e <= w (q >= 0), so a splat whose peak 2^w stays below alpha_max
                    // (with a margin far above the error of exp2) clamps no pixel.  It is
                    // applied on a path of its own before and after the update; the
                    // threshold is read inside each branch so that the compares stay there.
                    const bool near_max = __builtin_expect(s.w > w_noclamp, 0);
                    if (near_max) {
                        const float am = in_vgpr(alpha_max);
#pragma unroll
                        for (int p = 0; p < kQuad; ++p)
                            if (alpha[p] > am) alpha[p] = am;    // only a blending pixel has alpha > 0
                    }
                    // 1 / (1 - alpha) of the four pixels from one reciprocal of their
                    // product (each factor >= 1 - alpha_max, so the product neither
                    // underflows nor overflows): r = 1 / (o0 o1 o2 o3), 1 / o0 = r o1 o2 o3 ...
                    float inv[kQuad];
                    {
                        const float o0 = 1.0f - alpha[0], o1 = 1.0f - alpha[1];
                        const float o2 = 1.0f - alpha[2], o3 = 1.0f - alpha[3];
                        const float p01 = o0 * o1, p23 = o2 * o3;
                        const float r = __builtin_amdgcn_rcpf(p01 * p23);
                        const float r01 = r * p23, r23 = r * p01;
                        inv[0] = r01 * o1; inv[1] = r01 * o0;
                        inv[2] = r23 * o3; inv[3] = r23 * o2;
                    }
#pragma unroll
                    for (int p = 0; p < kQuad; ++p) {
                        const float iom = inv[p];
                        T[p] = T[p] * iom;                       // T in front of this splat
                        Ta[p] = T[p] * alpha[p];
                        const float gc = fmaf(gI0[p], s.cr, fmaf(gI1[p], s.cg, gI2[p] * s.cb));
                        const float t = gc - D[p];                       // dL/dalpha = T t (D holds E)
                        gw[p] = Ta[p] * t;                               // dL/de / ln 2
                        D[p] = fmaf(alpha[p], t, D[p]);
                    }
                    if (near_max) {
                        const float am = in_vgpr(alpha_max);
#pragma unroll
                        for (int p = 0; p < kQuad; ++p)
                            if (hit[p] && g[p] > am) gw[p] = 0.f;
                    }
                    // quad pixel p sits at (+(p & 1), +(p >> 1)) from pixel 0, so its
                    // dx is dx0 - (p & 1) and its dy is dy0 - (p >> 1)
                    const float gx = gw[1] + gw[3], gz = gw[0] + gw[2];
                    const float v4 = gx + gz;
                    const float v0 = fmaf(dx0, v4, -gx);
                    const float v1 = fmaf(dy0, v4, -(gw[2] + gw[3]));
                    // sum of gw q with q = w - e: w sum(gw) - sum(gw e)
                    float v2 = s.w * v4;
                    float v5 = Ta[0] * gI0[0], v6 = Ta[0] * gI1[0], v7 = Ta[0] * gI2[0];
#pragma unroll
                    for (int p = 0; p < kQuad; ++p) {
                        v2 = fmaf(-gw[p], e[p], v2);
                        if (p == 0) continue;
                        v5 = fmaf(Ta[p], gI0[p], v5);
                        v6 = fmaf(Ta[p], gI1[p], v6);
                        v7 = fmaf(Ta[p], gI2[p], v7);
                    }
                    {
                        const float v[kCols] = {v0, v1, v2, v4, v5, v6, v7};
                        float *dst = my_part + nslots * kSlotStride;
#pragma unroll
                        for (int i = 0; i < kCols; ++i) dst[i * kColStride] = v[i];
                    }
                    slotj |= (uint32_t)(par * kCompLanes + j) << (7 * nslots);
                    slot_par |= 1u << par;
                    if (++nslots == kSlots) {
                        __syncthreads();     // staged sums are written before other lanes read them
                        flush_slots(s_part, s_ids, slotj, kSlots, b.grad, lane);
                        __syncthreads();     // and read before the slots are written again
                        nslots = 0; slotj = 0; slot_par = 0;
                    }
                };
                // The chunk is walked back to front in groups of 16 records, each
                // fully unrolled so that every LDS read has a compile-time offset;
                // record j - 1 is read while record j is processed.  The records
                // past cnt in the top group are the inert ones of the chunk load.
                const float4 *rb = s_rec;
                for (int g0 = ((cnt - 1) / 16) * 16; g0 >= 0; g0 -= 16) {
#pragma unroll
                    for (int p = 0; p < kQuad; ++p) limg[p] = lim[p] - g0;
                    const float4 *gb = rb + 2 * g0;
                    float4 a0 = gb[2 * 15], a1 = gb[2 * 15 + 1];
#pragma unroll
                    for (int jj = 15; jj >= 0; --jj) {
                        float4 c0 = a0, c1 = a1;
                        if (jj > 0) { c0 = gb[2 * (jj - 1)]; c1 = gb[2 * (jj - 1) + 1]; }
                        splat(a0, a1, jj, g0 + jj);
                        a0 = c0; a1 = c1;
                    }
                }
#pragma unroll
                for (int p = 0; p < kQuad; ++p) lim[p] += kCompLanes;   // the previous chunk
                if (!more) break;
                cbeg -= kCompLanes;
                par ^= 1;
            }
        }
        if (nslots > 0) {
            __syncthreads();
            flush_slots(s_part, s_ids, slotj, nslots, b.grad, lane);
            __syncthreads();
        }
        w = pop_tile(b.queue);
    }
}

static uint32_t persistent_grid(uint32_t tiles, uint32_t per_cu) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    }
    const uint32_t g = (uint32_t)cus * per_cu;
    return tiles < g ? tiles : g;
}

template <bool COUNT, bool STATE>
static void launch_fwd(const CompositeArgs &a, bool persistent, hipStream_t st) {
    if (persistent) {
        hipLaunchKernelGGL((k_composite<true, COUNT, STATE>), dim3(persistent_grid(a.total_tiles, 8)),
                           dim3(kFwdThreads), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_composite<false, COUNT, STATE>), dim3(a.total_tiles), dim3(kFwdThreads), 0, st, a);
    }
}

hipError_t launch_composite_fwd(const CompositeArgs &a, bool persistent, hipStream_t st) {
    if (a.total_tiles == 0) return hipSuccess;
    // the blend count is kept only where the cap or the statistics need it,
    // the blend ends only where a backward follows
    const bool count = a.th.max_splats > 0 || (a.write_views && a.stats);
    const bool state = a.nlast != nullptr;
    if (count) state ? launch_fwd<true, true>(a, persistent, st) : launch_fwd<true, false>(a, persistent, st);
    else state ? launch_fwd<false, true>(a, persistent, st) : launch_fwd<false, false>(a, persistent, st);
    return hipGetLastError();
}

// Persistent, 16 waves per CU; the grid is sized from the tile count (the
// work-item count is read by the kernel itself).
hipError_t launch_composite_bwd(const BackwardArgs &b, hipStream_t st) {
    if (b.c.total_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_composite_bwd, dim3(persistent_grid(b.c.total_tiles, 16)), dim3(kCompLanes), 0, st, b);
    return hipGetLastError();
}

// Small host tables travel inside the kernel-argument buffer of this kernel,
// so their upload is ordered on the stream and never blocks the host (unlike
// a copy from pageable host memory).
constexpr int kUploadWords = 960;
struct UploadChunk {
    uint32_t nwords;
    uint32_t words[kUploadWords];
};

__global__ void k_upload(uint32_t *dst, UploadChunk c) {
    for (uint32_t i = threadIdx.x; i < c.nwords; i += blockDim.x) dst[i] = c.words[i];
}

hipError_t upload_async(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    const uint32_t *s = static_cast<const uint32_t *>(src);
    uint32_t *d = static_cast<uint32_t *>(dst);
    size_t n = bytes / 4;
    while (n > 0) {
        UploadChunk c;
        c.nwords = (uint32_t)(n < (size_t)kUploadWords ? n : (size_t)kUploadWords);
        for (uint32_t i = 0; i < c.nwords; ++i) c.words[i] = s[i];
        hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, st, d, c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        s += c.nwords;
        d += c.nwords;
        n -= c.nwords;
    }
    return hipSuccess;
}

// The same for a table of at most kUploadZeroWords words, in the one launch
// that also clears up to two word ranges (grid-stride).
constexpr int kUploadZeroWords = 896;
struct UploadZeroArgs {
    uint32_t *dst;
    uint32_t *z0, *z1;
    uint64_t n0, n1;
    uint32_t nwords;
    uint32_t words[kUploadZeroWords];
};

__global__ void k_upload_zero(UploadZeroArgs a) {
    if (blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < a.nwords; i += blockDim.x) a.dst[i] = a.words[i];
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t k = i0; k < a.n0; k += stride) a.z0[k] = 0u;
    for (uint64_t k = i0; k < a.n1; k += stride) a.z1[k] = 0u;
}

hipError_t upload_zero_async(void *dst, const void *src, size_t bytes, uint32_t *z0, uint64_t n0, uint32_t *z1,
                             uint64_t n1, hipStream_t st) {
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    if (bytes / 4 > (size_t)kUploadZeroWords) {
        hipError_t e = upload_async(dst, src, bytes, st);
        if (e == hipSuccess && n0) e = launch_fill_u32(z0, 0u, n0, st);
        if (e == hipSuccess && n1) e = launch_fill_u32(z1, 0u, n1, st);
        return e;
    }
    UploadZeroArgs a;
    a.dst = static_cast<uint32_t *>(dst);
    a.z0 = z0;
    a.z1 = z1;
    a.n0 = z0 ? n0 : 0;
    a.n1 = z1 ? n1 : 0;
    a.nwords = (uint32_t)(bytes / 4);
    memcpy(a.words, src, bytes);
    const uint64_t big = a.n0 > a.n1 ? a.n0 : a.n1;
    const uint64_t blocks = (big + 4ull * 256 - 1) / (4ull * 256);
    const uint32_t grid = (uint32_t)(blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks));
    hipLaunchKernelGGL(k_upload_zero, dim3(grid), dim3(256), 0, st, a);
    return hipGetLastError();
}

// The thread's pinned word and event for count read-backs (a pageable
// destination would go through the runtime's staging buffer).
namespace {
struct CountSlot {
    uint64_t *pinned = nullptr;
    hipEvent_t ev = nullptr;
};
thread_local CountSlot t_count;

hipError_t count_slot() {
    if (!t_count.pinned) {
        void *h = nullptr;
        const hipError_t e = hipHostMalloc(&h, 64, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        t_count.pinned = static_cast<uint64_t *>(h);
    }
    if (!t_count.ev) return hipEventCreateWithFlags(&t_count.ev, hipEventDisableTiming);
    return hipSuccess;
}
}  // namespace

hipError_t read_count(const uint64_t *dev, uint64_t *out, hipStream_t st) {
    hipError_t e = count_slot();
    if (e == hipSuccess) e = hipMemcpyAsync(t_count.pinned, dev, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) *out = *t_count.pinned;
    return e;
}

hipError_t read_count_begin(const uint64_t *dev, hipStream_t st) {
    hipError_t e = count_slot();
    if (e == hipSuccess) e = hipMemcpyAsync(t_count.pinned, dev, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(t_count.ev, st);
    return e;
}

hipError_t read_count_end(uint64_t *out) {
    const hipError_t e = hipEventSynchronize(t_count.ev);
    if (e == hipSuccess) *out = *t_count.pinned;
    return e;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t value, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t k = i; k < n; k += stride) p[k] = value;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, st, p, value, n);
    return hipGetLastError();
}

}  // namespace dpr
