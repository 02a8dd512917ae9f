// Per-tile front-to-back compositing (Sec. 3.2, Eq. 5-7) and its reverse-mode
// derivative.
//
// One workgroup of 256 lanes (4 waves) per 16x16 tile, one pixel per lane.
// The tile's depth-ordered list is consumed in chunks of 256 splat records
// staged in LDS (each lane gathers one 32-byte record); every lane then walks
// the chunk from LDS.  A lane stops after the first blended splat that leaves
// T < t_min; the workgroup leaves the list as soon as no lane is active
// (__syncthreads_count), which also ends idle waves early.
//
// The backward walks the same list in reverse from the furthest stop index,
// recovering T_i = T_{i+1} / (1 - alpha_i) (alpha <= alpha_max < 1), keeps the
// back-to-front colour sum, and turns each (pixel, splat) contribution into 8
// partial sums.  Those are reduced across the 64 lanes of a wave, then across
// the 4 waves in LDS, and leave the workgroup as one float atomic per quantity
// per (tile, splat).
#include "dpr_internal.h"

namespace dpr {

constexpr int kCompThreads = kTilePix;   // 256

struct TileCtx {
    uint32_t start, end;       // list range in pairs[]
    int32_t px, py;            // this lane's pixel
    bool inside;
    uint64_t pix;              // index into per-pixel state arrays (global)
    uint64_t lpix;             // pixel index within the view
    int v;                     // view
};

__device__ __forceinline__ TileCtx tile_ctx(const CompositeArgs &a, uint32_t tile) {
    TileCtx c;
    c.v = find_segment(a.tile_start, a.n_views, tile);
    const ViewDesc &vd = a.views[c.v];
    const uint32_t lt = tile - vd.tile_off;
    const uint32_t ty = lt / (uint32_t)vd.tiles_x;
    const uint32_t tx = lt - ty * (uint32_t)vd.tiles_x;
    c.px = (int)(tx * kTile + (threadIdx.x & (kTile - 1)));
    c.py = (int)(ty * kTile + (threadIdx.x >> 4));
    c.inside = c.px < vd.width && c.py < vd.height;
    const uint64_t rb = vd.cnt_off + (uint64_t)lt * vd.nchunks;
    c.start = a.range[rb];
    c.end = a.range[rb + vd.nchunks];
    c.lpix = (uint64_t)c.py * (uint64_t)vd.width + (uint64_t)c.px;
    c.pix = vd.pix_off + c.lpix;
    return c;
}

__device__ __forceinline__ float splat_alpha(float e, float alpha_max, bool &clamped) {
    const float g = __builtin_amdgcn_exp2f(e);
    clamped = g > alpha_max;
    return clamped ? alpha_max : g;
}

// next tile for persistent workgroups (thread 0 pops, broadcast through LDS)
__device__ __forceinline__ uint32_t pop_tile(uint32_t *queue, uint32_t *s_next) {
    __syncthreads();
    if (threadIdx.x == 0) *s_next = atomicAdd(queue, 1u) + gridDim.x;
    __syncthreads();
    return *s_next;
}

// ---------------------------------------------------------------------------
// forward (COLOR = true) and recompute of the per-pixel state (COLOR = false)
// ---------------------------------------------------------------------------
template <bool COLOR, bool PERSISTENT>
__global__ __launch_bounds__(kCompThreads) void k_composite(CompositeArgs a) {
    __shared__ SplatRec s_rec[kCompThreads];
    __shared__ uint32_t s_next;
    const float neg_lambda = -a.th.lambda;
    for (uint32_t tile = blockIdx.x; tile < a.total_tiles;) {
        const TileCtx c = tile_ctx(a, tile);
        const float ux = (float)c.px + 0.5f, uy = (float)c.py + 0.5f;
        float T = 1.0f, I0 = 0.f, I1 = 0.f, I2 = 0.f;
        uint32_t nlast = 0, nblend = 0;
        bool done = !c.inside;
        for (uint32_t base = c.start; base < c.end; base += kCompThreads) {
            const uint32_t k = base + threadIdx.x;
            if (k < c.end) {
                const float4 *src = reinterpret_cast<const float4 *>(a.rec + a.pairs[k]);
                float4 *dst = reinterpret_cast<float4 *>(&s_rec[threadIdx.x]);
                dst[0] = src[0];
                dst[1] = src[1];
            }
            __syncthreads();
            const uint32_t cnt = min((uint32_t)kCompThreads, c.end - base);
            if (!done) {
                for (uint32_t j = 0; j < cnt; ++j) {
                    const SplatRec &s = s_rec[j];
                    float dx, dy;
                    const float e = splat_exponent(s, ux, uy, dx, dy);
                    if (e < neg_lambda) continue;
                    bool clamped;
                    const float alpha = splat_alpha(e, a.th.alpha_max, clamped);
                    if (COLOR) {
                        const float Ta = T * alpha;
                        I0 = fmaf(Ta, s.cr, I0);
                        I1 = fmaf(Ta, s.cg, I1);
                        I2 = fmaf(Ta, s.cb, I2);
                    }
                    T = T * (1.0f - alpha);
                    ++nblend;
                    if (T < a.th.t_min) {
                        done = true;
                        nlast = base - c.start + j + 1;
                        break;
                    }
                }
            }
            if (__syncthreads_count(!done) == 0) break;
        }
        if (c.inside) {
            if (!done) nlast = c.end - c.start;
            const ViewDesc &vd = a.views[c.v];
            if (COLOR) {
                float *img = vd.image + 3 * c.lpix;
                img[0] = I0; img[1] = I1; img[2] = I2;
                if (vd.trans) vd.trans[c.lpix] = T;
                if (a.stats) a.stats[c.pix] = nblend;
            } else {
                a.tfinal[c.pix] = T;
            }
            if (a.nlast) a.nlast[c.pix] = nlast;
        }
        if (!PERSISTENT) break;
        tile = pop_tile(a.queue, &s_next);
    }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

template <bool PERSISTENT>
__global__ __launch_bounds__(kCompThreads) void k_composite_bwd(BackwardArgs b) {
    __shared__ SplatRec s_rec[kCompThreads];
    __shared__ uint32_t s_id[kCompThreads];
    __shared__ float s_acc[8][kCompThreads];
    __shared__ uint32_t s_max[kCompThreads / 64];
    __shared__ uint32_t s_next;
    const CompositeArgs &a = b.c;
    const float neg_lambda = -a.th.lambda;
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;

    for (uint32_t tile = blockIdx.x; tile < a.total_tiles;) {
        const TileCtx c = tile_ctx(a, tile);
        const ViewDesc &vd = a.views[c.v];
        const float ux = (float)c.px + 0.5f, uy = (float)c.py + 0.5f;
        uint32_t nl = 0;
        float T = 1.0f, gI0 = 0.f, gI1 = 0.f, gI2 = 0.f, gT = 0.f;
        if (c.inside) {
            nl = b.nlast[c.pix];
            T = b.tfinal_from_views ? vd.trans[c.lpix] : b.tfinal[c.pix];
            const float *gi = b.dimage[c.v] + 3 * c.lpix;
            gI0 = gi[0]; gI1 = gi[1]; gI2 = gi[2];
            if (b.dtrans && b.dtrans[c.v]) gT = b.dtrans[c.v][c.lpix];
        }
        const float Tfin = T;
        float B0 = 0.f, B1 = 0.f, B2 = 0.f;      // sum over blended splats behind of T_k alpha_k c_k

        // furthest stop index of the tile
        uint32_t m = nl;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d, 64));
        if (lane == 0) s_max[wave] = m;
        __syncthreads();
        uint32_t maxn = 0;
        for (int w = 0; w < kCompThreads / 64; ++w) maxn = max(maxn, s_max[w]);

        for (uint32_t cend = c.start + maxn; cend > c.start;) {
            const uint32_t cbeg = cend - c.start > (uint32_t)kCompThreads ? cend - kCompThreads : c.start;
            const uint32_t cnt = cend - cbeg;
            __syncthreads();
            if (threadIdx.x < cnt) {
                const uint32_t id = a.pairs[cbeg + threadIdx.x];
                s_id[threadIdx.x] = id;
                const float4 *src = reinterpret_cast<const float4 *>(a.rec + id);
                float4 *dst = reinterpret_cast<float4 *>(&s_rec[threadIdx.x]);
                dst[0] = src[0];
                dst[1] = src[1];
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) s_acc[q][threadIdx.x] = 0.f;
            __syncthreads();
            for (int j = (int)cnt - 1; j >= 0; --j) {
                const uint32_t pos = cbeg - c.start + (uint32_t)j;
                float v0 = 0.f, v1 = 0.f, v2 = 0.f, v3 = 0.f, v4 = 0.f, v5 = 0.f, v6 = 0.f, v7 = 0.f;
                bool hit = false;
                if (pos < nl) {
                    const SplatRec &s = s_rec[j];
                    float dx, dy;
                    const float e = splat_exponent(s, ux, uy, dx, dy);
                    if (e >= neg_lambda) {
                        hit = true;
                        bool clamped;
                        const float alpha = splat_alpha(e, a.th.alpha_max, clamped);
                        const float om = 1.0f - alpha;
                        const float iom = 1.0f / om;
                        T = T * iom;                         // T in front of this splat
                        const float Ta = T * alpha;
                        const float dA = gI0 * (T * s.cr - B0 * iom) + gI1 * (T * s.cg - B1 * iom) +
                                         gI2 * (T * s.cb - B2 * iom) - gT * Tfin * iom;
                        v5 = Ta * gI0; v6 = Ta * gI1; v7 = Ta * gI2;
                        B0 = fmaf(Ta, s.cr, B0);
                        B1 = fmaf(Ta, s.cg, B1);
                        B2 = fmaf(Ta, s.cb, B2);
                        if (!clamped) {
                            const float gw = dA * alpha * kLn2;    // dL/dw; dL/dq = -gw
                            v4 = gw;
                            v0 = gw * dx;
                            v1 = gw * dy;
                            v2 = v0 * dx;
                            v3 = v1 * dy;
                        }
                    }
                }
                if (__ballot(hit) != 0ull) {
                    v0 = wave_sum_f32(v0); v1 = wave_sum_f32(v1);
                    v2 = wave_sum_f32(v2); v3 = wave_sum_f32(v3);
                    v4 = wave_sum_f32(v4); v5 = wave_sum_f32(v5);
                    v6 = wave_sum_f32(v6); v7 = wave_sum_f32(v7);
                    if (lane == 0) {
                        atomicAdd(&s_acc[0][j], v0); atomicAdd(&s_acc[1][j], v1);
                        atomicAdd(&s_acc[2][j], v2); atomicAdd(&s_acc[3][j], v3);
                        atomicAdd(&s_acc[4][j], v4); atomicAdd(&s_acc[5][j], v5);
                        atomicAdd(&s_acc[6][j], v6); atomicAdd(&s_acc[7][j], v7);
                    }
                }
            }
            __syncthreads();
            if (threadIdx.x < cnt) {
                float *gdst = b.grad + 8 * (size_t)s_id[threadIdx.x];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const float v = s_acc[q][threadIdx.x];
                    if (v != 0.f) atomicAdd(gdst + q, v);
                }
            }
            cend = cbeg;
        }
        if (!PERSISTENT) break;
        tile = pop_tile(a.queue, &s_next);
    }
}

static uint32_t persistent_grid(uint32_t tiles) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) {
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
    }
    const uint32_t g = (uint32_t)cus * 8u;
    return tiles < g ? tiles : g;
}

hipError_t launch_composite_fwd(const CompositeArgs &a, bool persistent, hipStream_t st) {
    if (a.total_tiles == 0) return hipSuccess;
    if (persistent) {
        hipLaunchKernelGGL((k_composite<true, true>), dim3(persistent_grid(a.total_tiles)), dim3(kCompThreads), 0,
                           st, a);
    } else {
        hipLaunchKernelGGL((k_composite<true, false>), dim3(a.total_tiles), dim3(kCompThreads), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_recompute(const CompositeArgs &a, bool persistent, hipStream_t st) {
    if (a.total_tiles == 0) return hipSuccess;
    if (persistent) {
        hipLaunchKernelGGL((k_composite<false, true>), dim3(persistent_grid(a.total_tiles)), dim3(kCompThreads), 0,
                           st, a);
    } else {
        hipLaunchKernelGGL((k_composite<false, false>), dim3(a.total_tiles), dim3(kCompThreads), 0, st, a);
    }
    return hipGetLastError();
}

hipError_t launch_composite_bwd(const BackwardArgs &b, bool persistent, hipStream_t st) {
    if (b.c.total_tiles == 0) return hipSuccess;
    if (persistent) {
        hipLaunchKernelGGL((k_composite_bwd<true>), dim3(persistent_grid(b.c.total_tiles)), dim3(kCompThreads), 0,
                           st, b);
    } else {
        hipLaunchKernelGGL((k_composite_bwd<false>), dim3(b.c.total_tiles), dim3(kCompThreads), 0, st, b);
    }
    return hipGetLastError();
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
