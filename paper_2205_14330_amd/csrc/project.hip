// Projection, screen-space splat shape and SH colour of every (view, point)
// item (Sec. 3.1 Eq. 1-4), plus the depth key and the conservative tile
// rectangle of each splat's support (end of Sec. 3.2).
//
// One thread per scene point; it loops over every view of its scene, so the
// 128 bytes of per-point input (xyz, 27 SH floats, opacity, radius) are read
// from HBM once per point instead of once per view.  The SH rows of a block
// are staged through LDS with 16-byte loads so that each wave reads one
// contiguous span.
#include "dpr_internal.h"
#include "sh.h"

namespace dpr {

constexpr int kProjThreads = 128;

template <int DEG>
__global__ __launch_bounds__(kProjThreads) void k_project(Tables tb, Thresholds th, SplatRec *rec,
                                                          uint32_t *keys, uint32_t *vals, uint2 *rect) {
    extern __shared__ float s_sh[];
    const int s = find_segment(tb.scene_block_start, tb.n_scenes, blockIdx.x);
    const SceneDesc sc = tb.scenes[s];
    const int i0 = (int)(blockIdx.x - sc.block_off) * kProjThreads;
    const int i = i0 + (int)threadIdx.x;
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int row = 3 * K;
    constexpr int stride = row | 1;   // odd LDS stride: conflict-free per-thread reads

    // stage this block's SH rows [i0, i0 + 128) into LDS
    {
        const int npts = min(kProjThreads, sc.n - i0);
        const int total = npts * row;
        const float *src = sc.sh + (size_t)i0 * row;
        if ((((uintptr_t)src) & 15) == 0) {
            const int n4 = total >> 2;
            const float4 *src4 = reinterpret_cast<const float4 *>(src);
            for (int e = threadIdx.x; e < n4; e += kProjThreads) {
                float4 v = src4[e];
                int f = e * 4;
                s_sh[(f / row) * stride + f % row] = v.x; ++f;
                s_sh[(f / row) * stride + f % row] = v.y; ++f;
                s_sh[(f / row) * stride + f % row] = v.z; ++f;
                s_sh[(f / row) * stride + f % row] = v.w;
            }
            for (int f = n4 * 4 + threadIdx.x; f < total; f += kProjThreads)
                s_sh[(f / row) * stride + f % row] = src[f];
        } else {
            for (int f = threadIdx.x; f < total; f += kProjThreads)
                s_sh[(f / row) * stride + f % row] = src[f];
        }
    }
    __syncthreads();
    if (i >= sc.n) return;

    const float x = sc.xyz[3 * (size_t)i + 0];
    const float y = sc.xyz[3 * (size_t)i + 1];
    const float z = sc.xyz[3 * (size_t)i + 2];
    const float o = sc.opacity[i];
    const float r = sc.radius[i];
    const float log2o = __log2f(o);
    const float *h = s_sh + threadIdx.x * stride;

    for (uint32_t vv = 0; vv < sc.view_count; ++vv) {
        const ViewDesc &vd = tb.views[tb.scene_views[sc.view_start + vv]];
        const uint32_t g = vd.item_off + (uint32_t)i;
        const float Z = depth_z(vd.R, vd.t, x, y, z);
        const float X = vd.R[0] * x + vd.R[1] * y + vd.R[2] * z + vd.t[0];
        const float Yc = vd.R[3] * x + vd.R[4] * y + vd.R[5] * z + vd.t[1];

        SplatRec out;
        uint32_t key = kDroppedKey;
        uint2 rc = make_uint2(0u, 0u);
        out.px = out.py = out.a = out.b = 0.f;
        out.w = -INFINITY;
        out.cr = out.cg = out.cb = 0.f;
        if (Z > th.z_near) {
            const float iz = 1.0f / Z;
            out.px = vd.fx * X * iz + vd.cx;
            out.py = vd.fy * Yc * iz + vd.cy;
            const float sx = vd.fx * r * iz;
            const float sy = vd.fy * r * iz;
            out.a = (0.5f * kLog2e) / (sx * sx);
            out.b = (0.5f * kLog2e) / (sy * sy);
            // log2 of the amplitude: o, or o (2 pi sx sy)^-1/2 with Eq. (5)'s normalisation
            out.w = th.kernel_norm ? log2o - 0.5f * __log2f(kTwoPi * sx * sy) : log2o;

            // SH colour at the view direction (camera frame, or world frame)
            const float inrm = rsqrtf(X * X + Yc * Yc + Z * Z);
            float dx = X * inrm, dy = Yc * inrm, dz = Z * inrm;
            if (th.sh_frame == 1) {
                const float wx = vd.R[0] * dx + vd.R[3] * dy + vd.R[6] * dz;
                const float wy = vd.R[1] * dx + vd.R[4] * dy + vd.R[7] * dz;
                const float wz = vd.R[2] * dx + vd.R[5] * dy + vd.R[8] * dz;
                dx = wx; dy = wy; dz = wz;
            }
            float Yb[16];
            sh_values(DEG, dx, dy, dz, Yb);
            float c0 = 0.f, c1 = 0.f, c2 = 0.f;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                c0 = fmaf(h[3 * k + 0], Yb[k], c0);
                c1 = fmaf(h[3 * k + 1], Yb[k], c1);
                c2 = fmaf(h[3 * k + 2], Yb[k], c2);
            }
            out.cr = c0; out.cg = c1; out.cb = c2;

            // conservative tile rectangle of the ellipse a dx^2 + b dy^2 <= thr
            const float thr = out.w + th.lambda;   // candidate iff a dx^2 + b dy^2 <= thr
            if (thr >= 0.f && isfinite(out.px) && isfinite(out.py)) {
                const float slack = 1.0f + 1.0f / 1024.0f;
                const float hx = sqrtf(thr / out.a) * slack + (1.0f / 64.0f);
                const float hy = sqrtf(thr / out.b) * slack + (1.0f / 64.0f);
                // pixel centres x + 0.5 within [px - hx, px + hx]
                float fx0 = floorf(out.px - hx - 0.5f), fx1 = ceilf(out.px + hx - 0.5f);
                float fy0 = floorf(out.py - hy - 0.5f), fy1 = ceilf(out.py + hy - 0.5f);
                fx0 = fmaxf(fx0, 0.f); fy0 = fmaxf(fy0, 0.f);
                fx1 = fminf(fx1, (float)(vd.width - 1)); fy1 = fminf(fy1, (float)(vd.height - 1));
                if (fx0 <= fx1 && fy0 <= fy1) {
                    const uint32_t tx0 = (uint32_t)fx0 / kTile, tx1 = (uint32_t)fx1 / kTile + 1;
                    const uint32_t ty0 = (uint32_t)fy0 / kTile, ty1 = (uint32_t)fy1 / kTile + 1;
                    rc = make_uint2(tx0 | (ty0 << 16), tx1 | (ty1 << 16));
                    key = __float_as_uint(Z);
                }
            }
        }
        float4 *dst = reinterpret_cast<float4 *>(rec + g);
        dst[0] = make_float4(out.px, out.py, out.a, out.b);
        dst[1] = make_float4(out.w, out.cr, out.cg, out.cb);
        keys[g] = key;
        vals[g] = g;
        rect[g] = rc;
    }
}

hipError_t launch_project(const Tables &tb, const Thresholds &th, int sh_degree, uint32_t point_blocks,
                          SplatRec *rec, uint32_t *keys, uint32_t *vals, uint2 *rect,
                          hipStream_t st) {
    if (point_blocks == 0) return hipSuccess;
    const int row = 3 * (sh_degree + 1) * (sh_degree + 1);
    const size_t lds = (size_t)kProjThreads * (row | 1) * sizeof(float);
    switch (sh_degree) {
    case 0: hipLaunchKernelGGL(k_project<0>, dim3(point_blocks), dim3(kProjThreads), lds, st, tb, th, rec, keys, vals, rect); break;
    case 1: hipLaunchKernelGGL(k_project<1>, dim3(point_blocks), dim3(kProjThreads), lds, st, tb, th, rec, keys, vals, rect); break;
    case 2: hipLaunchKernelGGL(k_project<2>, dim3(point_blocks), dim3(kProjThreads), lds, st, tb, th, rec, keys, vals, rect); break;
    case 3: hipLaunchKernelGGL(k_project<3>, dim3(point_blocks), dim3(kProjThreads), lds, st, tb, th, rec, keys, vals, rect); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace dpr
