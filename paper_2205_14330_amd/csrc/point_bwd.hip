// Per-point chain rule from the per-(view, point) splat gradients to the
// scene parameters: positions through Eq. (1) and the perspective-scaled
// radius, SH coefficients through Eq. (4), the view direction through Eq. (3),
// and the opacity through w = log2(o) (plus log2 (2 pi sx sy)^-1/2 with Eq. (5)'s
// normalisation, which adds dL/dZ = A4 / Z).
//
// One thread per scene point loops over the scene's views in a fixed order,
// so the sum over views is deterministic and each output is written once.  A
// block's SH rows are read into LDS with 16-byte loads, and its SH gradients
// leave through the same LDS rows, so each wave touches contiguous spans.
//
// Gradient record of an item (accumulated by the compositing backward), with
// gw = (dL/de) / ln 2 per (pixel, splat), e = w - q, q = a dx^2 + b dy^2,
// dx = px - ux:
//   A0 = sum gw dx, A1 = sum gw dy, A2 = sum gw q, A3 = 0, A4 = sum gw, A5..A7 = dL/dc.
// Hence dL/dw = ln2 A4, dL/dpx = -2a ln2 A0, dL/dpy = -2b ln2 A1, and since a and
// b scale as Z^2, the part of dL/dZ through the splat shape is -(2 ln2 / Z) A2.
#include "dpr_internal.h"
#include "sh.h"

namespace dpr {

constexpr int kPointThreads = 128;

// The block's rows [i0, i0 + npts) of row floats, held in LDS rows of the odd
// stride row | 1 (conflict-free per-thread access), are moved from or to
// global memory with 16-byte accesses when the span is aligned.
__device__ __forceinline__ int lds_index(int f, int row) { return (f / row) * (row | 1) + f % row; }

__device__ __forceinline__ void load_rows(float *s_rows, const float *g, int npts, int row) {
    const int total = npts * row;
    int f0 = 0;
    if ((((uintptr_t)g) & 15) == 0) {
        const int n4 = total >> 2;
        const float4 *g4 = reinterpret_cast<const float4 *>(g);
        for (int e = threadIdx.x; e < n4; e += kPointThreads) {
            const float4 v = g4[e];
            s_rows[lds_index(4 * e + 0, row)] = v.x;
            s_rows[lds_index(4 * e + 1, row)] = v.y;
            s_rows[lds_index(4 * e + 2, row)] = v.z;
            s_rows[lds_index(4 * e + 3, row)] = v.w;
        }
        f0 = n4 * 4;
    }
    for (int f = f0 + threadIdx.x; f < total; f += kPointThreads) s_rows[lds_index(f, row)] = g[f];
}

__device__ __forceinline__ void store_rows(const float *s_rows, float *g, int npts, int row) {
    const int total = npts * row;
    int f0 = 0;
    if ((((uintptr_t)g) & 15) == 0) {
        const int n4 = total >> 2;
        float4 *g4 = reinterpret_cast<float4 *>(g);
        for (int e = threadIdx.x; e < n4; e += kPointThreads)
            g4[e] = make_float4(s_rows[lds_index(4 * e + 0, row)], s_rows[lds_index(4 * e + 1, row)],
                                s_rows[lds_index(4 * e + 2, row)], s_rows[lds_index(4 * e + 3, row)]);
        f0 = n4 * 4;
    }
    for (int f = f0 + threadIdx.x; f < total; f += kPointThreads) g[f] = s_rows[lds_index(f, row)];
}

template <int DEG>
__global__ __launch_bounds__(kPointThreads) void k_point_bwd(Tables tb, Thresholds th, const float *grad) {
    extern __shared__ float s_sh[];
    const int s = find_segment(tb.scene_block_start, tb.n_scenes, blockIdx.x);
    const SceneDesc sc = tb.scenes[s];
    const int i0 = (int)(blockIdx.x - sc.block_off) * kPointThreads;
    const int i = i0 + (int)threadIdx.x;
    constexpr int deg = DEG;
    constexpr int K = (DEG + 1) * (DEG + 1);
    constexpr int row = 3 * K;
    const int npts = min(kPointThreads, sc.n - i0);
    load_rows(s_sh, sc.sh + (size_t)i0 * row, npts, row);
    __syncthreads();
    if (i < sc.n) {
        const float x = sc.xyz[3 * (size_t)i + 0];
        const float y = sc.xyz[3 * (size_t)i + 1];
        const float z = sc.xyz[3 * (size_t)i + 2];
        const float o = sc.opacity[i];
        const float r = sc.radius[i];
        float *const h = s_sh + threadIdx.x * (row | 1);

        float gP0 = 0.f, gP1 = 0.f, gP2 = 0.f, gO = 0.f;
        float gH[3 * K];
#pragma unroll
        for (int k = 0; k < 3 * K; ++k) gH[k] = 0.f;

        for (uint32_t vv = 0; vv < sc.view_count; ++vv) {
            const ViewDesc &vd = tb.views[tb.scene_views[sc.view_start + vv]];
            const uint32_t g = vd.item_off + (uint32_t)i;
            const float Z = depth_z(vd.R, vd.t, x, y, z);
            if (!(Z > th.z_near)) continue;
            const float4 ga = reinterpret_cast<const float4 *>(grad + 8 * (size_t)g)[0];
            const float4 gb = reinterpret_cast<const float4 *>(grad + 8 * (size_t)g)[1];
            if (ga.x == 0.f && ga.y == 0.f && ga.z == 0.f && ga.w == 0.f && gb.x == 0.f && gb.y == 0.f &&
                gb.z == 0.f && gb.w == 0.f)
                continue;
            const float X = vd.R[0] * x + vd.R[1] * y + vd.R[2] * z + vd.t[0];
            const float Yc = vd.R[3] * x + vd.R[4] * y + vd.R[5] * z + vd.t[1];
            const float iz = 1.0f / Z;
            const float sx = vd.fx * r * iz, sy = vd.fy * r * iz;
            const float a = (0.5f * kLog2e) / (sx * sx);
            const float bb = (0.5f * kLog2e) / (sy * sy);

            const float g_px = -2.f * kLn2 * a * ga.x;
            const float g_py = -2.f * kLn2 * bb * ga.y;
            const float g_w = kLn2 * gb.x;
            const float gc0 = gb.y, gc1 = gb.z, gc2 = gb.w;

            // projection px = fx X/Z + cx, py = fy Y/Z + cy; a, b ~ Z^2
            float dX = g_px * vd.fx * iz;
            float dY = g_py * vd.fy * iz;
            float dZ = -(g_px * vd.fx * X + g_py * vd.fy * Yc) * iz * iz - 2.f * kLn2 * ga.z * iz;
            // with Eq. (5)'s normalisation w = log2 o - log2 sqrt(2 pi sx sy) grows as log2 Z
            if (th.kernel_norm) dZ += gb.x * iz;
            // opacity: w = log2(o)
            gO += g_w / (o * kLn2);

            // colour: c = sum_k h_k Y_k(d), d = v (camera) or R^T v (world), v = X/|X|
            const float inrm = rsqrtf(X * X + Yc * Yc + Z * Z);
            const float v0 = X * inrm, v1 = Yc * inrm, v2 = Z * inrm;
            float d0 = v0, d1 = v1, d2 = v2;
            if (th.sh_frame == 1) {
                d0 = vd.R[0] * v0 + vd.R[3] * v1 + vd.R[6] * v2;
                d1 = vd.R[1] * v0 + vd.R[4] * v1 + vd.R[7] * v2;
                d2 = vd.R[2] * v0 + vd.R[5] * v1 + vd.R[8] * v2;
            }
            float Yb[16], wk[16];
            sh_values(deg, d0, d1, d2, Yb);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                gH[3 * k + 0] = fmaf(Yb[k], gc0, gH[3 * k + 0]);
                gH[3 * k + 1] = fmaf(Yb[k], gc1, gH[3 * k + 1]);
                gH[3 * k + 2] = fmaf(Yb[k], gc2, gH[3 * k + 2]);
                wk[k] = gc0 * h[3 * k + 0] + gc1 * h[3 * k + 1] + gc2 * h[3 * k + 2];
            }
            float gd0, gd1, gd2;
            sh_grad_dot(deg, d0, d1, d2, wk, gd0, gd1, gd2);
            float gv0 = gd0, gv1 = gd1, gv2 = gd2;
            if (th.sh_frame == 1) {
                gv0 = vd.R[0] * gd0 + vd.R[1] * gd1 + vd.R[2] * gd2;
                gv1 = vd.R[3] * gd0 + vd.R[4] * gd1 + vd.R[5] * gd2;
                gv2 = vd.R[6] * gd0 + vd.R[7] * gd1 + vd.R[8] * gd2;
            }
            const float vdot = v0 * gv0 + v1 * gv1 + v2 * gv2;
            dX += (gv0 - v0 * vdot) * inrm;
            dY += (gv1 - v1 * vdot) * inrm;
            dZ += (gv2 - v2 * vdot) * inrm;

            // X_cam = R P + t  ->  dP = R^T dX_cam
            gP0 += vd.R[0] * dX + vd.R[3] * dY + vd.R[6] * dZ;
            gP1 += vd.R[1] * dX + vd.R[4] * dY + vd.R[7] * dZ;
            gP2 += vd.R[2] * dX + vd.R[5] * dY + vd.R[8] * dZ;
        }
        if (sc.dxyz) {
            sc.dxyz[3 * (size_t)i + 0] = gP0;
            sc.dxyz[3 * (size_t)i + 1] = gP1;
            sc.dxyz[3 * (size_t)i + 2] = gP2;
        }
        if (sc.dopacity) sc.dopacity[i] = gO;
        if (sc.dsh) {
            // the row's SH values are no longer read: it takes the gradients
#pragma unroll
            for (int k = 0; k < 3 * K; ++k) h[k] = gH[k];
        }
    }
    __syncthreads();
    if (sc.dsh) store_rows(s_sh, sc.dsh + (size_t)i0 * row, npts, row);
}

hipError_t launch_point_bwd(const Tables &tb, const Thresholds &th, int sh_degree, uint32_t point_blocks,
                            const float *grad, hipStream_t st) {
    if (point_blocks == 0) return hipSuccess;
    auto lds = [](int d) { return (size_t)kPointThreads * ((3 * (d + 1) * (d + 1)) | 1) * sizeof(float); };
    switch (sh_degree) {
    case 0: hipLaunchKernelGGL(k_point_bwd<0>, dim3(point_blocks), dim3(kPointThreads), lds(0), st, tb, th, grad); break;
    case 1: hipLaunchKernelGGL(k_point_bwd<1>, dim3(point_blocks), dim3(kPointThreads), lds(1), st, tb, th, grad); break;
    case 2: hipLaunchKernelGGL(k_point_bwd<2>, dim3(point_blocks), dim3(kPointThreads), lds(2), st, tb, th, grad); break;
    case 3: hipLaunchKernelGGL(k_point_bwd<3>, dim3(point_blocks), dim3(kPointThreads), lds(3), st, tb, th, grad); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace dpr
