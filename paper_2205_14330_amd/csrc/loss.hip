// The training loss of Eq. (8) for a batch of rendered images and its
// gradient, fused in one pass:
//   L_v = sum_{x,y,c} (R - I)^2 + lambda (sum |R(x+1,y) - R(x,y)| + sum |R(x,y+1) - R(x,y)|)
// (squared L2 plus lambda times the anisotropic total variation, forward
// differences between horizontally and vertically adjacent pixels, Sec. 3.3),
// and dL/dR = 2 (R - I) + lambda (s(R - R_left) - s(R_right - R) + s(R - R_up)
// - s(R_down - R)) with s = sign, s(0) = 0, terms dropped at the border.
//
// An image is a flat array of 3 W H floats; its horizontal neighbours are 3
// floats away and its vertical ones 3 W.  Each thread owns 4 consecutive
// floats and reads them, their horizontal neighbourhood, the target and (when
// 3 W is a multiple of 4) the rows above and below as aligned 16-byte loads;
// the gradient is written as one 16-byte store.  The loss terms of a float are
// its squared difference and its differences to the right and lower
// neighbours; a block sums them in FP32, and a second kernel adds each
// image's block sums in FP64 in a fixed order, so the result does not depend
// on scheduling.  With lambda = 0 (the plain L2 loss) no neighbour is read.  Up to kLossBatch images travel in the kernel arguments.
#include "dpr_internal.h"

namespace dpr {

constexpr int kLossThreads = 256;
constexpr int kLossFloats = 4 * kLossThreads;     // floats per block

struct LossBatch {
    LossImage img[kLossBatch];
    uint32_t block_start[kLossBatch + 1];
    int32_t n;
    float lambda;
    float *partial;      // [block_start[n]]
    double *loss;        // [n]
};

__device__ __forceinline__ float sgn(float d) { return (float)(d > 0.f) - (float)(d < 0.f); }

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }

__device__ __forceinline__ float at(const float4 &v, int k) {
    return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w;
}

__global__ __launch_bounds__(kLossThreads) void k_loss(LossBatch bt) {
    __shared__ float s_sum[kLossThreads / 64];
    int v = 0;
    while (v + 1 < bt.n && bt.block_start[v + 1] <= blockIdx.x) ++v;
    const LossImage im = bt.img[v];
    const int W = im.width, H = im.height;
    const int64_t nf = 3ll * W * H;
    const int64_t row = 3ll * W;
    const int64_t i = ((int64_t)(blockIdx.x - bt.block_start[v]) * kLossThreads + threadIdx.x) * 4;
    const float lambda = bt.lambda;
    float acc = 0.f;
    if (i < nf) {
        const float *R = im.render, *T = im.target;
        const bool vec = i + 4 <= nf && (((uintptr_t)R | (uintptr_t)T | (uintptr_t)im.grad) & 15) == 0;
        const bool vrow = vec && (row & 3) == 0;
        // first float's pixel and channel; the 4 floats span at most 2 pixels
        const int64_t p0 = i / 3;
        const int c0 = (int)(i - 3 * p0);
        const int y0 = (int)(p0 / W), x0 = (int)(p0 - (int64_t)y0 * W);
        float4 r, t, up, dn, lf, rt;
        if (vec) {
            r = ld4(R + i);
            t = ld4(T + i);
            lf = rt = up = dn = make_float4(0.f, 0.f, 0.f, 0.f);
            if (lambda != 0.f) {                      // the neighbours enter only the TV term
                if (i >= 4) lf = ld4(R + i - 4);
                if (i + 8 <= nf) {
                    rt = ld4(R + i + 4);
                } else {                              // the image ends inside the next group
                    rt.x = i + 4 < nf ? R[i + 4] : 0.f;
                    rt.y = i + 5 < nf ? R[i + 5] : 0.f;
                    rt.z = i + 6 < nf ? R[i + 6] : 0.f;
                    rt.w = 0.f;                       // i + 7: only e + 3 <= i + 6 is ever read
                }
                if (vrow) {
                    if (i >= row) up = ld4(R + i - row);
                    if (i + row + 4 <= nf) dn = ld4(R + i + row);
                }
            }
        }
        float g[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t e = i + k;
            if (e >= nf) { g[k] = 0.f; continue; }
            const int c = c0 + k;
            const bool next = c >= 3;                 // second pixel of the group
            int x = x0 + (next ? 1 : 0), y = y0;
            if (x == W) { x = 0; ++y; }
            float Rv, Tv, Rl = 0.f, Rr = 0.f, Ru = 0.f, Rd = 0.f;
            if (vec) {
                Rv = at(r, k);
                Tv = at(t, k);
                // e - 3 is float k - 3 of the group: k >= 3 in r, else float k + 1 of lf
                Rl = k >= 3 ? at(r, k - 3) : at(lf, k + 1);
                // e + 3: float k + 3 of the group: k == 0 in r, else float k - 1 of rt
                Rr = k == 0 ? at(r, 3) : at(rt, k - 1);
                if (vrow) { Ru = at(up, k); Rd = at(dn, k); }
                else if (lambda != 0.f) {
                    if (y > 0) Ru = R[e - row];
                    if (y + 1 < H) Rd = R[e + row];
                }
            } else {
                Rv = R[e];
                Tv = T[e];
                if (x > 0) Rl = R[e - 3];
                if (x + 1 < W) Rr = R[e + 3];
                if (y > 0) Ru = R[e - row];
                if (y + 1 < H) Rd = R[e + row];
            }
            const float d = Rv - Tv;
            float gr = 2.f * d;
            acc = fmaf(d, d, acc);
            if (x + 1 < W) {
                const float dx = Rr - Rv;
                acc = fmaf(lambda, fabsf(dx), acc);
                gr -= lambda * sgn(dx);
            }
            if (x > 0) gr += lambda * sgn(Rv - Rl);
            if (y + 1 < H) {
                const float dy = Rd - Rv;
                acc = fmaf(lambda, fabsf(dy), acc);
                gr -= lambda * sgn(dy);
            }
            if (y > 0) gr += lambda * sgn(Rv - Ru);
            g[k] = gr;
        }
        if (vec) {
            *reinterpret_cast<float4 *>(im.grad + i) = make_float4(g[0], g[1], g[2], g[3]);
        } else {
            for (int k = 0; k < 4 && i + k < nf; ++k) im.grad[i + k] = g[k];
        }
    }
    // block sum: within each wave, then across the 4 waves in a fixed order
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) bt.partial[blockIdx.x] = (s_sum[0] + s_sum[1]) + (s_sum[2] + s_sum[3]);
}

// One block of kLossSumThreads per image: thread l adds block sums l,
// l + kLossSumThreads, ... in FP64, then a fixed butterfly in each wave and a
// fixed order across the waves combine them.
constexpr int kLossSumThreads = 256;

__global__ __launch_bounds__(kLossSumThreads) void k_loss_sum(LossBatch bt) {
    __shared__ double s_w[kLossSumThreads / 64];
    const int v = blockIdx.x;
    const uint32_t b0 = bt.block_start[v], b1 = bt.block_start[v + 1];
    double s = 0.0;
#pragma unroll 8
    for (uint32_t b = b0 + threadIdx.x; b < b1; b += kLossSumThreads) s += (double)bt.partial[b];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) bt.loss[v] = (s_w[0] + s_w[1]) + (s_w[2] + s_w[3]);
}

uint32_t loss_blocks(int32_t width, int32_t height) {
    const uint64_t nf = 3ull * (uint64_t)width * (uint64_t)height;
    return (uint32_t)((nf + kLossFloats - 1) / kLossFloats);
}

hipError_t launch_loss(const LossImage *img, int n, float lambda, float *partial, double *loss, hipStream_t st) {
    for (int b0 = 0; b0 < n; b0 += kLossBatch) {
        LossBatch bt;
        bt.n = n - b0 < kLossBatch ? n - b0 : kLossBatch;
        bt.lambda = lambda;
        uint32_t blocks = 0;
        for (int v = 0; v < bt.n; ++v) {
            bt.img[v] = img[b0 + v];
            bt.block_start[v] = blocks;
            blocks += loss_blocks(img[b0 + v].width, img[b0 + v].height);
        }
        bt.block_start[bt.n] = blocks;
        bt.partial = partial;
        bt.loss = loss + b0;
        hipLaunchKernelGGL(k_loss, dim3(blocks), dim3(kLossThreads), 0, st, bt);
        hipLaunchKernelGGL(k_loss_sum, dim3(bt.n), dim3(kLossSumThreads), 0, st, bt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace dpr
