// The training loss of Eq. (8) for a batch of rendered images and its
// gradient, fused in one pass over the pixels:
//   L_v = sum_{x,y,c} (R - I)^2 + lambda (sum |R(x+1,y) - R(x,y)| + sum |R(x,y+1) - R(x,y)|)
// (squared L2 plus lambda times the anisotropic total variation, forward
// differences between horizontally and vertically adjacent pixels, Sec. 3.3).
//
// Each thread owns whole pixels and writes their gradient, reading the four
// neighbours (the same lines are read by the neighbouring lanes, so HBM sees
// each image once): dL/dR = 2 (R - I) + lambda (s(R - R_left) - s(R_right - R)
// + s(R - R_up) - s(R_down - R)) with s = sign and s(0) = 0, terms dropped at
// the border.  The loss terms of a pixel are its squared difference and the
// two differences to its right and lower neighbours; a block sums them in
// FP32, and a second kernel adds each image's block sums in FP64 in a fixed
// order, so the result does not depend on scheduling.
#include "dpr_internal.h"

namespace dpr {

constexpr int kLossThreads = 256;
constexpr int kLossPix = 4 * kLossThreads;     // pixels per block

__device__ __forceinline__ float sgn(float d) { return (float)(d > 0.f) - (float)(d < 0.f); }

__global__ __launch_bounds__(kLossThreads) void k_loss(const LossImage *img, const uint32_t *block_start, int n,
                                                       float lambda, float *partial) {
    __shared__ float s_sum[kLossThreads / 64];
    const int v = find_segment(block_start, n, blockIdx.x);
    const LossImage im = img[v];
    const int W = im.width, H = im.height;
    const uint64_t npix = (uint64_t)W * (uint64_t)H;
    const uint64_t p0 = (uint64_t)(blockIdx.x - block_start[v]) * kLossPix;
    float acc = 0.f;
    for (int k = 0; k < kLossPix / kLossThreads; ++k) {
        const uint64_t p = p0 + (uint64_t)k * kLossThreads + threadIdx.x;
        if (p >= npix) break;
        const int y = (int)(p / (uint64_t)W), x = (int)(p - (uint64_t)y * W);
        const float *r = im.render + 3 * p;
        const float *t = im.target + 3 * p;
        float *g = im.grad + 3 * p;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float R = r[c];
            const float d = R - t[c];
            float gr = 2.f * d;
            acc = fmaf(d, d, acc);
            if (x + 1 < W) {
                const float dx = r[3 + c] - R;
                acc = fmaf(lambda, fabsf(dx), acc);
                gr -= lambda * sgn(dx);
            }
            if (x > 0) gr += lambda * sgn(R - r[c - 3]);
            if (y + 1 < H) {
                const float dy = r[3 * (size_t)W + c] - R;
                acc = fmaf(lambda, fabsf(dy), acc);
                gr -= lambda * sgn(dy);
            }
            if (y > 0) gr += lambda * sgn(R - r[c - 3 * (ptrdiff_t)W]);
            g[c] = gr;
        }
    }
    // block sum: within each wave, then across the 4 waves in a fixed order
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (s_sum[0] + s_sum[1]) + (s_sum[2] + s_sum[3]);
}

// One wave per image: lane l adds block sums l, l + 64, ... in FP64, then a
// fixed butterfly combines the lanes.
__global__ __launch_bounds__(64) void k_loss_sum(const uint32_t *block_start, const float *partial, double *loss) {
    const int v = blockIdx.x;
    const uint32_t b0 = block_start[v], b1 = block_start[v + 1];
    double s = 0.0;
    for (uint32_t b = b0 + threadIdx.x; b < b1; b += 64) s += (double)partial[b];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
    if (threadIdx.x == 0) loss[v] = s;
}

uint32_t loss_blocks(int32_t width, int32_t height) {
    const uint64_t npix = (uint64_t)width * (uint64_t)height;
    return (uint32_t)((npix + kLossPix - 1) / kLossPix);
}

hipError_t launch_loss(const LossImage *img, const uint32_t *block_start, int n, uint32_t total_blocks, float lambda,
                       float *partial, double *loss, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (total_blocks > 0)
        hipLaunchKernelGGL(k_loss, dim3(total_blocks), dim3(kLossThreads), 0, st, img, block_start, n, lambda,
                           partial);
    hipLaunchKernelGGL(k_loss_sum, dim3(n), dim3(64), 0, st, block_start, partial, loss);
    return hipGetLastError();
}

}  // namespace dpr
