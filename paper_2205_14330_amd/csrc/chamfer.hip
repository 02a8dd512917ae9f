// Video warm start (Sec. 3.4 "Video Synthesis"): the Chamfer distance of
// Eq. (9) between the learned cloud S1 of a frame and the initial cloud S2 of
// the next, its gradient with respect to the positions of S2, an Adam step on
// them, and the transfer to each S2 point of the mean SH coefficients of its
// k nearest S1 points.
//
// Nearest neighbours by brute force over LDS tiles: a block takes 256 threads
// x 2 queries against one 4096-point range of the other cloud (so that a frame
// of some 10^4 points still fills the GPU), and folds its result into a
// 64-bit key per query with one atomic minimum: key = (d2 bits << 32) | index,
// which orders by (d2, index) because d2 >= 0 (ties go to the lower index,
// whatever the order in which the blocks finish).  Distances in float32 with
// each operation rounded: ((dx dx + dy dy) + dz dz).  Sums of Eq. (9) in FP64
// (block partials, then one block in a fixed order); the gradient term that
// collects the S1 points whose nearest is y_j uses FP64 atomics.
// Top-k: one thread per query keeps its k best keys in registers (sorted)
// while all of S1 streams through LDS; SH means in FP64 in neighbour order.
#include <cmath>

#include "dpr_internal.h"

#pragma clang fp contract(off)

namespace dpr {

constexpr int kNnThreads = 256;
constexpr int kNnQueries = 2;                          // queries per thread
constexpr int kNnTile = 1024;                          // candidate points per LDS tile
constexpr int kNnRange = 4096;                         // candidate points per block

__device__ __forceinline__ float d2f(float ax, float ay, float az, float bx, float by, float bz) {
    const float a = ax - bx, b = ay - by, c = az - bz;
    float s = a * a;
    s = s + b * b;
    return s + c * c;
}

// key[i] = min over this block's candidate range of (d2(q_i, c_j) bits << 32 | j)
__global__ __launch_bounds__(kNnThreads) void k_nn(const float *q, uint32_t nq, const float *c, uint32_t nc,
                                                   unsigned long long *key) {
    __shared__ float s_x[kNnTile], s_y[kNnTile], s_z[kNnTile];
    const uint32_t q0 = blockIdx.x * (kNnThreads * kNnQueries) + threadIdx.x;
    const uint32_t cbeg = blockIdx.y * (uint32_t)kNnRange, cend = min(cbeg + (uint32_t)kNnRange, nc);
    float qx[kNnQueries], qy[kNnQueries], qz[kNnQueries], best[kNnQueries];
    uint32_t bj[kNnQueries];
#pragma unroll
    for (int k = 0; k < kNnQueries; ++k) {
        const uint32_t i = q0 + k * kNnThreads;
        const uint32_t ii = i < nq ? i : 0;
        qx[k] = q[3 * (size_t)ii]; qy[k] = q[3 * (size_t)ii + 1]; qz[k] = q[3 * (size_t)ii + 2];
        best[k] = INFINITY;
        bj[k] = 0xFFFFFFFFu;
    }
    for (uint32_t t0 = cbeg; t0 < cend; t0 += kNnTile) {
        const uint32_t tn = min((uint32_t)kNnTile, cend - t0);
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < tn; t += kNnThreads) {
            s_x[t] = c[3 * (size_t)(t0 + t)];
            s_y[t] = c[3 * (size_t)(t0 + t) + 1];
            s_z[t] = c[3 * (size_t)(t0 + t) + 2];
        }
        __syncthreads();
        for (uint32_t t = 0; t < tn; ++t) {
            const float cx = s_x[t], cy = s_y[t], cz = s_z[t];
#pragma unroll
            for (int k = 0; k < kNnQueries; ++k) {
                const float d = d2f(qx[k], qy[k], qz[k], cx, cy, cz);
                if (d < best[k]) {          // scanning in index order: the first minimum is the lowest index
                    best[k] = d;
                    bj[k] = t0 + t;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kNnQueries; ++k) {
        const uint32_t i = q0 + k * kNnThreads;
        if (i < nq && bj[k] != 0xFFFFFFFFu)
            atomicMin(key + i, ((unsigned long long)__float_as_uint(best[k]) << 32) | bj[k]);
    }
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static hipError_t nearest(const float *q, uint32_t nq, const float *c, uint32_t nc, unsigned long long *key,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3((nq + 255) / 256), dim3(256), 0, st, key, ~0ull, nq);
    const dim3 grid((nq + kNnThreads * kNnQueries - 1) / (kNnThreads * kNnQueries), (nc + kNnRange - 1) / kNnRange);
    hipLaunchKernelGGL(k_nn, grid, dim3(kNnThreads), 0, st, q, nq, c, nc, key);
    return hipGetLastError();
}

// per S2 point j: acc[j] = sum of the S1 points whose nearest is j (FP64), cnt[j] their number
__global__ void k_collect(const unsigned long long *key12, uint32_t n1, const float *s1, double *acc, uint32_t *cnt) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n1) return;
    const uint32_t j = (uint32_t)(key12[i] & 0xFFFFFFFFull);
#pragma unroll
    for (int a = 0; a < 3; ++a) atomicAdd(acc + 3 * (size_t)j + a, (double)s1[3 * (size_t)i + a]);
    atomicAdd(cnt + j, 1u);
}

// grad2[j] = 2/n2 (y_j - nn(y_j)) + 2/n1 (cnt_j y_j - acc_j), FP64 then rounded
__global__ void k_grad(const unsigned long long *key21, uint32_t n2, const float *s2, const float *s1, uint32_t n1,
                       const double *acc, const uint32_t *cnt, float *grad2, int32_t *nn21) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n2) return;
    const uint32_t k = (uint32_t)(key21[j] & 0xFFFFFFFFull);
    if (nn21) nn21[j] = (int32_t)k;
    if (!grad2) return;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double y = (double)s2[3 * (size_t)j + a];
        const double g = 2.0 / (double)n2 * (y - (double)s1[3 * (size_t)k + a]) +
                         2.0 / (double)n1 * ((double)cnt[j] * y - acc[3 * (size_t)j + a]);
        grad2[3 * (size_t)j + a] = (float)g;
    }
}

__global__ void k_nn_index(const unsigned long long *key, uint32_t n, int32_t *nn) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) nn[i] = (int32_t)(uint32_t)(key[i] & 0xFFFFFFFFull);
}

constexpr int kSumThreads = 256;

// part[b] = FP64 sum of the d2 of keys [b 256 .. ), in index order within the block
__global__ __launch_bounds__(kSumThreads) void k_sum_d2(const unsigned long long *key, uint32_t n, double *part) {
    __shared__ double s[kSumThreads];
    const uint32_t i = blockIdx.x * kSumThreads + threadIdx.x;
    s[threadIdx.x] = i < n ? (double)__uint_as_float((uint32_t)(key[i] >> 32)) : 0.0;
    __syncthreads();
    for (int w = kSumThreads / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// cd = (sum part1) / n1 + (sum part2) / n2, each summed in block order by one thread
__global__ void k_cd(const double *part1, uint32_t nb1, uint32_t n1, const double *part2, uint32_t nb2, uint32_t n2,
                     double *cd) {
    if (threadIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (uint32_t k = 0; k < nb1; ++k) a += part1[k];
    for (uint32_t k = 0; k < nb2; ++k) b += part2[k];
    *cd = a / (double)n1 + b / (double)n2;
}

ChamferLayout chamfer_layout(uint64_t n1, uint64_t n2) {
    ChamferLayout L;
    uint64_t off = 0;
    auto add = [&](uint64_t bytes) {
        const uint64_t at = off;
        off += (bytes + 255) & ~255ull;
        return at;
    };
    L.key12 = add(8 * n1);
    L.key21 = add(8 * n2);
    L.acc = add(8 * 3 * n2);
    L.cnt = add(4 * n2);
    L.part1 = add(8 * ((n1 + kSumThreads - 1) / kSumThreads));
    L.part2 = add(8 * ((n2 + kSumThreads - 1) / kSumThreads));
    L.bytes = off;
    return L;
}

hipError_t launch_chamfer(uint32_t n1, const float *s1, uint32_t n2, const float *s2, double *cd, float *grad2,
                          int32_t *nn12, int32_t *nn21, uint8_t *ws, hipStream_t st) {
    const ChamferLayout L = chamfer_layout(n1, n2);
    auto *key12 = reinterpret_cast<unsigned long long *>(ws + L.key12);
    auto *key21 = reinterpret_cast<unsigned long long *>(ws + L.key21);
    double *acc = reinterpret_cast<double *>(ws + L.acc);
    uint32_t *cnt = reinterpret_cast<uint32_t *>(ws + L.cnt);
    double *part1 = reinterpret_cast<double *>(ws + L.part1), *part2 = reinterpret_cast<double *>(ws + L.part2);
    hipError_t e = nearest(s1, n1, s2, n2, key12, st);
    if (e != hipSuccess) return e;
    e = nearest(s2, n2, s1, n1, key21, st);
    if (e != hipSuccess) return e;
    const uint32_t nb1 = (n1 + kSumThreads - 1) / kSumThreads, nb2 = (n2 + kSumThreads - 1) / kSumThreads;
    if (cd) {
        hipLaunchKernelGGL(k_sum_d2, dim3(nb1), dim3(kSumThreads), 0, st, key12, n1, part1);
        hipLaunchKernelGGL(k_sum_d2, dim3(nb2), dim3(kSumThreads), 0, st, key21, n2, part2);
        hipLaunchKernelGGL(k_cd, dim3(1), dim3(64), 0, st, part1, nb1, n1, part2, nb2, n2, cd);
    }
    if (nn12) hipLaunchKernelGGL(k_nn_index, dim3((n1 + 255) / 256), dim3(256), 0, st, key12, n1, nn12);
    if (grad2) {
        e = launch_fill_u32(reinterpret_cast<uint32_t *>(acc), 0u, 6ull * n2, st);
        if (e != hipSuccess) return e;
        e = launch_fill_u32(cnt, 0u, n2, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_collect, dim3((n1 + 255) / 256), dim3(256), 0, st, key12, n1, s1, acc, cnt);
    }
    if (grad2 || nn21)
        hipLaunchKernelGGL(k_grad, dim3((n2 + 255) / 256), dim3(256), 0, st, key21, n2, s2, s1, n1, acc, cnt, grad2,
                           nn21);
    return hipGetLastError();
}

// Top-k: a group of kTopkLanes consecutive lanes per query y of S2.  Lane s of
// the group scans the candidates t = s mod kTopkLanes of every LDS tile of S1
// and keeps the KM smallest keys (d2 bits << 32 | index, ascending) it met;
// the group's lists are then merged by exchanging them between partner lanes
// (xor 1, 2, 4).  The keys are distinct and totally ordered, so the K smallest
// are found exactly, whatever the split.
constexpr int kTopkLanes = 8;
constexpr int kTopkBlock = 256;                          // 32 queries per block

template <int KM>
__device__ __forceinline__ void topk_insert(unsigned long long (&best)[KM], int K, unsigned long long x,
                                            unsigned long long &worst) {
    if (x >= worst) return;
    // keep the smaller key in each place, carry the larger one on
#pragma unroll
    for (int k = 0; k < KM; ++k) {
        if (k < K) {
            const unsigned long long lo = best[k] < x ? best[k] : x;
            x = best[k] < x ? x : best[k];
            best[k] = lo;
        }
    }
#pragma unroll
    for (int k = 0; k < KM; ++k)
        if (k == K - 1) worst = best[k];
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((unsigned long long)hi << 32) | lo;
}

template <int KM>
__global__ __launch_bounds__(kTopkBlock) void k_topk_sh(const float *s1, const float *sh1, uint32_t n1,
                                                        const float *s2, uint32_t n2, int k3, int K,
                                                        float *out_sh, int32_t *idx) {
    __shared__ float s_x[kNnTile], s_y[kNnTile], s_z[kNnTile];
    const uint32_t sub = threadIdx.x % (uint32_t)kTopkLanes;
    const uint32_t j = blockIdx.x * (uint32_t)(kTopkBlock / kTopkLanes) + threadIdx.x / (uint32_t)kTopkLanes;
    const uint32_t jj = j < n2 ? j : 0;
    const float qx = s2[3 * (size_t)jj], qy = s2[3 * (size_t)jj + 1], qz = s2[3 * (size_t)jj + 2];
    unsigned long long best[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) best[k] = ~0ull;
    unsigned long long worst = ~0ull;
    for (uint32_t t0 = 0; t0 < n1; t0 += kNnTile) {
        const uint32_t tn = min((uint32_t)kNnTile, n1 - t0);
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < tn; t += kTopkBlock) {
            s_x[t] = s1[3 * (size_t)(t0 + t)];
            s_y[t] = s1[3 * (size_t)(t0 + t) + 1];
            s_z[t] = s1[3 * (size_t)(t0 + t) + 2];
        }
        __syncthreads();
        for (uint32_t t = sub; t < tn; t += kTopkLanes) {
            const float d = d2f(qx, qy, qz, s_x[t], s_y[t], s_z[t]);
            topk_insert(best, K, ((unsigned long long)__float_as_uint(d) << 32) | (t0 + t), worst);
        }
    }
    // merge the group's lists: after the exchange with lane ^ m every lane of a
    // pair holds the K smallest of both (all lanes take part in the shuffles)
#pragma unroll
    for (int m = 1; m < kTopkLanes; m <<= 1) {
        unsigned long long other[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) other[k] = shfl_xor_u64(best[k], m);
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (k < K) topk_insert(best, K, other[k], worst);
    }
    if (j >= n2 || sub != 0) return;
    const int kk = (int)min((uint32_t)K, n1);
    if (idx) {
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (k < K) idx[(size_t)j * K + k] = k < kk ? (int32_t)(uint32_t)(best[k] & 0xFFFFFFFFull) : -1;
    }
    for (int a = 0; a < k3; ++a) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (k < kk) acc += (double)sh1[(size_t)k3 * (uint32_t)(best[k] & 0xFFFFFFFFull) + a];
        out_sh[(size_t)k3 * j + a] = (float)(acc / (double)kk);
    }
}

hipError_t launch_topk_sh(uint32_t n1, const float *s1, const float *sh1, uint32_t n2, const float *s2, int k3, int K,
                          float *out_sh, int32_t *idx, hipStream_t st) {
    if (n2 == 0) return hipSuccess;
    if (K < 1 || K > kTopkMax) return hipErrorInvalidValue;
    const dim3 grid((n2 + kTopkBlock / kTopkLanes - 1) / (kTopkBlock / kTopkLanes));
    if (K <= 4) {
        hipLaunchKernelGGL(k_topk_sh<4>, grid, dim3(kTopkBlock), 0, st, s1, sh1, n1, s2, n2, k3, K, out_sh, idx);
    } else if (K <= 8) {
        hipLaunchKernelGGL(k_topk_sh<8>, grid, dim3(kTopkBlock), 0, st, s1, sh1, n1, s2, n2, k3, K, out_sh, idx);
    } else if (K <= 16) {
        hipLaunchKernelGGL(k_topk_sh<16>, grid, dim3(kTopkBlock), 0, st, s1, sh1, n1, s2, n2, k3, K, out_sh, idx);
    } else {
        hipLaunchKernelGGL(k_topk_sh<kTopkMax>, grid, dim3(kTopkBlock), 0, st, s1, sh1, n1, s2, n2, k3, K, out_sh,
                           idx);
    }
    return hipGetLastError();
}

// Adam with bias correction (c1 = 1 - b1^t, c2 = 1 - b2^t computed on the host)
__global__ void k_adam(uint32_t n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(uint32_t n, float *p, const float *g, float *m, float *v, int t, float lr, float b1, float b2,
                       float eps, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)t));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)t));
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, c1, c2, eps);
    return hipGetLastError();
}

}  // namespace dpr
