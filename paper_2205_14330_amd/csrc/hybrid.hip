// Hybrid coarse-to-fine update of the point cloud (Sec. 3.3 "Hybrid
// Coarse-to-Fine Updates", Alg. 1):
//   1. voxel reduction: the points' bounding box is split into N^3 equal
//      voxels and every non-empty voxel becomes the average of its points
//      (position, SH coefficients, opacity, radius);
//   2. outlier removal: a point whose K nearest neighbours lie at distances of
//      standard deviation delta > eps is removed;
//   3. point generation: every kept point adds the average of its K nearest
//      kept neighbours.
// Decisions taken from float comparisons (voxel and grid cells, neighbour
// order, delta > eps) use float32 with every operation rounded on its own, in
// the order documented in include/dpr.h; averages are accumulated in FP64 in
// a fixed order (ascending point index within a voxel, neighbour order for a
// generated point).
//
// Voxels: cell keys per point, a stable radix sort of (key, point index),
// segment starts where the key changes, one thread per voxel.
// Neighbours: a uniform grid over the points' bounding box (about 2 points per
// cell), points sorted by cell, one thread per query walking Chebyshev shells
// of cells around its own; it keeps the K best (distance, index) pairs packed
// in 64-bit keys and stops once the K-th distance is below the smallest
// distance any cell of the next shell can hold (with a margin far above the
// float32 rounding of the distances), so the result is the exact K nearest.
#include <algorithm>

#include "dpr_internal.h"

// Every float32 decision above is made with each multiply and add rounded on
// its own, so no multiply-add may be fused in this file.  (The rounding
// intrinsics of the HIP headers would not do: their operators take the
// contraction setting of the header, and fuse once inlined.)
#pragma clang fp contract(off)

namespace dpr {

constexpr int kHyThreads = 256;

__global__ __launch_bounds__(kHyThreads) void k_bbox_partial(const float *xyz, uint32_t n, float *part) {
    __shared__ float s[6][kHyThreads / 64];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = blockIdx.x * kHyThreads + threadIdx.x; i < n; i += gridDim.x * kHyThreads) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = xyz[3 * (size_t)i + a];
            lo[a] = fminf(lo[a], v);
            hi[a] = fmaxf(hi[a], v);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], d, 64));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], d, 64));
        }
    }
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) { s[a][threadIdx.x >> 6] = lo[a]; s[3 + a][threadIdx.x >> 6] = hi[a]; }
    __syncthreads();
    if (threadIdx.x < 6) {
        float v = s[threadIdx.x][0];
        for (int w = 1; w < kHyThreads / 64; ++w)
            v = threadIdx.x < 3 ? fminf(v, s[threadIdx.x][w]) : fmaxf(v, s[threadIdx.x][w]);
        part[6 * blockIdx.x + threadIdx.x] = v;
    }
}

// One block of kHyThreads threads over nb <= kHyBoxBlocks partials (min and
// max are exact in any order, so the box is that of one sequential pass).
__global__ __launch_bounds__(kHyThreads) void k_bbox_final(const float *part, uint32_t nb, float *box) {
    __shared__ float s[6][kHyThreads / 64];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t b = threadIdx.x; b < nb; b += kHyThreads) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], part[6 * b + a]);
            hi[a] = fmaxf(hi[a], part[6 * b + 3 + a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], d, 64));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], d, 64));
        }
    }
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) { s[a][threadIdx.x >> 6] = lo[a]; s[3 + a][threadIdx.x >> 6] = hi[a]; }
    __syncthreads();
    if (threadIdx.x < 6) {
        float v = s[threadIdx.x][0];
        for (int w = 1; w < kHyThreads / 64; ++w)
            v = threadIdx.x < 3 ? fminf(v, s[threadIdx.x][w]) : fmaxf(v, s[threadIdx.x][w]);
        box[threadIdx.x] = v;
    }
}

__device__ __forceinline__ uint32_t axis_cell(float p, float lo, float s, uint32_t N) {
    if (!(s > 0.f)) return 0;
    const float t = floorf((p - lo) * s);
    if (!(t > 0.f)) return 0;
    return t >= (float)(N - 1) ? N - 1 : (uint32_t)t;
}

__device__ __forceinline__ float axis_scale(float lo, float hi, uint32_t N) {
    return hi > lo ? __fdiv_rn((float)N, hi - lo) : 0.f;
}

// key = (iz N + iy) N + ix of the N^3 cells of box; vals = point index
__global__ __launch_bounds__(kHyThreads) void k_cell_keys(const float *xyz, uint32_t n, const float *box, uint32_t N,
                                                         uint32_t *keys, uint32_t *vals) {
    const uint32_t i = blockIdx.x * kHyThreads + threadIdx.x;
    if (i >= n) return;
    const float sx = axis_scale(box[0], box[3], N), sy = axis_scale(box[1], box[4], N),
                sz = axis_scale(box[2], box[5], N);
    const uint32_t ix = axis_cell(xyz[3 * (size_t)i + 0], box[0], sx, N);
    const uint32_t iy = axis_cell(xyz[3 * (size_t)i + 1], box[1], sy, N);
    const uint32_t iz = axis_cell(xyz[3 * (size_t)i + 2], box[2], sz, N);
    keys[i] = (iz * N + iy) * N + ix;
    vals[i] = i;
}

__global__ __launch_bounds__(kHyThreads) void k_seg_flags(const uint32_t *keys, uint32_t n, uint32_t *flags) {
    const uint32_t i = blockIdx.x * kHyThreads + threadIdx.x;
    if (i < n) flags[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// starts[s] = first sorted position of segment s; starts[segments] = n (the
// last element's segment is seg[n-1] + flags[n-1] - 1, exclusive scan)
__global__ __launch_bounds__(kHyThreads) void k_seg_starts(const uint32_t *flags, const uint32_t *seg, uint32_t n,
                                                          uint32_t *starts) {
    const uint32_t i = blockIdx.x * kHyThreads + threadIdx.x;
    if (i >= n) return;
    if (flags[i]) starts[seg[i]] = i;
    if (i == n - 1) starts[seg[i] + flags[i]] = n;
}

struct CloudIn {
    const float *xyz, *sh, *op, *rad;
};
struct CloudOut {
    float *xyz, *sh, *op, *rad;
};

// Per-point attribute rows: 3 position floats, K3 SH floats, opacity and
// radius.  The kernels below walk whole rows (all K3 SH floats of a row
// loaded together); K3 = 3 (degree + 1)^2 is a template argument so the rows
// unroll, and HY_K3_DISPATCH picks the instance.  An FP64 accumulator per
// attribute adds its terms in the same order as a per-attribute loop would.
template <int K3>
struct RowSum {
    double x[3], sh[K3], op, rad;
    __device__ __forceinline__ void clear() {
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] = 0.0;
#pragma unroll
        for (int a = 0; a < K3; ++a) sh[a] = 0.0;
        op = rad = 0.0;
    }
    __device__ __forceinline__ void add(const float *xyz, const float *shp, const float *opp, const float *radp,
                                        size_t j) {
        float v[3 + K3 + 2];
#pragma unroll
        for (int a = 0; a < 3; ++a) v[a] = xyz[3 * j + a];
#pragma unroll
        for (int a = 0; a < K3; ++a) v[3 + a] = shp[(size_t)K3 * j + a];
        v[3 + K3] = opp[j];
        v[4 + K3] = radp[j];
#pragma unroll
        for (int a = 0; a < 3; ++a) x[a] += (double)v[a];
#pragma unroll
        for (int a = 0; a < K3; ++a) sh[a] += (double)v[3 + a];
        op += (double)v[3 + K3];
        rad += (double)v[4 + K3];
    }
    __device__ __forceinline__ void store_mean(const CloudOut &c, size_t o, double cnt) const {
#pragma unroll
        for (int a = 0; a < 3; ++a) c.xyz[3 * o + a] = (float)(x[a] / cnt);
#pragma unroll
        for (int a = 0; a < K3; ++a) c.sh[(size_t)K3 * o + a] = (float)(sh[a] / cnt);
        c.op[o] = (float)(op / cnt);
        c.rad[o] = (float)(rad / cnt);
    }
};

// one thread per voxel: FP64 sums over its points in ascending index order
template <int K3>
__global__ __launch_bounds__(kHyThreads) void k_voxel_average(const uint32_t *starts, uint32_t m, const uint32_t *order,
                                                             CloudIn in, CloudOut out) {
    const uint32_t v = blockIdx.x * kHyThreads + threadIdx.x;
    if (v >= m) return;
    const uint32_t b = starts[v], e = starts[v + 1];
    RowSum<K3> acc;
    acc.clear();
    for (uint32_t q = b; q < e; ++q) acc.add(in.xyz, in.sh, in.op, in.rad, order[q]);
    acc.store_mean(out, v, (double)(e - b));
}

// cell_start[c] = first sorted position with key >= c, for c in [0, ncells]
__global__ __launch_bounds__(kHyThreads) void k_cell_start(const uint32_t *skeys, uint32_t m, uint32_t ncells,
                                                          uint32_t *cell_start) {
    const uint32_t i = blockIdx.x * kHyThreads + threadIdx.x;
    if (i > m) return;
    const uint32_t lo = i == 0 ? 0u : skeys[i - 1] + 1u;
    const uint32_t hi = i == m ? ncells : skeys[i];
    for (uint32_t c = lo; c <= hi; ++c) cell_start[c] = i;
}

// float32 squared distance ((dx dx + dy dy) + dz dz), dx = x_j - x_i
__device__ __forceinline__ float dist2(const float *pi, const float *pj) {
    const float dx = pj[0] - pi[0], dy = pj[1] - pi[1], dz = pj[2] - pi[2];
    float s = dx * dx;
    s = s + dy * dy;
    return s + dz * dz;
}

struct KnnGrid {
    const float *xyz;
    const uint32_t *skeys, *svals, *cell_start;
    const float *box;
    uint32_t m, G;
    int K, keff;
    int32_t *idx;
    float *d2;
};

// One thread per query (queries in cell order).  best[] holds the K smallest
// (distance bits << 32 | index) keys in ascending order.  KMAX (8, 16 or 32,
// at least K) sizes the list, so that an insertion takes KMAX predicated
// steps rather than always 32.
template <int KMAX>
__global__ __launch_bounds__(kHyThreads) void k_knn(KnnGrid g) {
    const uint32_t t = blockIdx.x * kHyThreads + threadIdx.x;
    if (t >= g.m) return;
    const uint32_t p = g.svals[t];
    const uint32_t key = g.skeys[t];
    const int G = (int)g.G;
    const int cx = (int)(key % g.G), cy = (int)((key / g.G) % g.G), cz = (int)(key / (g.G * g.G));
    float hmin = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float ext = g.box[3 + a] - g.box[a];
        if (ext > 0.f) hmin = fminf(hmin, ext / (float)G);
    }
    const float *pp = g.xyz + 3 * (size_t)p;
    uint64_t best[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) best[k] = ~0ull;
    const int K = g.keff;
    uint64_t worst = ~0ull;           // best[K - 1]
    int found = 0;
    const int rmax = max(max(max(cx, G - 1 - cx), max(cy, G - 1 - cy)), max(cz, G - 1 - cz));
    for (int r = 0; r <= rmax; ++r) {
        for (int dz = -r; dz <= r; ++dz) {
            const int z = cz + dz;
            if (z < 0 || z >= G) continue;
            for (int dy = -r; dy <= r; ++dy) {
                const int y = cy + dy;
                if (y < 0 || y >= G) continue;
                const bool full = dz == -r || dz == r || dy == -r || dy == r;
                for (int dx = -r; dx <= r; dx += full ? 1 : (r > 0 ? 2 * r : 1)) {
                    const int x = cx + dx;
                    if (x < 0 || x >= G) continue;
                    const uint32_t c = ((uint32_t)z * g.G + (uint32_t)y) * g.G + (uint32_t)x;
                    const uint32_t b = g.cell_start[c], e = g.cell_start[c + 1];
                    for (uint32_t j = b; j < e; ++j) {
                        const uint32_t q = g.svals[j];
                        if (q == p) continue;
                        const float d = dist2(pp, g.xyz + 3 * (size_t)q);
                        uint64_t x64 = ((uint64_t)__float_as_uint(d) << 32) | q;
                        ++found;
                        if (x64 >= worst) continue;
                        // insert into the sorted prefix: keep the smaller, carry the larger on
#pragma unroll
                        for (int k = 0; k < KMAX; ++k) {
                            if (k < K) {
                                const uint64_t lo = best[k] < x64 ? best[k] : x64;
                                x64 = best[k] < x64 ? x64 : best[k];
                                best[k] = lo;
                            }
                        }
#pragma unroll
                        for (int k = 0; k < KMAX; ++k)
                            if (k == K - 1) worst = best[k];
                    }
                }
            }
        }
        if (found >= K) {
            // any point of shell r + 1 or beyond is at least r * hmin away
            const float kth = __uint_as_float((uint32_t)(worst >> 32));
            const float bound = (float)r * hmin;
            if (kth < 0.9999f * bound * bound) break;
        }
    }
    for (int k = 0; k < g.K; ++k) {
        const bool ok = k < K;
        g.idx[(size_t)p * g.K + k] = ok ? (int32_t)(uint32_t)(best[k] & 0xFFFFFFFFull) : -1;
        g.d2[(size_t)p * g.K + k] = ok ? __uint_as_float((uint32_t)(best[k] >> 32)) : 0.f;
    }
}

// delta of the neighbour distances (float32, each operation rounded) > eps -> removed
__global__ __launch_bounds__(kHyThreads) void k_spread_keep(const float *d2, uint32_t m, int K, int keff, float eps,
                                                           uint32_t *keep) {
    const uint32_t i = blockIdx.x * kHyThreads + threadIdx.x;
    if (i >= m) return;
    if (keff == 0) { keep[i] = 1u; return; }
    const float *d = d2 + (size_t)i * K;
    float sum = 0.f;
    for (int q = 0; q < keff; ++q) sum = sum + sqrtf(d[q]);
    const float mean = __fdiv_rn(sum, (float)keff);
    float var = 0.f;
    for (int q = 0; q < keff; ++q) {
        const float e = sqrtf(d[q]) - mean;
        var = var + e * e;
    }
    const float delta = sqrtf(__fdiv_rn(var, (float)keff));
    keep[i] = (delta > eps) ? 0u : 1u;
}

template <int K3>
__global__ __launch_bounds__(kHyThreads) void k_gather_kept(const uint32_t *keep, const uint32_t *pos, uint32_t m,
                                                           CloudIn in, CloudOut out) {
    const uint32_t i = blockIdx.x * kHyThreads + threadIdx.x;
    if (i >= m || !keep[i]) return;
    const uint32_t o = pos[i];
    float v[3 + K3 + 2];
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a] = in.xyz[3 * (size_t)i + a];
#pragma unroll
    for (int a = 0; a < K3; ++a) v[3 + a] = in.sh[(size_t)K3 * i + a];
    v[3 + K3] = in.op[i];
    v[4 + K3] = in.rad[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) out.xyz[3 * (size_t)o + a] = v[a];
#pragma unroll
    for (int a = 0; a < K3; ++a) out.sh[(size_t)K3 * o + a] = v[3 + a];
    out.op[o] = v[3 + K3];
    out.rad[o] = v[4 + K3];
}

// generated point i (written at m + i) = FP64 average of point i's neighbours, in neighbour order
template <int K3>
__global__ __launch_bounds__(kHyThreads) void k_generate(CloudOut c, uint32_t m, const int32_t *idx, int K, int keff) {
    const uint32_t i = blockIdx.x * kHyThreads + threadIdx.x;
    if (i >= m) return;
    const int32_t *nb = idx + (size_t)i * K;
    RowSum<K3> acc;
    acc.clear();
    for (int q = 0; q < keff; ++q) acc.add(c.xyz, c.sh, c.op, c.rad, (size_t)nb[q]);
    acc.store_mean(c, (size_t)m + i, (double)keff);
}

// ---------------------------------------------------------------------------
// host sequencing
// ---------------------------------------------------------------------------
static uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + kHyThreads - 1) / kHyThreads); }

// Launches KERNEL<K3> for the SH row length k3 = 3 (degree + 1)^2, degree 0..3.
#define HY_K3_DISPATCH(k3, KERNEL, ...)                                                        \
    do {                                                                                         \
        switch (k3) {                                                                            \
        case 3: hipLaunchKernelGGL(KERNEL<3>, __VA_ARGS__); break;                               \
        case 12: hipLaunchKernelGGL(KERNEL<12>, __VA_ARGS__); break;                             \
        case 27: hipLaunchKernelGGL(KERNEL<27>, __VA_ARGS__); break;                             \
        case 48: hipLaunchKernelGGL(KERNEL<48>, __VA_ARGS__); break;                             \
        default: return hipErrorInvalidValue;                                                    \
        }                                                                                        \
    } while (0)

static int key_bits(uint64_t ncells) {
    int b = 0;
    while ((1ull << b) < ncells) ++b;
    return b;
}

uint32_t knn_grid_size(uint64_t m) {
    uint32_t g = 1;
    while ((uint64_t)(g + 1) * (g + 1) * (g + 1) * 2 <= m && g < kKnnMaxGrid) ++g;
    return g;
}

HyScratchBytes hy_scratch_bytes(uint64_t n, int K) {
    const uint64_t hw = radix_hist_words(n);
    const uint64_t G = knn_grid_size(n);
    HyScratchBytes b;
    b.keys = b.vals = b.keys_alt = b.vals_alt = 4 * n;
    b.hist = 4 * (hw + 1);                 // the scan also writes the total after the last word
    b.part = 8 * (std::max(scan_partials(n + 2), scan_partials(hw)) + 2);
    b.total64 = 8;
    b.flags = b.seg = b.starts = 4 * (n + 2);
    b.cell_start = 4 * (G * G * G + 2);
    b.box_part = 4 * 6 * (uint64_t)kHyBoxBlocks;
    b.box = 4 * 6;
    b.idx = b.d2 = 4 * n * (uint64_t)K;
    return b;
}

static hipError_t bbox(const float *xyz, uint32_t n, HyScratch &s, hipStream_t st) {
    const uint32_t nb = std::min<uint32_t>(blocks_for(n), kHyBoxBlocks);
    hipLaunchKernelGGL(k_bbox_partial, dim3(nb), dim3(kHyThreads), 0, st, xyz, n, s.box_part);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kHyThreads), 0, st, s.box_part, nb, s.box);
    return hipGetLastError();
}

// keys of the N^3 cells of the points' bounding box, stable-sorted with the
// point indices; *keys_out / *vals_out point at the sorted arrays
static hipError_t sorted_cells(const float *xyz, uint32_t n, uint32_t N, HyScratch &s, uint32_t **keys_out,
                               uint32_t **vals_out, hipStream_t st) {
    hipError_t e = bbox(xyz, n, s, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cell_keys, dim3(blocks_for(n)), dim3(kHyThreads), 0, st, xyz, n, s.box, N, s.keys, s.vals);
    bool alt = false;
    e = launch_radix_sort(n, key_bits((uint64_t)N * N * N), s.keys, s.vals, s.keys_alt, s.vals_alt, s.hist, s.part,
                          &alt, st);
    *keys_out = alt ? s.keys_alt : s.keys;
    *vals_out = alt ? s.vals_alt : s.vals;
    return e;
}

hipError_t launch_knn(const float *xyz, uint32_t m, int K, int32_t *idx, float *d2, HyScratch &s, hipStream_t st) {
    if (m == 0) return hipSuccess;
    const uint32_t G = knn_grid_size(m);
    uint32_t *skeys, *svals;
    hipError_t e = sorted_cells(xyz, m, G, s, &skeys, &svals, st);
    if (e != hipSuccess) return e;
    const uint32_t ncells = G * G * G;
    hipLaunchKernelGGL(k_cell_start, dim3(blocks_for((uint64_t)m + 1)), dim3(kHyThreads), 0, st, skeys, m, ncells,
                       s.cell_start);
    KnnGrid g;
    g.xyz = xyz;
    g.skeys = skeys;
    g.svals = svals;
    g.cell_start = s.cell_start;
    g.box = s.box;
    g.m = m;
    g.G = G;
    g.K = K;
    g.keff = (int)std::min<uint64_t>((uint64_t)K, (uint64_t)m - 1);
    g.idx = idx;
    g.d2 = d2;
    if (g.K <= 8) hipLaunchKernelGGL(k_knn<8>, dim3(blocks_for(m)), dim3(kHyThreads), 0, st, g);
    else if (g.K <= 16) hipLaunchKernelGGL(k_knn<16>, dim3(blocks_for(m)), dim3(kHyThreads), 0, st, g);
    else hipLaunchKernelGGL(k_knn<kKnnMax>, dim3(blocks_for(m)), dim3(kHyThreads), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_voxel_reduce(const float *xyz, const float *sh, const float *op, const float *rad, uint32_t n,
                               int k3, uint32_t N, float *oxyz, float *osh, float *oop, float *orad, HyScratch &s,
                               uint64_t *m_host, hipStream_t st) {
    uint32_t *skeys, *svals;
    hipError_t e = sorted_cells(xyz, n, N, s, &skeys, &svals, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_flags, dim3(blocks_for(n)), dim3(kHyThreads), 0, st, skeys, n, s.flags);
    e = launch_scan(s.flags, s.seg, n, s.part, s.total64, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_seg_starts, dim3(blocks_for(n)), dim3(kHyThreads), 0, st, s.flags, s.seg, n, s.starts);
    e = read_count(s.total64, m_host, st);
    if (e != hipSuccess) return e;
    const uint32_t m = (uint32_t)*m_host;
    CloudIn in{xyz, sh, op, rad};
    CloudOut out{oxyz, osh, oop, orad};
    HY_K3_DISPATCH(k3, k_voxel_average, dim3(blocks_for(m)), dim3(kHyThreads), 0, st, s.starts, m, svals, in,
                       out);
    return hipGetLastError();
}

hipError_t launch_filter_generate(const float *xyz, const float *sh, const float *op, const float *rad, uint32_t m,
                                  int k3, int K, float eps, float *oxyz, float *osh, float *oop, float *orad,
                                  HyScratch &s, uint64_t *kept_host, uint64_t *count_host, hipStream_t st) {
    *kept_host = 0;
    *count_host = 0;
    if (m == 0) return hipSuccess;
    hipError_t e = launch_knn(xyz, m, K, s.idx, s.d2, s, st);
    if (e != hipSuccess) return e;
    const int keff = (int)std::min<uint64_t>((uint64_t)K, (uint64_t)m - 1);
    hipLaunchKernelGGL(k_spread_keep, dim3(blocks_for(m)), dim3(kHyThreads), 0, st, s.d2, m, K, keff, eps, s.flags);
    e = launch_scan(s.flags, s.seg, m, s.part, s.total64, st);
    if (e != hipSuccess) return e;
    CloudIn in{xyz, sh, op, rad};
    CloudOut out{oxyz, osh, oop, orad};
    HY_K3_DISPATCH(k3, k_gather_kept, dim3(blocks_for(m)), dim3(kHyThreads), 0, st, s.flags, s.seg, m, in, out);
    e = read_count(s.total64, kept_host, st);
    if (e != hipSuccess) return e;
    const uint32_t mk = (uint32_t)*kept_host;
    *count_host = mk;
    if (mk < 2) return hipSuccess;
    e = launch_knn(oxyz, mk, K, s.idx, s.d2, s, st);
    if (e != hipSuccess) return e;
    const int keff2 = (int)std::min<uint64_t>((uint64_t)K, (uint64_t)mk - 1);
    HY_K3_DISPATCH(k3, k_generate, dim3(blocks_for(mk)), dim3(kHyThreads), 0, st, out, mk, s.idx, K, keff2);
    *count_host = 2ull * mk;
    return hipGetLastError();
}

}  // namespace dpr
