// Visual-hull initialisation and multi-view consistency filter (Sec. 3.1
// "Initialization"; the appendix's consistency check CC): a point is kept when
// its projection (Eq. 1) falls on a foreground pixel of every camera's mask.
//   sampling: candidates drawn uniformly in a box from a counter-based
//             generator (Philox4x32-10, Salmon et al. SC 2011: counter = the
//             candidate index, key = the seed), the consistent ones returned
//             in candidate order;
//   filter:   the consistent points of a cloud, every parameter, in order.
// The pixel decision is taken in float32 with the operations documented in
// include/dpr.h, each rounded once, so it is reproducible bit for bit.
//
// The masks are first packed to one bit per pixel in the workspace (sixteen
// 800x800 masks take 1.25 MB instead of 10 MB, so every XCD's L2 holds them
// all: the lookups of random candidates are L2 hits).
// Two passes over blocks of 1024 items (4 per thread): the first decides CC
// (the 4 items of a thread walk the cameras together so that 4 mask gathers
// are in flight; a wave leaves the camera loop once none of its items is still
// inside) and writes one bit per item and one count per block; a scan of the
// counts gives each block its output offset; the second pass writes the kept
// items at offset + rank (popcounts of the bits before them), which keeps the
// input order.  Camera and mask descriptors sit in one table in the
// workspace and are read through uniform (scalar) loads.
#include <vector>

#include "dpr_internal.h"

#pragma clang fp contract(off)

namespace dpr {

constexpr int kHullThreads = 256;
constexpr int kHullPer = 4;                                  // items per thread
constexpr int kHullBlockItems = kHullThreads * kHullPer;     // 1024
constexpr int kHullWords = kHullBlockItems / 32;             // bitmask words per block

uint64_t hull_blocks(uint64_t n) { return (n + kHullBlockItems - 1) / kHullBlockItems; }

struct HullArgs {
    const HullCam *cams;
    int32_t n_cams;
    uint64_t n;
    // sampling (xyz == nullptr) or filter (xyz != nullptr)
    const float *xyz;
    uint32_t key0, key1;
    float lo[3], width[3];
    uint32_t *bits;        // [blocks][kHullWords]
    uint32_t *counts;      // [blocks]
    uint8_t *keep;         // [n] CC per item (optional)
};

// Ten rounds of Philox4x32 (multipliers and key increments of the SC 2011 paper).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t p0 = c[0], p2 = c[2];
        const uint32_t hi0 = __umulhi(0xD2511F53u, p0), lo0 = 0xD2511F53u * p0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, p2), lo1 = 0xCD9E8D57u * p2;
        c[0] = hi1 ^ c[1] ^ k0;
        c[1] = lo1;
        c[2] = hi0 ^ c[3] ^ k1;
        c[3] = lo0;
    }
}

// Candidate j: u = (r >> 8) 2^-24 of the first three words, lo + u (hi - lo) in one rounding.
__device__ __forceinline__ void candidate(const HullArgs &a, uint64_t j, float p[3]) {
    uint32_t c[4] = {(uint32_t)j, (uint32_t)(j >> 32), 0u, 0u};
    philox4x32_10(c, a.key0, a.key1);
#pragma unroll
    for (int d = 0; d < 3; ++d) p[d] = fmaf((float)(c[d] >> 8) * 0x1p-24f, a.width[d], a.lo[d]);
}

__device__ __forceinline__ void load_item(const HullArgs &a, uint64_t j, float p[3]) {
    if (a.xyz) {
        p[0] = a.xyz[3 * j];
        p[1] = a.xyz[3 * j + 1];
        p[2] = a.xyz[3 * j + 2];
    } else {
        candidate(a, j, p);
    }
}

// 1 if p falls on a foreground pixel of camera c (float32 decisions as documented).
__device__ __forceinline__ bool inside(const HullCam &c, const float p[3]) {
    float X[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) X[r] = fmaf(c.R[3 * r], p[0], fmaf(c.R[3 * r + 1], p[1], fmaf(c.R[3 * r + 2], p[2], c.t[r])));
    if (!(X[2] > 0.f)) return false;
    const float px = fmaf(c.fx, X[0] / X[2], c.cx);
    const float py = fmaf(c.fy, X[1] / X[2], c.cy);
    if (!(px >= 0.f && px < (float)c.width && py >= 0.f && py < (float)c.height)) return false;
    const uint64_t idx = (uint64_t)(int32_t)py * (uint32_t)c.width + (uint32_t)(int32_t)px;
    return (c.bits[idx >> 5] >> (idx & 31u)) & 1u;
}

// Packed word w of all cameras: bit b = 1 iff mask byte 32 w' + b != 0 (w' the
// word within its camera, bytes past the mask read as 0).
__global__ __launch_bounds__(kHullThreads) void k_pack_masks(const HullCam *cams, int32_t n_cams, uint64_t words,
                                                             uint32_t *packed) {
    const uint64_t w = (uint64_t)blockIdx.x * kHullThreads + threadIdx.x;
    if (w >= words) return;
    int32_t lo = 0, hi = n_cams - 1;                // last camera with word_off <= w
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (cams[mid].word_off <= w) lo = mid; else hi = mid - 1;
    }
    const HullCam &c = cams[lo];
    const uint64_t npix = (uint64_t)c.width * (uint32_t)c.height;
    const uint64_t p0 = (w - c.word_off) * 32;
    uint32_t v = 0;
    for (uint32_t b = 0; b < 32 && p0 + b < npix; ++b) v |= (c.mask[p0 + b] != 0 ? 1u : 0u) << b;
    packed[w] = v;
}

__global__ __launch_bounds__(kHullThreads) void k_hull_flags(HullArgs a) {
    __shared__ uint32_t s_cnt[kHullThreads / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t base = (uint64_t)blockIdx.x * kHullBlockItems;
    float p[kHullPer][3];
    bool in[kHullPer];
#pragma unroll
    for (int k = 0; k < kHullPer; ++k) {
        const uint64_t j = base + (uint64_t)k * kHullThreads + tid;
        in[k] = j < a.n;
        if (in[k]) load_item(a, j, p[k]);
    }
    for (int32_t i = 0; i < a.n_cams; ++i) {
        bool any = false;
#pragma unroll
        for (int k = 0; k < kHullPer; ++k) any = any || in[k];
        if (__ballot(any) == 0ull) break;
        const HullCam &c = a.cams[i];
#pragma unroll
        for (int k = 0; k < kHullPer; ++k)
            if (in[k]) in[k] = inside(c, p[k]);
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < kHullPer; ++k) {
        // items base + k 256 + 64 wave + lane -> bits of words 8 k + 2 wave, + 1
        const uint64_t m = __ballot(in[k]);
        if (lane == 0) {
            uint32_t *w = a.bits + (uint64_t)blockIdx.x * kHullWords + 8 * k + 2 * wave;
            w[0] = (uint32_t)m;
            w[1] = (uint32_t)(m >> 32);
            cnt += (uint32_t)__popcll(m);
        }
        if (a.keep) {
            const uint64_t j = base + (uint64_t)k * kHullThreads + tid;
            if (j < a.n) a.keep[j] = in[k] ? 1 : 0;
        }
    }
    if (lane == 0) s_cnt[wave] = cnt;
    __syncthreads();
    if (tid == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kHullThreads / 64; ++w) s += s_cnt[w];
        a.counts[blockIdx.x] = s;
    }
}

struct HullOut {
    const uint32_t *offsets;     // [blocks] exclusive scan of the counts
    uint64_t capacity;
    // sampling: positions; filter: every parameter (k3 floats of SH per point)
    float *xyz, *sh, *opacity, *radius;
    const float *in_sh, *in_opacity, *in_radius;
    int k3;
};

__global__ __launch_bounds__(kHullThreads) void k_hull_scatter(HullArgs a, HullOut o) {
    __shared__ uint32_t s_bits[kHullWords], s_pre[kHullWords];
    const uint32_t tid = threadIdx.x;
    if (tid < (uint32_t)kHullWords) s_bits[tid] = a.bits[(uint64_t)blockIdx.x * kHullWords + tid];
    __syncthreads();
    if (tid == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kHullWords; ++w) {
            s_pre[w] = s;
            s += (uint32_t)__popc(s_bits[w]);
        }
    }
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kHullBlockItems;
    const uint64_t off = o.offsets[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kHullPer; ++k) {
        const uint32_t l = (uint32_t)k * kHullThreads + tid;      // item within the block
        const uint32_t w = l >> 5, b = l & 31;
        if (!((s_bits[w] >> b) & 1u)) continue;
        const uint64_t rank = off + s_pre[w] + (uint32_t)__popc(s_bits[w] & ((1u << b) - 1u));
        if (rank >= o.capacity) continue;
        const uint64_t j = base + l;
        float p[3];
        load_item(a, j, p);
        o.xyz[3 * rank] = p[0];
        o.xyz[3 * rank + 1] = p[1];
        o.xyz[3 * rank + 2] = p[2];
        if (a.xyz) {
            for (int q = 0; q < o.k3; ++q) o.sh[(uint64_t)o.k3 * rank + q] = o.in_sh[(uint64_t)o.k3 * j + q];
            o.opacity[rank] = o.in_opacity[j];
            o.radius[rank] = o.in_radius[j];
        }
    }
}

HullLayout hull_layout(uint64_t n, int32_t n_cams, const HullCam *cams) {
    const uint64_t nb = hull_blocks(n);
    HullLayout h;
    h.words = 0;
    for (int32_t i = 0; i < n_cams; ++i) h.words += ((uint64_t)cams[i].width * (uint32_t)cams[i].height + 31) / 32;
    uint64_t off = 0;
    auto add = [&](uint64_t bytes) {
        const uint64_t at = off;
        off += (bytes + 255) & ~255ull;
        return at;
    };
    h.cams = add(sizeof(HullCam) * (uint64_t)n_cams);
    h.packed = add(4 * h.words);
    h.bits = add(4 * kHullWords * nb);
    h.counts = add(4 * (nb + 1));
    h.offsets = add(4 * (nb + 1));                 // the scan also writes the total after the last entry
    h.part = add(8 * (scan_partials(nb + 1) + 2));
    h.total = add(8);
    h.bytes = off;
    return h;
}

hipError_t launch_hull(const HullJob &job, uint8_t *ws, uint64_t *kept_host, hipStream_t st) {
    const HullLayout L = hull_layout(job.n, job.n_cams, job.cams);
    *kept_host = 0;
    // the table with each camera's packed words
    std::vector<HullCam> tab(job.cams, job.cams + job.n_cams);
    uint32_t *packed = reinterpret_cast<uint32_t *>(ws + L.packed);
    uint64_t woff = 0;
    for (HullCam &c : tab) {
        c.word_off = woff;
        c.bits = packed + woff;
        woff += ((uint64_t)c.width * (uint32_t)c.height + 31) / 32;
    }
    HullArgs a;
    a.cams = reinterpret_cast<const HullCam *>(ws + L.cams);
    a.n_cams = job.n_cams;
    a.n = job.n;
    a.xyz = job.xyz;
    a.key0 = (uint32_t)job.seed;
    a.key1 = (uint32_t)(job.seed >> 32);
    for (int d = 0; d < 3; ++d) {
        a.lo[d] = job.lo[d];
        a.width[d] = job.hi[d] - job.lo[d];
    }
    a.bits = reinterpret_cast<uint32_t *>(ws + L.bits);
    a.counts = reinterpret_cast<uint32_t *>(ws + L.counts);
    a.keep = job.keep;
    hipError_t e = upload_async(ws + L.cams, tab.data(), sizeof(HullCam) * (size_t)job.n_cams, st);
    if (e != hipSuccess || job.n == 0) return e;
    hipLaunchKernelGGL(k_pack_masks, dim3((uint32_t)((L.words + kHullThreads - 1) / kHullThreads)),
                       dim3(kHullThreads), 0, st, a.cams, job.n_cams, L.words, packed);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint64_t nb = hull_blocks(job.n);
    hipLaunchKernelGGL(k_hull_flags, dim3((uint32_t)nb), dim3(kHullThreads), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess || (!job.out_xyz && !job.sync)) return e;     // the predicate alone needs no scan
    uint64_t *total = reinterpret_cast<uint64_t *>(ws + L.total);
    uint32_t *offsets = reinterpret_cast<uint32_t *>(ws + L.offsets);
    e = launch_scan(a.counts, offsets, nb, reinterpret_cast<uint64_t *>(ws + L.part), total, st);
    if (e != hipSuccess) return e;
    if (job.out_xyz && job.capacity > 0) {
        HullOut o;
        o.offsets = offsets;
        o.capacity = job.capacity;
        o.xyz = job.out_xyz;
        o.sh = job.out_sh;
        o.opacity = job.out_opacity;
        o.radius = job.out_radius;
        o.in_sh = job.sh;
        o.in_opacity = job.opacity;
        o.in_radius = job.radius;
        o.k3 = job.k3;
        hipLaunchKernelGGL(k_hull_scatter, dim3((uint32_t)nb), dim3(kHullThreads), 0, st, a, o);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!job.sync) return hipSuccess;
    return read_count(total, kept_host, st);
}

}  // namespace dpr
