// Device exclusive scan and a segmented stable LSD radix sort.
//
// The radix sort orders each view's items by their 32-bit depth key (the
// float bits of camera Z, which order like unsigned integers for positive
// values), four 8-bit passes.  It is stable, and the items enter it in point
// index order, so equal depths keep ascending point index: the tie-break of
// the front-to-back order (Sec. 3.2: points sorted by z-distance).
//
// Segmentation costs nothing extra: the per-block digit histograms are laid
// out view-major ([view][digit][block of view]); a block's output positions
// are its view's first item, plus the view's counts of the smaller digits,
// plus its digit's counts in the view's earlier blocks, so they stay inside
// each view's item range.
#include "dpr_internal.h"

namespace dpr {

// ---------------------------------------------------------------------------
// wave / block primitives (64-lane wavefronts)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

// Exclusive scan over the block (any multiple of 64 threads); returns the block total in *total.
__device__ __forceinline__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t *s_wave, uint32_t *total) {
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const uint32_t incl = wave_incl_scan_u32(v);
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
        const uint32_t c = s_wave[w];
        if (w < wave) base += c;
        tot += c;
    }
    *total = tot;
    __syncthreads();
    return base + incl - v;
}

// ---------------------------------------------------------------------------
// scan: reduce -> scan partials -> downsweep
// ---------------------------------------------------------------------------
uint64_t scan_partials(uint64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t *in, uint64_t n, uint64_t *part) {
    __shared__ uint64_t s[kScanThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint64_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItemsPerThread; ++j) {
        const uint64_t idx = base + (uint64_t)j * kScanThreads + threadIdx.x;
        if (idx < n) sum += in[idx];
    }
    sum = wave_sum_u64(sum);
    if (__lane_id() == 0) s[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) t += s[w];
        part[blockIdx.x] = t;
    }
}

// One block: exclusive scan of nb partials in place; total to *total64 and
// the low 32 bits of it to out[n].
__global__ __launch_bounds__(kScanThreads) void k_scan_partials(uint64_t *part, uint64_t nb, uint64_t *total64,
                                                                uint32_t *out, uint64_t n) {
    __shared__ uint64_t s_w[kScanThreads / 64];
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    uint64_t carry = 0;
    for (uint64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        const uint64_t idx = b0 + threadIdx.x;
        const uint64_t v = idx < nb ? part[idx] : 0;
        uint64_t incl = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            uint64_t o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        if (lane == 63) s_w[wave] = incl;
        __syncthreads();
        uint64_t base = carry, tot = 0;
        for (int w = 0; w < kScanThreads / 64; ++w) {
            if (w < wave) base += s_w[w];
            tot += s_w[w];
        }
        if (idx < nb) part[idx] = base + incl - v;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *total64 = carry;
        out[n] = (uint32_t)carry;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t *in, uint32_t *out, uint64_t n,
                                                            const uint64_t *part) {
    __shared__ uint32_t s_wave[kScanThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItemsPerThread;
    uint32_t v[kScanItemsPerThread];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItemsPerThread; ++j) {
        const uint64_t idx = base + j;
        v[j] = idx < n ? in[idx] : 0u;
        sum += v[j];
    }
    uint32_t total;
    uint32_t run = block_excl_scan_u32(sum, s_wave, &total) + (uint32_t)part[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItemsPerThread; ++j) {
        const uint64_t idx = base + j;
        if (idx < n) out[idx] = run;
        run += v[j];
    }
}

// Downsweep for a scan of few blocks: each block adds up the partials of the
// blocks before it itself (at most kScanFewBlocks values), and the last block
// writes the total, so no separate scan of the partials is launched.
constexpr uint64_t kScanFewBlocks = 512;

__global__ __launch_bounds__(kScanThreads) void k_scan_down_few(const uint32_t *in, uint32_t *out, uint64_t n,
                                                                const uint64_t *part, uint64_t *total64) {
    __shared__ uint32_t s_wave[kScanThreads / 64];
    __shared__ uint64_t s_pre[kScanThreads / 64];
    uint64_t pre = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kScanThreads) pre += part[b];
    pre = wave_sum_u64(pre);
    if (__lane_id() == 0) s_pre[threadIdx.x >> 6] = pre;
    __syncthreads();
    uint64_t block_base = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; ++w) block_base += s_pre[w];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItemsPerThread;
    uint32_t v[kScanItemsPerThread];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItemsPerThread; ++j) {
        const uint64_t idx = base + j;
        v[j] = idx < n ? in[idx] : 0u;
        sum += v[j];
    }
    uint32_t total;
    uint32_t run = block_excl_scan_u32(sum, s_wave, &total) + (uint32_t)block_base;
#pragma unroll
    for (int j = 0; j < kScanItemsPerThread; ++j) {
        const uint64_t idx = base + j;
        if (idx < n) out[idx] = run;
        run += v[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const uint64_t t = block_base + total;
        *total64 = t;
        out[n] = (uint32_t)t;
    }
}

hipError_t launch_scan(const uint32_t *in, uint32_t *out, uint64_t n, uint64_t *part,
                       uint64_t *total64, hipStream_t st) {
    const uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb > 0 && nb <= kScanFewBlocks) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)nb), dim3(kScanThreads), 0, st, in, n, part);
        hipLaunchKernelGGL(k_scan_down_few, dim3((uint32_t)nb), dim3(kScanThreads), 0, st, in, out, n, part, total64);
        return hipGetLastError();
    }
    if (nb > 0) {
        hipLaunchKernelGGL(k_scan_reduce, dim3((uint32_t)nb), dim3(kScanThreads), 0, st, in, n, part);
    }
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanThreads), 0, st, part, nb, total64, out, n);
    if (nb > 0) {
        hipLaunchKernelGGL(k_scan_down, dim3((uint32_t)nb), dim3(kScanThreads), 0, st, in, out, n, part);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// segmented radix sort
// ---------------------------------------------------------------------------
struct SortSeg {
    uint32_t lb;       // block index within the segment
    uint32_t beg, end; // item range of this block
    uint32_t nsb;      // sort blocks of the segment
    uint32_t base;     // first item of the segment
    uint64_t hist_off;
};

// Segments = the views of a plan (the depth sort), blocks of kDepthSortTile keys.
struct ViewSegs {
    Tables tb;
    __device__ __forceinline__ SortSeg operator()() const {
        const int v = find_segment(tb.sort_block_start, tb.n_views, blockIdx.x);
        const ViewDesc &vd = tb.views[v];
        SortSeg s;
        s.lb = blockIdx.x - vd.sort_block_off;
        s.base = vd.item_off;
        s.beg = vd.item_off + s.lb * (uint32_t)kDepthSortTile;
        s.end = min(s.beg + (uint32_t)kDepthSortTile, vd.item_off + (uint32_t)vd.n);
        s.nsb = vd.nsort_blocks;
        s.hist_off = vd.hist_off;
        return s;
    }
};

// One segment of n keys, blocks of kSortTile keys.
struct FlatSeg {
    uint32_t n, nblocks;
    __device__ __forceinline__ SortSeg operator()() const {
        SortSeg s;
        s.lb = blockIdx.x;
        s.base = 0;
        s.beg = blockIdx.x * (uint32_t)kSortTile;
        s.end = min(s.beg + (uint32_t)kSortTile, n);
        s.nsb = nblocks;
        s.hist_off = 0;
        return s;
    }
};

template <int THREADS, class SEG>
__global__ __launch_bounds__(THREADS) void k_radix_hist(SEG seg, const uint32_t *keys, uint32_t *hist, int shift) {
    __shared__ uint32_t h[256];
    const SortSeg sg = seg();
    for (uint32_t d = threadIdx.x; d < 256u; d += THREADS) h[d] = 0;
    __syncthreads();
    // eight keys per thread loaded together, then counted
    for (uint32_t i0 = sg.beg + threadIdx.x; i0 < sg.end; i0 += 8u * THREADS) {
        uint32_t kk[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = i0 + (uint32_t)u * THREADS;
            kk[u] = i < sg.end ? keys[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i0 + (uint32_t)u * THREADS < sg.end) atomicAdd(&h[(kk[u] >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < 256u; d += THREADS)
        hist[sg.hist_off + (uint64_t)d * sg.nsb + sg.lb] = h[d];
}

// Stable scatter of one block of THREADS * ITEMS keys by one 8-bit digit.
// OWN_OFFSETS: `offs` is the raw histogram ([digit][block] per segment), and
// the block adds up the output base of each of its digits itself (the
// segment's totals of the smaller digits and its own digit's counts in the
// earlier blocks: at most 256 x the segment's blocks reads); otherwise `offs`
// is the exclusive scan of the histogram.
template <int THREADS, int ITEMS, bool OWN_OFFSETS, class SEG>
__global__ __launch_bounds__(THREADS) void k_radix_scatter(SEG seg, const uint32_t *keys_in,
                                                          const uint32_t *vals_in, uint32_t *keys_out,
                                                          uint32_t *vals_out, const uint32_t *offs, int shift) {
    constexpr int TILE = THREADS * ITEMS, WAVES = THREADS / 64;
    static_assert(THREADS >= 256 && THREADS % 64 == 0, "one thread per digit");
    __shared__ uint32_t s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];
    __shared__ uint32_t s_wcnt[WAVES][256];
    __shared__ uint32_t s_run[256];
    __shared__ uint32_t s_start[256];
    __shared__ uint32_t s_gbase[256];
    __shared__ uint32_t s_wave[WAVES];

    const SortSeg sg = seg();
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    const uint32_t tid = threadIdx.x;

    if (tid < 256u) s_run[tid] = 0;
    uint32_t k_[ITEMS], v_[ITEMS], r_[ITEMS];
    // the thread's keys and values, all loads in flight together (the
    // ranking rounds below are separated by barriers, past which the
    // compiler does not move loads)
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = sg.beg + (uint32_t)r * THREADS + tid;
        const bool valid = idx < sg.end;
        k_[r] = valid ? keys_in[idx] : 0u;
        v_[r] = valid ? vals_in[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = sg.beg + (uint32_t)r * THREADS + tid;
        const bool valid = idx < sg.end;
        const uint32_t key = k_[r];
        const uint32_t d = (key >> shift) & 255u;
#pragma unroll
        for (int q = 0; q < 4; ++q) s_wcnt[wave][lane + 64 * q] = 0;
        __syncthreads();
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t lrank = (uint32_t)__popcll(peers & lt_mask);
        if (valid && lrank == 0) s_wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (tid < 256u) {   // digit tid: running count + earlier waves of this round
            uint32_t acc = s_run[tid];
#pragma unroll
            for (int w = 0; w < WAVES; ++w) {
                const uint32_t c = s_wcnt[w][tid];
                s_wcnt[w][tid] = acc;
                acc += c;
            }
            s_run[tid] = acc;
        }
        __syncthreads();
        r_[r] = valid ? s_wcnt[wave][d] + lrank : 0xFFFFFFFFu;
        __syncthreads();
    }
    // local start of every digit, and the global base of this block's digit runs
    uint32_t total;
    const uint32_t cnt = tid < 256u ? s_run[tid] : 0u;
    const uint32_t start = block_excl_scan_u32(cnt, s_wave, &total);
    if (tid < 256u) s_start[tid] = start;
    if (OWN_OFFSETS) {
        uint32_t tot = 0, pre = 0;
        if (tid < 256u) {
            const uint32_t *hd = offs + sg.hist_off + (uint64_t)tid * sg.nsb;
            for (uint32_t b = 0; b < sg.nsb; ++b) {
                const uint32_t v = hd[b];
                tot += v;
                pre += b < sg.lb ? v : 0u;
            }
        }
        uint32_t all;
        const uint32_t below = block_excl_scan_u32(tot, s_wave, &all);
        if (tid < 256u) s_gbase[tid] = sg.base + below + pre;
    } else {
        if (tid < 256u) s_gbase[tid] = offs[sg.hist_off + (uint64_t)tid * sg.nsb + sg.lb];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        if (r_[r] != 0xFFFFFFFFu) {
            const uint32_t d = (k_[r] >> shift) & 255u;
            const uint32_t pos = s_start[d] + r_[r];
            s_keys[pos] = k_[r];
            s_vals[pos] = v_[r];
        }
    }
    __syncthreads();
    const uint32_t count = sg.end > sg.beg ? sg.end - sg.beg : 0u;
    for (uint32_t i = tid; i < count; i += THREADS) {
        const uint32_t key = s_keys[i];
        const uint32_t d = (key >> shift) & 255u;
        const uint32_t dst = s_gbase[d] + (i - s_start[d]);
        keys_out[dst] = key;
        vals_out[dst] = s_vals[i];
    }
}

// The same scatter with each wave owning a contiguous run of ITEMS * 64 keys
// (the input order is wave-major, then round, then lane): a wave ranks its
// keys with its own digit counters, round after round, with no block
// barrier; one barrier then turns the counters into per-wave bases.  Used by
// the depth sort, with its own offsets.
template <int THREADS, int ITEMS, class SEG>
__global__ __launch_bounds__(THREADS) void k_radix_scatter_wm(SEG seg, const uint32_t *keys_in,
                                                             const uint32_t *vals_in, uint32_t *keys_out,
                                                             uint32_t *vals_out, const uint32_t *hist, int shift) {
    constexpr int TILE = THREADS * ITEMS, WAVES = THREADS / 64;
    static_assert(THREADS >= 256 && THREADS % 256 == 0, "whole threads per digit");
    __shared__ uint32_t s_keys[TILE];
    __shared__ uint32_t s_vals[TILE];
    __shared__ uint32_t s_wcnt[WAVES][256];
    __shared__ uint32_t s_start[256];
    __shared__ uint32_t s_gbase[256];
    __shared__ uint32_t s_wave[WAVES];

    constexpr int QUARTERS = THREADS / 256;
    __shared__ uint32_t s_tot[QUARTERS][256], s_pre[QUARTERS][256];
    const SortSeg sg = seg();
    const uint32_t lane = (uint32_t)__lane_id();
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t tid = threadIdx.x;
    const uint64_t lt_mask = (1ull << lane) - 1ull;
    // this block's offsets, issued first so that their loads overlap the
    // ranking: thread (q, d) sums digit d's counts over blocks q, q + QUARTERS, ...
    uint32_t tot_q = 0, pre_q = 0;
    {
        const uint32_t d = tid & 255u, q = tid >> 8;
        const uint32_t *hd = hist + sg.hist_off + (uint64_t)d * sg.nsb;
#pragma unroll 4
        for (uint32_t b = q; b < sg.nsb; b += QUARTERS) {
            const uint32_t v = hd[b];
            tot_q += v;
            pre_q += b < sg.lb ? v : 0u;
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) s_wcnt[wave][lane + 64 * q] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    uint32_t k_[ITEMS], v_[ITEMS], r_[ITEMS];
    const uint32_t wbeg = sg.beg + wave * (uint32_t)(ITEMS * 64);
    // the wave's keys and values, all loads in flight together (the ranking
    // rounds below are separated by fences, past which the compiler does not
    // move loads)
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = wbeg + (uint32_t)r * 64u + lane;
        const bool valid = idx < sg.end;
        k_[r] = valid ? keys_in[idx] : 0u;
        v_[r] = valid ? vals_in[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = wbeg + (uint32_t)r * 64u + lane;
        const bool valid = idx < sg.end;
        const uint32_t d = (k_[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t lrank = (uint32_t)__popcll(peers & lt_mask);
        // every lane of a digit reads the counter before its first lane adds
        // the digit's count (one wave: its LDS operations complete in order)
        const uint32_t before = s_wcnt[wave][d];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (valid && lrank == 0) s_wcnt[wave][d] = before + (uint32_t)__popcll(peers);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        r_[r] = valid ? before + lrank : 0xFFFFFFFFu;
    }
    __syncthreads();
    // digit tid: the waves' counts -> per-wave bases, and the block's total
    uint32_t cnt = 0;
    if (tid < 256u) {
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
            const uint32_t c = s_wcnt[w][tid];
            s_wcnt[w][tid] = cnt;
            cnt += c;
        }
    }
    uint32_t total;
    const uint32_t start = block_excl_scan_u32(cnt, s_wave, &total);
    if (tid < 256u) s_start[tid] = start;
    s_tot[tid >> 8][tid & 255u] = tot_q;
    s_pre[tid >> 8][tid & 255u] = pre_q;
    __syncthreads();
    uint32_t tot = 0, pre = 0;
    if (tid < 256u) {
#pragma unroll
        for (int q = 0; q < QUARTERS; ++q) {
            tot += s_tot[q][tid];
            pre += s_pre[q][tid];
        }
    }
    uint32_t all;
    const uint32_t below = block_excl_scan_u32(tot, s_wave, &all);
    if (tid < 256u) s_gbase[tid] = sg.base + below + pre;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        if (r_[r] != 0xFFFFFFFFu) {
            const uint32_t d = (k_[r] >> shift) & 255u;
            const uint32_t pos = s_start[d] + s_wcnt[wave][d] + r_[r];
            s_keys[pos] = k_[r];
            s_vals[pos] = v_[r];
        }
    }
    __syncthreads();
    const uint32_t count = sg.end > sg.beg ? sg.end - sg.beg : 0u;
    for (uint32_t i = tid; i < count; i += THREADS) {
        const uint32_t key = s_keys[i];
        const uint32_t d = (key >> shift) & 255u;
        const uint32_t dst = s_gbase[d] + (i - s_start[d]);
        keys_out[dst] = key;
        vals_out[dst] = s_vals[i];
    }
}

// The depth sort: 4 passes of 2 launches (histogram, scatter with its own
// offsets); the histogram of a view is small enough (256 x its blocks of
// kDepthSortTile keys) for every block to read the part it needs.
hipError_t launch_depth_sort(const Tables &tb, uint32_t sort_blocks, uint32_t items,
                             uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                             uint32_t *hist, uint64_t *part, hipStream_t st) {
    (void)items;
    (void)part;
    if (sort_blocks == 0) return hipSuccess;
    uint32_t *kin = keys, *vin = vals, *kout = keys_alt, *vout = vals_alt;
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 8 * pass;
        const ViewSegs seg{tb};
        hipLaunchKernelGGL((k_radix_hist<kDepthSortThreads, ViewSegs>), dim3(sort_blocks), dim3(kDepthSortThreads),
                           0, st, seg, kin, hist, shift);
        hipLaunchKernelGGL((k_radix_scatter_wm<kDepthSortThreads, kDepthSortTile / kDepthSortThreads, ViewSegs>),
                           dim3(sort_blocks), dim3(kDepthSortThreads), 0, st, seg, kin, vin, kout, vout, hist,
                           shift);
        uint32_t *t;
        t = kin; kin = kout; kout = t;
        t = vin; vin = vout; vout = t;
    }
    return hipGetLastError();
}

uint64_t radix_hist_words(uint64_t n) { return ((n + kSortTile - 1) / kSortTile) * 256u; }

hipError_t launch_radix_sort(uint32_t n, int bits, uint32_t *keys, uint32_t *vals, uint32_t *keys_alt,
                             uint32_t *vals_alt, uint32_t *hist, uint64_t *part, bool *in_alt, hipStream_t st) {
    *in_alt = false;
    if (n == 0) return hipSuccess;
    const uint32_t nb = (n + kSortTile - 1) / kSortTile;
    const uint64_t nh = (uint64_t)nb * 256u;
    const FlatSeg seg{n, nb};
    uint32_t *kin = keys, *vin = vals, *kout = keys_alt, *vout = vals_alt;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL((k_radix_hist<kSortThreads, FlatSeg>), dim3(nb), dim3(kSortThreads), 0, st, seg, kin, hist,
                           shift);
        hipError_t e = launch_scan(hist, hist, nh, part, part + scan_partials(nh), st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_radix_scatter<kSortThreads, kSortItemsPerThread, false, FlatSeg>), dim3(nb),
                           dim3(kSortThreads), 0, st, seg, kin, vin, kout, vout, hist, shift);
        uint32_t *t;
        t = kin; kin = kout; kout = t;
        t = vin; vin = vout; vout = t;
        *in_alt = !*in_alt;
    }
    return hipGetLastError();
}

}  // namespace dpr
