// Host stand-in for the part of the HIP runtime and device library that the
// hybrid-update, visual-hull and warm-start kernels and the library's scan
// and radix sort use, so that those kernels compile with g++ and run on
// CPU threads under AddressSanitizer.  Test infrastructure only: it checks the
// kernels' indexing and host sequencing, not GPU code generation.
//
// Execution model: the blocks of a launch run one after another; the threads
// of a block run concurrently on a pool of host threads, so __syncthreads,
// 64-lane __shfl_xor and __ballot are real barriers.  __shared__ variables are function
// statics, which is block-shared memory when one block runs at a time.
#pragma once

#include <algorithm>
#include <barrier>
#include <cmath>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) alignas(n)

struct dim3 {
    uint32_t x, y, z;
    dim3(uint32_t x_ = 1, uint32_t y_ = 1, uint32_t z_ = 1) : x(x_), y(y_), z(z_) {}
};
struct HostIdx {
    uint32_t x = 0, y = 0, z = 0;
};
inline thread_local HostIdx threadIdx;
inline thread_local HostIdx blockIdx;
inline HostIdx blockDim, gridDim;

struct float2 { float x, y; };
struct float4 { float x, y, z, w; };
struct uint2 { uint32_t x, y; };
struct uint4 { uint32_t x, y, z, w; };
inline uint2 make_uint2(uint32_t x, uint32_t y) { return uint2{x, y}; }
inline float2 make_float2(float x, float y) { return float2{x, y}; }
inline float4 make_float4(float x, float y, float z, float w) { return float4{x, y, z, w}; }

typedef int hipError_t;
constexpr hipError_t hipSuccess = 0;
constexpr hipError_t hipErrorInvalidValue = 1;
typedef void *hipStream_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };

inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
inline hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind, hipStream_t) {
    std::memcpy(dst, src, bytes);
    return hipSuccess;
}

// Arithmetic: the build uses -ffp-contract=off, so each operator rounds once.
inline float __fadd_rn(float a, float b) { return a + b; }
inline float __fsub_rn(float a, float b) { return a - b; }
inline float __fmul_rn(float a, float b) { return a * b; }
inline float __fdiv_rn(float a, float b) { return a / b; }
// median of three (v_med3_f32 for finite operands)
inline float __builtin_amdgcn_fmed3f(float a, float b, float c) {
    const float lo = a < b ? a : b, hi = a < b ? b : a;
    const float m = hi < c ? hi : c;
    return lo < m ? m : lo;
}
// leading zero bits of a 32-bit word (32 for zero)
inline int __clz(unsigned x) { return x ? __builtin_clz(x) : 32; }
inline float __fmaf_rn(float a, float b, float c) { return std::fma(a, b, c); }
inline uint32_t __float_as_uint(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    return u;
}
inline float __uint_as_float(uint32_t u) {
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
template <class T>
inline T min(T a, T b) { return b < a ? b : a; }
template <class T>
inline T max(T a, T b) { return a < b ? b : a; }

namespace hostrt {

constexpr uint32_t kMaxBlock = 256;

struct Block {
    std::unique_ptr<std::barrier<>> bar;                 // the block's threads
    std::unique_ptr<std::barrier<>> wave[kMaxBlock / 64];  // each wave's lanes
    uint64_t slot[kMaxBlock];                            // shuffle exchange
};

// A pool of kMaxBlock threads; thread t runs thread t of the current block.
class Pool {
  public:
    Pool() : start_(kMaxBlock + 1), end_(kMaxBlock + 1) {
        for (uint32_t t = 0; t < kMaxBlock; ++t) threads_.emplace_back([this, t] { worker(t); });
    }
    ~Pool() {
        quit_ = true;
        start_.arrive_and_wait();
        for (auto &th : threads_) th.join();
    }
    void run(dim3 grid, dim3 block, const std::function<void()> &body) {
        if (block.x == 0 || block.x > kMaxBlock || block.y != 1 || block.z != 1 || grid.z != 1) {
            std::fprintf(stderr, "host launch: unsupported shape grid %u block %u\n", grid.x, block.x);
            std::abort();
        }
        gridDim.x = grid.x;
        gridDim.y = grid.y;
        blockDim.x = block.x;
        body_ = &body;
        for (uint32_t by = 0; by < grid.y; ++by)
            for (uint32_t b = 0; b < grid.x; ++b) {
                blk_.bar = std::make_unique<std::barrier<>>(block.x);
                for (uint32_t w = 0; w < (block.x + 63) / 64; ++w)
                    blk_.wave[w] = std::make_unique<std::barrier<>>(std::min<uint32_t>(64, block.x - 64 * w));
                block_ = b;
                block_y_ = by;
                start_.arrive_and_wait();
                end_.arrive_and_wait();
            }
    }
    Block &block() { return blk_; }

  private:
    void worker(uint32_t t) {
        for (;;) {
            start_.arrive_and_wait();
            if (quit_) return;
            if (t < blockDim.x) {
                threadIdx.x = t;
                blockIdx.x = block_;
                blockIdx.y = block_y_;
                (*body_)();
                // an exited thread no longer takes part in barriers, and a
                // ballot reads its predicate as 0
                blk_.slot[t] = 0;
                blk_.wave[t / 64]->arrive_and_drop();
                blk_.bar->arrive_and_drop();
            }
            end_.arrive_and_wait();
        }
    }
    std::vector<std::thread> threads_;
    std::barrier<> start_, end_;
    const std::function<void()> *body_ = nullptr;
    uint32_t block_ = 0, block_y_ = 0;
    Block blk_;
    bool quit_ = false;
};

inline Pool &pool() {
    static Pool p;
    return p;
}

template <class... P, class... A>
inline void launch(void (*kernel)(P...), dim3 grid, dim3 block, A... args) {
    if (grid.x == 0) return;
    const std::function<void()> body = [=] { kernel(args...); };
    pool().run(grid, block, body);
}

}  // namespace hostrt

inline void __syncthreads() { hostrt::pool().block().bar->arrive_and_wait(); }

template <class T>
inline T __shfl_xor(T v, int mask, int width = 64) {
    static_assert(sizeof(T) <= 8, "shuffle of a value wider than 8 bytes");
    if (width != 64) std::abort();
    hostrt::Block &b = hostrt::pool().block();
    const uint32_t t = threadIdx.x;
    uint64_t bits = 0;
    std::memcpy(&bits, &v, sizeof(T));
    b.slot[t] = bits;
    b.wave[t / 64]->arrive_and_wait();
    const uint64_t o = b.slot[(t & ~63u) | ((t & 63u) ^ (uint32_t)mask)];
    b.wave[t / 64]->arrive_and_wait();
    T r;
    std::memcpy(&r, &o, sizeof(T));
    return r;
}

inline int __lane_id() { return (int)(threadIdx.x & 63u); }

// A memory fence of the given order and scope; here a full fence of the host.
inline void __builtin_amdgcn_fence(int, const char *) { std::atomic_thread_fence(std::memory_order_seq_cst); }

// The lanes of a wave run in lockstep on the GPU; here they meet at a barrier.
inline void __builtin_amdgcn_wave_barrier() {
    hostrt::pool().block().wave[threadIdx.x / 64]->arrive_and_wait();
}

// Lane l receives lane l - delta's value; lanes below delta keep their own.
template <class T>
inline T __shfl_up(T v, unsigned delta, int width = 64) {
    static_assert(sizeof(T) <= 8, "shuffle of a value wider than 8 bytes");
    if (width != 64) std::abort();
    hostrt::Block &b = hostrt::pool().block();
    const uint32_t t = threadIdx.x;
    uint64_t bits = 0;
    std::memcpy(&bits, &v, sizeof(T));
    b.slot[t] = bits;
    b.wave[t / 64]->arrive_and_wait();
    const uint64_t o = b.slot[(t & 63u) >= delta ? t - delta : t];
    b.wave[t / 64]->arrive_and_wait();
    T r;
    std::memcpy(&r, &o, sizeof(T));
    return r;
}

// 64-lane ballot: bit l of the result is lane l's predicate (lanes of the
// wave that have exited count as 0).
inline uint64_t __ballot(int pred) {
    hostrt::Block &b = hostrt::pool().block();
    const uint32_t t = threadIdx.x, w0 = t & ~63u;
    b.slot[t] = pred ? 1u : 0u;
    b.wave[t / 64]->arrive_and_wait();
    uint64_t m = 0;
    for (uint32_t l = 0; l < 64 && w0 + l < blockDim.x; ++l)
        if (b.slot[w0 + l] == 1u) m |= 1ull << l;
    b.wave[t / 64]->arrive_and_wait();
    return m;
}

// Device atomics on host memory (the threads of a block run concurrently).
inline unsigned long long atomicMin(unsigned long long *p, unsigned long long v) {
    unsigned long long old = __atomic_load_n(p, __ATOMIC_RELAXED);
    while (v < old && !__atomic_compare_exchange_n(p, &old, v, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
    }
    return old;
}
inline double atomicAdd(double *p, double v) {
    uint64_t *w = reinterpret_cast<uint64_t *>(p);
    uint64_t old = __atomic_load_n(w, __ATOMIC_RELAXED), upd;
    double o;
    do {
        std::memcpy(&o, &old, 8);
        const double n = o + v;
        std::memcpy(&upd, &n, 8);
    } while (!__atomic_compare_exchange_n(w, &old, upd, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED));
    return o;
}
inline uint32_t atomicAdd(uint32_t *p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_RELAXED); }
inline uint32_t atomicOr(uint32_t *p, uint32_t v) { return __atomic_fetch_or(p, v, __ATOMIC_RELAXED); }

inline uint32_t __umulhi(uint32_t a, uint32_t b) { return (uint32_t)(((uint64_t)a * b) >> 32); }
inline int __popc(uint32_t x) { return __builtin_popcount(x); }
inline int __popcll(uint64_t x) { return __builtin_popcountll(x); }

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) \
    hostrt::launch(kernel, dim3(grid), dim3(block), __VA_ARGS__)
