// Host build of the video warm-start kernels (Sec. 3.4: Chamfer distance of
// Eq. (9) and its gradient, top-k SH transfer, Adam step) for checking their
// indexing under AddressSanitizer; test infrastructure only.  chamfer.hip
// compiles unchanged against the host stand-in of <hip/hip_runtime.h>; inputs
// and outputs are allocations of exactly their size and the padding after
// each workspace region is poisoned.
//
//   chamfer_host chamfer DIR       DIR/{s1,s2}.bin -> DIR/{cd,grad2,nn12,nn21}.bin
//   chamfer_host topk    DIR k3 K  DIR/{s1,sh1,s2}.bin -> DIR/{out_sh,idx}.bin
//   chamfer_host adam    DIR t lr b1 b2 eps   DIR/{p,g,m,v}.bin -> same files, updated
#include "chamfer.hip"
#include "sort.hip"

#include <sanitizer/asan_interface.h>

#include <string>

#include "stand_ins.h"

namespace {

std::vector<uint8_t> read_bytes(const std::string &path) {
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) {
        std::fprintf(stderr, "cannot open %s\n", path.c_str());
        std::exit(2);
    }
    std::fseek(f, 0, SEEK_END);
    const long bytes = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    std::vector<uint8_t> v((size_t)bytes);
    if (bytes && std::fread(v.data(), 1, v.size(), f) != v.size()) std::exit(2);
    std::fclose(f);
    return v;
}

void write_raw(const std::string &path, const void *p, size_t bytes) {
    FILE *f = std::fopen(path.c_str(), "wb");
    if (!f || (bytes && std::fwrite(p, 1, bytes, f) != bytes)) std::exit(2);
    std::fclose(f);
}

template <class T>
T *exact(const std::vector<uint8_t> &v) {
    void *p = std::malloc(v.size() ? v.size() : 1);
    if (v.size()) std::memcpy(p, v.data(), v.size());
    return static_cast<T *>(p);
}

template <class T>
T *poisoned(uint64_t bytes) {
    void *p = std::malloc(bytes ? bytes : 1);
    std::memset(p, 0xFF, bytes ? bytes : 1);
    return static_cast<T *>(p);
}

}  // namespace

int main(int argc, char **argv) {
    if (argc < 3) return 2;
    const std::string mode = argv[1], dir = argv[2];
    if (mode == "chamfer") {
        const std::vector<uint8_t> a = read_bytes(dir + "/s1.bin"), b = read_bytes(dir + "/s2.bin");
        const uint32_t n1 = (uint32_t)(a.size() / 12), n2 = (uint32_t)(b.size() / 12);
        float *s1 = exact<float>(a), *s2 = exact<float>(b);
        const dpr::ChamferLayout L = dpr::chamfer_layout(n1, n2);
        uint8_t *ws = poisoned<uint8_t>(L.bytes);
        const uint64_t starts[] = {L.key12, L.key21, L.acc, L.cnt, L.part1, L.part2, L.bytes};
        const uint64_t sizes[] = {8ull * n1, 8ull * n2, 24ull * n2, 4ull * n2, 8ull * ((n1 + 255) / 256),
                                  8ull * ((n2 + 255) / 256)};
        for (int r = 0; r < 6; ++r)
            if (starts[r] + sizes[r] < starts[r + 1])
                ASAN_POISON_MEMORY_REGION(ws + starts[r] + sizes[r], starts[r + 1] - starts[r] - sizes[r]);
        double *cd = poisoned<double>(8);
        float *grad2 = poisoned<float>(12ull * n2);
        int32_t *nn12 = poisoned<int32_t>(4ull * n1), *nn21 = poisoned<int32_t>(4ull * n2);
        if (dpr::launch_chamfer(n1, s1, n2, s2, cd, grad2, nn12, nn21, ws, nullptr) != hipSuccess) return 3;
        write_raw(dir + "/cd.bin", cd, 8);
        write_raw(dir + "/grad2.bin", grad2, 12ull * n2);
        write_raw(dir + "/nn12.bin", nn12, 4ull * n1);
        write_raw(dir + "/nn21.bin", nn21, 4ull * n2);
        ASAN_UNPOISON_MEMORY_REGION(ws, L.bytes);
        std::free(ws); std::free(cd); std::free(grad2); std::free(nn12); std::free(nn21); std::free(s1); std::free(s2);
    } else if (mode == "topk") {
        const int k3 = std::atoi(argv[3]), K = std::atoi(argv[4]);
        const std::vector<uint8_t> a = read_bytes(dir + "/s1.bin"), h = read_bytes(dir + "/sh1.bin"),
                                   b = read_bytes(dir + "/s2.bin");
        const uint32_t n1 = (uint32_t)(a.size() / 12), n2 = (uint32_t)(b.size() / 12);
        float *s1 = exact<float>(a), *sh1 = exact<float>(h), *s2 = exact<float>(b);
        float *out = poisoned<float>(4ull * n2 * (uint64_t)k3);
        int32_t *idx = poisoned<int32_t>(4ull * n2 * (uint64_t)K);
        if (dpr::launch_topk_sh(n1, s1, sh1, n2, s2, k3, K, out, idx, nullptr) != hipSuccess) return 3;
        write_raw(dir + "/out_sh.bin", out, 4ull * n2 * (uint64_t)k3);
        write_raw(dir + "/idx.bin", idx, 4ull * n2 * (uint64_t)K);
        std::free(s1); std::free(sh1); std::free(s2); std::free(out); std::free(idx);
    } else if (mode == "adam") {
        const int t = std::atoi(argv[3]);
        const float lr = std::strtof(argv[4], nullptr), b1 = std::strtof(argv[5], nullptr),
                    b2 = std::strtof(argv[6], nullptr), eps = std::strtof(argv[7], nullptr);
        const std::vector<uint8_t> pb = read_bytes(dir + "/p.bin");
        const uint32_t n = (uint32_t)(pb.size() / 4);
        float *p = exact<float>(pb), *g = exact<float>(read_bytes(dir + "/g.bin")),
              *m = exact<float>(read_bytes(dir + "/m.bin")), *v = exact<float>(read_bytes(dir + "/v.bin"));
        if (dpr::launch_adam(n, p, g, m, v, t, lr, b1, b2, eps, nullptr) != hipSuccess) return 3;
        write_raw(dir + "/p.bin", p, 4ull * n);
        write_raw(dir + "/m.bin", m, 4ull * n);
        write_raw(dir + "/v.bin", v, 4ull * n);
        std::free(p); std::free(g); std::free(m); std::free(v);
    } else {
        return 2;
    }
    return 0;
}
