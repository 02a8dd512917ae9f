// Host build of the hybrid-update kernels (Sec. 3.3, Alg. 1) for checking
// their indexing under AddressSanitizer; test infrastructure only.
//
// The kernels and host sequencing of hybrid.hip compile unchanged against the
// host stand-in of <hip/hip_runtime.h>, and so do the library's flat scan and
// radix sort (sort.hip), with their real launch sequence.  Every scratch
// array is its own allocation of exactly the size the library reserves,
// filled with 0xFF, so an unset index or an access past an array's end is
// reported instead of landing in a neighbouring array.
//
//   hybrid_host knn    DIR K          DIR/xyz.bin -> DIR/idx.bin, DIR/d2.bin
//   hybrid_host voxel  DIR N k3       DIR/{xyz,sh,op,rad}.bin -> DIR/out_*.bin, DIR/counts.txt
//   hybrid_host hybrid DIR N K eps k3 same, counts = voxels kept points
#include "hybrid.hip"
#include "sort.hip"

#include <string>

#include "stand_ins.h"

namespace {

template <class T>
T *poisoned(uint64_t bytes) {
    void *p = std::malloc(bytes ? bytes : 1);
    std::memset(p, 0xFF, bytes ? bytes : 1);
    return static_cast<T *>(p);
}

struct Scratch {
    dpr::HyScratch s;
    std::vector<void *> owned;
    template <class T>
    T *take(uint64_t bytes) {
        T *p = poisoned<T>(bytes);
        owned.push_back(p);
        return p;
    }
    Scratch(uint64_t n, int K) {
        const dpr::HyScratchBytes b = dpr::hy_scratch_bytes(n, K);
        s.keys = take<uint32_t>(b.keys);
        s.vals = take<uint32_t>(b.vals);
        s.keys_alt = take<uint32_t>(b.keys_alt);
        s.vals_alt = take<uint32_t>(b.vals_alt);
        s.hist = take<uint32_t>(b.hist);
        s.part = take<uint64_t>(b.part);
        s.total64 = take<uint64_t>(b.total64);
        s.flags = take<uint32_t>(b.flags);
        s.seg = take<uint32_t>(b.seg);
        s.starts = take<uint32_t>(b.starts);
        s.cell_start = take<uint32_t>(b.cell_start);
        s.box_part = take<float>(b.box_part);
        s.box = take<float>(b.box);
        s.idx = take<int32_t>(b.idx);
        s.d2 = take<float>(b.d2);
    }
    ~Scratch() {
        for (void *p : owned) std::free(p);
    }
};

std::vector<float> read_f32(const std::string &path) {
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) {
        std::fprintf(stderr, "cannot open %s\n", path.c_str());
        std::exit(2);
    }
    std::fseek(f, 0, SEEK_END);
    const long bytes = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    std::vector<float> v((size_t)bytes / 4);
    if (std::fread(v.data(), 4, v.size(), f) != v.size()) std::exit(2);
    std::fclose(f);
    return v;
}

void write_raw(const std::string &path, const void *p, size_t bytes) {
    FILE *f = std::fopen(path.c_str(), "wb");
    if (!f || std::fwrite(p, 1, bytes, f) != bytes) std::exit(2);
    std::fclose(f);
}

// exact-size copy of a host array, so reads past its end are reported
template <class T>
T *exact_copy(const std::vector<T> &v) {
    T *p = poisoned<T>(sizeof(T) * v.size());
    std::memcpy(p, v.data(), sizeof(T) * v.size());
    return p;
}

struct Cloud {
    float *xyz, *sh, *op, *rad;
    uint64_t n;
    int k3;
    Cloud(uint64_t n_, int k3_) : n(n_), k3(k3_) {
        xyz = poisoned<float>(12 * n);
        sh = poisoned<float>(4 * n * (uint64_t)k3);
        op = poisoned<float>(4 * n);
        rad = poisoned<float>(4 * n);
    }
    ~Cloud() {
        std::free(xyz);
        std::free(sh);
        std::free(op);
        std::free(rad);
    }
    void write(const std::string &dir, uint64_t count) const {
        write_raw(dir + "/out_xyz.bin", xyz, 12 * count);
        write_raw(dir + "/out_sh.bin", sh, 4 * count * (uint64_t)k3);
        write_raw(dir + "/out_op.bin", op, 4 * count);
        write_raw(dir + "/out_rad.bin", rad, 4 * count);
    }
};

int check(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        std::fprintf(stderr, "%s failed (%d)\n", what, e);
        std::exit(3);
    }
    return 0;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc < 4) {
        std::fprintf(stderr, "usage: hybrid_host knn|voxel|hybrid DIR ...\n");
        return 2;
    }
    const std::string mode = argv[1], dir = argv[2];
    const std::vector<float> xyz_v = read_f32(dir + "/xyz.bin");
    const uint64_t n = xyz_v.size() / 3;
    float *xyz = exact_copy(xyz_v);
    if (mode == "knn") {
        const int K = std::atoi(argv[3]);
        Scratch sc(n, K);
        int32_t *idx = poisoned<int32_t>(4 * n * (uint64_t)K);
        float *d2 = poisoned<float>(4 * n * (uint64_t)K);
        check(dpr::launch_knn(xyz, (uint32_t)n, K, idx, d2, sc.s, nullptr), "knn");
        write_raw(dir + "/idx.bin", idx, 4 * n * (uint64_t)K);
        write_raw(dir + "/d2.bin", d2, 4 * n * (uint64_t)K);
        std::free(idx);
        std::free(d2);
        std::free(xyz);
        return 0;
    }
    const bool hybrid = mode == "hybrid";
    if ((hybrid && argc != 7) || (!hybrid && argc != 5)) {
        std::fprintf(stderr, "bad arguments for %s\n", mode.c_str());
        return 2;
    }
    const uint32_t N = (uint32_t)std::atoi(argv[3]);
    const int K = hybrid ? std::atoi(argv[4]) : 1;
    const float eps = hybrid ? std::strtof(argv[5], nullptr) : 0.f;
    const int k3 = std::atoi(argv[hybrid ? 6 : 4]);
    float *sh = exact_copy(read_f32(dir + "/sh.bin"));
    float *op = exact_copy(read_f32(dir + "/op.bin"));
    float *rad = exact_copy(read_f32(dir + "/rad.bin"));
    Scratch sc(n, K);
    uint64_t m = 0;
    FILE *cf = std::fopen((dir + "/counts.txt").c_str(), "w");
    if (!hybrid) {
        Cloud out(n, k3);
        check(dpr::launch_voxel_reduce(xyz, sh, op, rad, (uint32_t)n, k3, N, out.xyz, out.sh, out.op, out.rad, sc.s,
                                       &m, nullptr),
              "voxel_reduce");
        out.write(dir, m);
        std::fprintf(cf, "%llu\n", (unsigned long long)m);
    } else {
        Cloud red(n, k3), out(2 * n, k3);
        uint64_t kept = 0, count = 0;
        check(dpr::launch_voxel_reduce(xyz, sh, op, rad, (uint32_t)n, k3, N, red.xyz, red.sh, red.op, red.rad, sc.s,
                                       &m, nullptr),
              "voxel_reduce");
        check(dpr::launch_filter_generate(red.xyz, red.sh, red.op, red.rad, (uint32_t)m, k3, K, eps, out.xyz, out.sh,
                                          out.op, out.rad, sc.s, &kept, &count, nullptr),
              "filter_generate");
        out.write(dir, count);
        std::fprintf(cf, "%llu %llu %llu\n", (unsigned long long)m, (unsigned long long)kept,
                     (unsigned long long)count);
    }
    std::fclose(cf);
    std::free(xyz);
    std::free(sh);
    std::free(op);
    std::free(rad);
    return 0;
}
