// Host build of the visual-hull / consistency-check kernels (Sec. 3.1
// initialisation, the appendix's consistency check) for checking their
// indexing under AddressSanitizer; test infrastructure only.
//
// hull.hip and the library's scan (sort.hip) compile unchanged against the
// host stand-in of <hip/hip_runtime.h>; the small-table upload comes from
// stand_ins.h.  Inputs,
// masks and outputs are allocations of exactly their size, and the padding
// after each region of the workspace is poisoned, so an access past any array
// is reported.
//
//   hull_host sample DIR seed n capacity   DIR/{cams,dims,masks,box}.bin -> DIR/out_xyz.bin, DIR/count.txt
//   hull_host keep   DIR                   + DIR/xyz.bin -> DIR/keep.bin
//   hull_host filter DIR k3                + DIR/{xyz,sh,op,rad}.bin -> DIR/out_*.bin, DIR/count.txt
#include "hull.hip"
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

// The workspace of hull_layout, with the padding after each region poisoned.
uint8_t *workspace(uint64_t n, int32_t n_cams, const dpr::HullCam *tab) {
    const dpr::HullLayout L = dpr::hull_layout(n, n_cams, tab);
    uint8_t *w = poisoned<uint8_t>(L.bytes);
    const uint64_t nb = dpr::hull_blocks(n);
    const uint64_t starts[] = {L.cams, L.packed, L.bits, L.counts, L.offsets, L.part, L.total, L.bytes};
    const uint64_t sizes[] = {sizeof(dpr::HullCam) * (uint64_t)n_cams, 4 * L.words, 4ull * 32 * nb, 4 * (nb + 1),
                              4 * (nb + 1), 8 * (dpr::scan_partials(nb + 1) + 2), 8};
    for (int r = 0; r < 7; ++r)
        if (starts[r] + sizes[r] < starts[r + 1])
            ASAN_POISON_MEMORY_REGION(w + starts[r] + sizes[r], starts[r + 1] - starts[r] - sizes[r]);
    return w;
}

}  // namespace

int main(int argc, char **argv) {
    if (argc < 3) {
        std::fprintf(stderr, "usage: hull_host sample|keep|filter DIR ...\n");
        return 2;
    }
    const std::string mode = argv[1], dir = argv[2];
    const std::vector<uint8_t> cams_b = read_bytes(dir + "/cams.bin"), dims_b = read_bytes(dir + "/dims.bin"),
                               masks_b = read_bytes(dir + "/masks.bin");
    const int32_t n_cams = (int32_t)(cams_b.size() / 64);
    const float *cams = reinterpret_cast<const float *>(cams_b.data());
    const int32_t *dims = reinterpret_cast<const int32_t *>(dims_b.data());
    std::vector<dpr::HullCam> tab((size_t)n_cams);
    std::vector<uint8_t *> masks;
    uint64_t moff = 0;
    for (int32_t i = 0; i < n_cams; ++i) {
        dpr::HullCam &h = tab[(size_t)i];
        std::memcpy(h.R, cams + 16 * i, 9 * 4);
        std::memcpy(h.t, cams + 16 * i + 9, 3 * 4);
        h.fx = cams[16 * i + 12]; h.fy = cams[16 * i + 13]; h.cx = cams[16 * i + 14]; h.cy = cams[16 * i + 15];
        h.width = dims[2 * i]; h.height = dims[2 * i + 1];
        const uint64_t mb = (uint64_t)h.width * (uint64_t)h.height;
        uint8_t *m = static_cast<uint8_t *>(std::malloc(mb));
        std::memcpy(m, masks_b.data() + moff, mb);
        moff += mb;
        masks.push_back(m);
        h.mask = m;
    }
    dpr::HullJob job = {};
    job.n_cams = n_cams;
    job.cams = tab.data();
    job.sync = true;
    uint64_t kept = 0;
    std::vector<void *> owned;
    auto keep_ptr = [&](void *p) { owned.push_back(p); return p; };
    if (mode == "sample") {
        const std::vector<uint8_t> box = read_bytes(dir + "/box.bin");
        const float *b = reinterpret_cast<const float *>(box.data());
        job.seed = std::strtoull(argv[3], nullptr, 10);
        job.n = std::strtoull(argv[4], nullptr, 10);
        job.capacity = std::strtoull(argv[5], nullptr, 10);
        for (int d = 0; d < 3; ++d) { job.lo[d] = b[d]; job.hi[d] = b[3 + d]; }
        job.out_xyz = static_cast<float *>(keep_ptr(poisoned<float>(12 * job.capacity)));
        uint8_t *ws = workspace(job.n, n_cams, tab.data());
        if (dpr::launch_hull(job, ws, &kept, nullptr) != hipSuccess) return 3;
        write_raw(dir + "/out_xyz.bin", job.out_xyz, 12 * std::min<uint64_t>(kept, job.capacity));
        ASAN_UNPOISON_MEMORY_REGION(ws, dpr::hull_layout(job.n, n_cams, tab.data()).bytes);
        std::free(ws);
    } else {
        const std::vector<uint8_t> xyz_b = read_bytes(dir + "/xyz.bin");
        job.n = xyz_b.size() / 12;
        job.xyz = static_cast<const float *>(keep_ptr(exact<float>(xyz_b)));
        uint8_t *ws = workspace(job.n, n_cams, tab.data());
        if (mode == "keep") {
            job.keep = static_cast<uint8_t *>(keep_ptr(poisoned<uint8_t>(job.n)));
            job.sync = false;
            if (dpr::launch_hull(job, ws, &kept, nullptr) != hipSuccess) return 3;
            write_raw(dir + "/keep.bin", job.keep, job.n);
        } else {
            job.k3 = std::atoi(argv[3]);
            job.sh = static_cast<const float *>(keep_ptr(exact<float>(read_bytes(dir + "/sh.bin"))));
            job.opacity = static_cast<const float *>(keep_ptr(exact<float>(read_bytes(dir + "/op.bin"))));
            job.radius = static_cast<const float *>(keep_ptr(exact<float>(read_bytes(dir + "/rad.bin"))));
            job.capacity = job.n;
            job.out_xyz = static_cast<float *>(keep_ptr(poisoned<float>(12 * job.n)));
            job.out_sh = static_cast<float *>(keep_ptr(poisoned<float>(4 * job.n * (uint64_t)job.k3)));
            job.out_opacity = static_cast<float *>(keep_ptr(poisoned<float>(4 * job.n)));
            job.out_radius = static_cast<float *>(keep_ptr(poisoned<float>(4 * job.n)));
            if (dpr::launch_hull(job, ws, &kept, nullptr) != hipSuccess) return 3;
            write_raw(dir + "/out_xyz.bin", job.out_xyz, 12 * kept);
            write_raw(dir + "/out_sh.bin", job.out_sh, 4 * kept * (uint64_t)job.k3);
            write_raw(dir + "/out_op.bin", job.out_opacity, 4 * kept);
            write_raw(dir + "/out_rad.bin", job.out_radius, 4 * kept);
        }
        ASAN_UNPOISON_MEMORY_REGION(ws, dpr::hull_layout(job.n, n_cams, tab.data()).bytes);
        std::free(ws);
    }
    FILE *cf = std::fopen((dir + "/count.txt").c_str(), "w");
    std::fprintf(cf, "%llu\n", (unsigned long long)kept);
    std::fclose(cf);
    for (void *p : owned) std::free(p);
    for (uint8_t *m : masks) std::free(m);
    return 0;
}
