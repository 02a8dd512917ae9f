// Sequential host stand-ins for the library routines that the kernels under
// test call but that live in other sources (flat scan, radix sort, fill,
// small-table upload).  Each keeps its routine's contract: it touches exactly the scratch
// words the library's version uses, and the sort leaves its result in the
// buffer the library's would.  Test infrastructure only.
#pragma once

#include <algorithm>
#include <utility>
#include <vector>

namespace dpr {

uint64_t scan_partials(uint64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }
uint64_t radix_hist_words(uint64_t n) { return ((n + kSortTile - 1) / kSortTile) * 256u; }

hipError_t launch_scan(const uint32_t *in, uint32_t *out, uint64_t n, uint64_t *part, uint64_t *total64,
                       hipStream_t) {
    const uint64_t np = scan_partials(n);
    for (uint64_t i = 0; i < np; ++i) part[i] = 0;
    uint64_t s = 0;
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t v = in[i];
        out[i] = (uint32_t)s;
        s += v;
    }
    out[n] = (uint32_t)s;
    *total64 = s;
    return hipSuccess;
}

hipError_t launch_radix_sort(uint32_t n, int bits, uint32_t *keys, uint32_t *vals, uint32_t *keys_alt,
                             uint32_t *vals_alt, uint32_t *hist, uint64_t *part, bool *in_alt, hipStream_t) {
    *in_alt = false;
    if (n == 0 || bits == 0) return hipSuccess;
    const uint64_t nh = radix_hist_words(n);
    for (uint64_t i = 0; i <= nh; ++i) hist[i] = 0;
    for (uint64_t i = 0; i <= scan_partials(nh); ++i) part[i] = 0;
    std::vector<std::pair<uint32_t, uint32_t>> kv(n);
    for (uint32_t i = 0; i < n; ++i) {
        if (bits < 32 && (keys[i] >> bits) != 0) {
            std::fprintf(stderr, "radix sort: key %u of item %u has more than %d bits\n", keys[i], i, bits);
            std::abort();
        }
        kv[i] = {keys[i], vals[i]};
    }
    std::stable_sort(kv.begin(), kv.end(), [](const auto &a, const auto &b) { return a.first < b.first; });
    *in_alt = ((bits + 7) / 8) % 2 == 1;
    uint32_t *ko = *in_alt ? keys_alt : keys, *vo = *in_alt ? vals_alt : vals;
    for (uint32_t i = 0; i < n; ++i) {
        ko[i] = kv[i].first;
        vo[i] = kv[i].second;
    }
    return hipSuccess;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t) {
    for (uint64_t i = 0; i < n; ++i) p[i] = value;
    return hipSuccess;
}

hipError_t upload_async(void *dst, const void *src, size_t bytes, hipStream_t) {
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    std::memcpy(dst, src, bytes);
    return hipSuccess;
}

}  // namespace dpr
