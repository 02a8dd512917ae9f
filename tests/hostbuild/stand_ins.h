// Sequential host stand-ins for the small library routines that the kernels
// under test call but that live in the compositing source (a fill, the
// small-table upload and the count read-back).  Each keeps its routine's contract.  The scan and
// the radix sort are not stood in for: the harnesses compile the library's own
// sort.hip.  Test infrastructure only.
#pragma once

#include <cstring>

namespace dpr {

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t) {
    for (uint64_t i = 0; i < n; ++i) p[i] = value;
    return hipSuccess;
}

hipError_t upload_async(void *dst, const void *src, size_t bytes, hipStream_t) {
    if (bytes % 4 != 0) return hipErrorInvalidValue;
    std::memcpy(dst, src, bytes);
    return hipSuccess;
}

hipError_t read_count(const uint64_t *dev, uint64_t *out, hipStream_t) {
    *out = *dev;
    return hipSuccess;
}

}  // namespace dpr
