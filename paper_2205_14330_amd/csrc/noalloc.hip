// dpr_render_forward_1_noalloc: the single-view forward of
// dpr_render_forward_1 with its workspace in a static device array, for
// callers that cannot allocate device memory.
//
// The array below is a device symbol.  In host code its name is only a
// host-side stand-in: the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device (with that device current) and
// kept; only that address is ever handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dpr_internal.h"

namespace {

__device__ __align__(256) unsigned char scratch[DPR_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
int scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return dpr::set_last_error(DPR_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return dpr::set_last_error(DPR_ERR_UNSUPPORTED, "device %d: the static scratch covers devices 0..%d", dev,
                                   kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return dpr::set_last_error(DPR_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                                       hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DPR_OK;
}

}  // namespace

extern "C" int dpr_render_forward_1_noalloc(const dpr_scene *scene, const dpr_camera *cam, const dpr_params *params,
                                            float *image, float *trans, void *stream) {
    if (!params) return dpr::set_last_error(DPR_ERR_INVALID_ARG, "params is NULL");
    if (params->flags & DPR_FLAG_TIMING)
        return dpr::set_last_error(DPR_ERR_INVALID_ARG,
                                   "DPR_FLAG_TIMING creates HIP events, which this entry point does not do");
    // The plan lives only inside this call, so no backward state is kept.
    dpr_params pr = *params;
    pr.bwd_mode = DPR_BWD_RECOMPUTE;
    void *ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    size_t need = 0;
    rc = dpr_render_forward_1(scene, cam, &pr, image, trans, ws, (size_t)DPR_NOALLOC_SCRATCH_BYTES, &need, stream);
    if (rc == DPR_ERR_WORKSPACE)
        return dpr::set_last_error(DPR_ERR_WORKSPACE,
                                   "this scene and camera need %zu bytes of workspace; the static scratch of "
                                   "dpr_render_forward_1_noalloc holds %llu (use dpr_render_forward_1)",
                                   need, (unsigned long long)DPR_NOALLOC_SCRATCH_BYTES);
    return rc;
}
