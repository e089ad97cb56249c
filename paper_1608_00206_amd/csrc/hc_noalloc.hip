// The forward convolution for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Its workspace is a file-scope device array of fixed size that
// the code object holds on every GPU it is loaded on; the kernels are those
// of hc_convolve_batch, which receive the array's device address exactly as
// they receive a caller's workspace.
#include "hc.h"

#include <hip/hip_runtime.h>

#include <mutex>

#include "hc_internal.hpp"

using namespace hc;

// Host code must never pass this name to a kernel: on the host it is a
// stand-in, not a device address.  Its address on each device comes from
// hipGetSymbolAddress and is kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[HC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
int scratch_on_current_device(void** out)
{
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return fail(HC_ERR_NO_DEVICE, "no HIP device available");
    }
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(HC_ERR_NO_DEVICE, "device index %d unsupported", dev);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(HC_ERR_HIP, "hipGetSymbolAddress(scratch) gave a null address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HC_OK;
}

}  // namespace

extern "C" int hc_convolve_batch_noalloc(const void* x, const void* y, void* z, int D, int dtype, int batch,
                                         hipStream_t stream)
{
    const size_t need = hc_workspace_bytes(D, dtype, batch);
    // invalid D, dtype or batch: the checks of the shared path report them
    if (need == (size_t)-1) return convolve_batch_last(x, y, z, D, dtype, batch, nullptr, 0, stream, nullptr);
    if (need > (size_t)HC_NOALLOC_SCRATCH_BYTES)
        return fail(HC_ERR_WORKSPACE,
                    "D=%d, batch=%d needs %zu bytes of workspace; the allocation-free entry point holds %zu",
                    D, batch, need, (size_t)HC_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    if (need > 0) {
        const int rc = scratch_on_current_device(&ws);
        if (rc != HC_OK) return rc;
    }
    return convolve_batch_last(x, y, z, D, dtype, batch, ws, need > 0 ? (size_t)HC_NOALLOC_SCRATCH_BYTES : 0,
                               stream, nullptr);
}
