// noalloc.hip -- the stiffness product for callers that cannot allocate device memory.
//
// ebbx_fem_Kmul keeps its scratch (the shared-vertex partials of the block strategies, the
// per-corner partials of SEG) in buffers the domain allocates when its strategy is set.
// This variant runs the same kernels with that scratch in one file-scope device array
// instead, so a call allocates nothing: it suits code under stream capture, serving loops
// and harnesses that forbid allocation.  Each GPU holds its own copy of the array for the
// life of the process; every call on one GPU shares it, so calls that overlap on one GPU
// (other streams, other threads) race.  Every scratch entry a call reads is written
// earlier in the same call, so nothing needs clearing between calls.
#include <mutex>

#include "fem.h"

namespace ebbx {
namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)EBBX_NOALLOC_SCRATCH_MIB << 20;
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// The device address of the current device's copy of the array, looked up once per
// device (the host-side name of the array is not a device address).
void *device_scratch() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) fail(EBBX_E_ARG, "device %d is beyond the %d devices supported", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(EBBX_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace ebbx

using namespace ebbx;

extern "C" ebbx_status ebbx_fem_Kmul_noalloc(ebbx_fem fem, const double *d, const double *u, double *y,
                                             int32_t accumulate, ebbx_stream stream) {
    EBBX_API_BEGIN
    auto *F = check_fem(fem);
    if ((!d || !u || !y) && F->nv > 0) fail(EBBX_E_ARG, "d, u or y is NULL");
    const size_t bytes = (size_t)(3 * F->nv) * sizeof(double);
    if (F->nv > 0 && (overlap(d, y, bytes) || overlap(u, y, bytes)))
        fail(EBBX_E_PHASE, "y aliases d or u (read-only and reduce phases overlap)");
    const size_t need = elem_scratch_bytes(F, OP_KMUL);
    if (need > NOALLOC_SCRATCH_BYTES)
        fail(EBBX_E_ARG, "this domain's stiffness product needs %zu bytes of scratch, beyond the %zu of the "
             "allocation-free call; use ebbx_fem_Kmul or a strategy with less scratch", need, NOALLOC_SCRATCH_BYTES);
    void *p = need > 0 ? device_scratch() : nullptr;
    elem_launch(F, OP_KMUL, d, u, y, accumulate ? 1 : 0, (hipStream_t)stream, nullptr, nullptr, nullptr, true, p);
    EBBX_API_END
}
