// rt_subcycle_noalloc: the subcycle driver of rt_subcycle for callers that
// cannot allocate device memory during the call (code under stream capture,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The only scratch memory of a subcycle call beyond the state's fields and
// its face-state buffer (both allocated when the state is created) is the
// per-workgroup partials of the flux and chemistry kernels, the first-stage
// reduction records and the diagnostics record.  Here they live in one
// static device array, `scratch`, of kNoAllocScratchBytes per device.  Its
// device address is looked up once per device with hipGetSymbolAddress (the
// array's name in host code is only a host-side stand-in) and every use goes
// through that address.  All calls on one device share the array: calls
// that overlap on one device race, and each call clears the partials it
// uses before its first kernel.  rt_subcycle's roll-back copy is not kept.

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "rt.h"
#include "rt_internal.hpp"
#include "rt_kernels.hpp"

using namespace rtk;

namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)RT_NOALLOC_SCRATCH_MB << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev`, looked up on the
// first call for that device.
int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return rt_fail(RT_EDEVICE, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return rt_fail(RT_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RT_OK;
}

}  // namespace

extern "C" int rt_subcycle_noalloc(rt_state* s, int n, double dt, void* hip_stream) {
    if (!s) return rt_fail(RT_EINVAL, "null state");
    if (n < 0) return rt_fail(RT_EINVAL, "n_subcycles=%d", n);
    if (!std::isfinite(dt)) return rt_fail(RT_EINVAL, "dt=%g", dt);
    if (!(dt <= 0) && !(dt <= s->dt_cfl)) return rt_fail(RT_EINVAL, "dt=%g above the CFL step %g", dt, s->dt_cfl);
    const size_t need = rt_partial_bytes(s->n_fblk, s->n_cblk);
    if (need > kNoAllocScratchBytes)
        return rt_fail(RT_EINVAL,
                       "rt_subcycle_noalloc: %lld cells x %d bins need %zu bytes of scratch, more than the %zu of "
                       "its static array (RT_NOALLOC_SCRATCH_MB); use rt_subcycle",
                       (long long)s->nc, s->nb, need, kNoAllocScratchBytes);
    if (!s->fused() && !s->FV.ptr) return rt_fail(RT_ESTATE, "the split transport path has no face-state buffer");
    DeviceGuard dg(s->mesh->device);
    void* base = nullptr;
    int rc = scratch_address(s->mesh->device, &base);
    if (rc) return rc;
    // Redirect the partials into the static array for this call; profiling
    // (which creates events) is off for the call.
    const PartialBufs own = s->pb;
    const bool prof = s->prof;
    s->pb = rt_partials_at(base, s->n_fblk, s->n_cblk);
    s->prof = false;
    rc = rt_subcycle_run(s, n, dt <= 0 ? s->dt_cfl : dt, (hipStream_t)hip_stream, false);
    s->pb = own;
    s->prof = prof;
    return rc;
}
