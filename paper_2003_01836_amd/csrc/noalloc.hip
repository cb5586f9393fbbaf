// noalloc.hip -- the FP64 direct sum of eq. 1 without any device allocation.
//
// bltc_direct stages each charge vector's sources as packed (x, y, z, q)
// records in a buffer it allocates per call.  bltc_direct_noalloc runs the
// same kernels with that staging buffer in a file-scope device array of fixed
// size, so that callers that cannot allocate (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc) can use it.  Every GPU the
// library runs on holds its own copy of the array until the process ends; the
// host side keeps each device's address of it (hipGetSymbolAddress, once per
// device with that device current) and passes that address to the kernels.
// The array's name is never used as a device address on the host.
#include "bltc.h"
#include "internal.hpp"
#include "kernels.hpp"

#include <mutex>

namespace {

// staging records of at most kNoAllocSources sources (32 B each: 32 MiB per device)
constexpr int64_t kNoAllocSources = int64_t(1) << 20;
__device__ __align__(256) double4 scratch[kNoAllocSources];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double4* g_scratch_ptr[kMaxDevices] = {};

// This device's address of `scratch`, looked up on its first use.
int scratch_for_current_device(double4** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return bltc_detail::fail(BLTC_EUNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return bltc_detail::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                         "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<double4*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return BLTC_OK;
}

}  // namespace

extern "C" int bltc_direct_noalloc(const bltc_params* p, int64_t nt, const double* tx,
                                   const double* ty, const double* tz, int64_t ns,
                                   const double* sx, const double* sy, const double* sz,
                                   const double* q, int32_t num_q, int64_t q_ld, double* phi,
                                   int64_t phi_ld, void* stream)
{
    using bltc_detail::fail;
    int rc = bltc_internal_check_direct(p, nt, tx, ty, tz, ns, sx, sy, sz, q, num_q, phi);
    if (rc != BLTC_OK)
        return rc;
    if (ns > kNoAllocSources)
        return fail(BLTC_EUNSUPPORTED,
                    "bltc_direct_noalloc takes at most %lld sources (its fixed staging array); "
                    "%lld given: use bltc_direct",
                    static_cast<long long>(kNoAllocSources), static_cast<long long>(ns));
    if (nt == 0)
        return BLTC_OK;
    double4* packed = nullptr;
    rc = scratch_for_current_device(&packed);
    if (rc != BLTC_OK)
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    bltc::KernelParams kp;
    kp.kernel = p->kernel;
    kp.kappa = p->kappa;
    kp.delta = p->delta;
    hipError_t e = hipSuccess;
    for (int32_t m = 0; m < num_q && e == hipSuccess; ++m) {
        // no sources: the direct-sum kernel writes zeros and reads no record
        if (ns > 0)
            e = bltc::launch_pack_sources(ns, sx, sy, sz, q + static_cast<int64_t>(m) * q_ld,
                                          packed, s);
        if (e == hipSuccess)
            e = bltc::launch_direct(nt, tx, ty, tz, ns, packed, kp,
                                    phi + static_cast<int64_t>(m) * phi_ld, s);
    }
    if (e != hipSuccess)
        return bltc_detail::hip_fail(e, "direct-sum launch");
    return BLTC_OK;
}
