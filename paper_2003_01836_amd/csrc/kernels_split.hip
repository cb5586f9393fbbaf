// kernels_split.hip -- partial potentials of plans with several lanes per
// target: each lane of a target summed a contiguous piece of its batch's
// interaction lists into its own row; this adds the rows per target in piece
// order (deterministic), one target per thread (HBM-bound, coalesced).
// replicate_targets writes the T copies of the targets such a plan walks.
#include "kernels_split.hpp"

namespace bltc {
namespace {

__global__ __launch_bounds__(256) void sum_parts(const double* __restrict__ buf, int64_t n,
                                                 int32_t parts, double* __restrict__ phi)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    double v = buf[i];
    for (int32_t p = 1; p < parts; ++p)
        v += buf[p * n + i];
    phi[i] = v;
}

// copy p of target i: tgt_t[p n + i] = tgt[i], orig_t[p n + i] = p n + orig[i]
__global__ __launch_bounds__(256) void replicate_targets(double4* __restrict__ tgt_t,
                                                         int64_t* __restrict__ orig_t,
                                                         const double4* __restrict__ tgt,
                                                         const int64_t* __restrict__ orig,
                                                         int64_t n, int64_t total)
{
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= total)
        return;
    const int64_t p = k / n, i = k - p * n;
    tgt_t[k] = tgt[i];
    orig_t[k] = p * n + orig[i];
}

}  // namespace

hipError_t launch_replicate_targets(double4* tgt_t, int64_t* orig_t, const double4* tgt,
                                    const int64_t* orig, int64_t n, int32_t parts, hipStream_t s)
{
    const int64_t total = n * parts;
    if (total == 0)
        return hipSuccess;
    if (!tgt_t || !orig_t || !tgt || !orig || parts < 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(replicate_targets, dim3(static_cast<unsigned>((total + 255) / 256)),
                       dim3(256), 0, s, tgt_t, orig_t, tgt, orig, n, total);
    return hipGetLastError();
}

hipError_t launch_sum_parts(const double* buf, int64_t n, int32_t parts, double* phi,
                            hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(sum_parts, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s,
                       buf, n, parts, phi);
    return hipGetLastError();
}

}  // namespace bltc
