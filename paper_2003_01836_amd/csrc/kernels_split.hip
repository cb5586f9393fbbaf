// kernels_split.hip -- partial potentials of plans with several lanes per
// target: each lane of a target summed a contiguous piece of its batch's
// interaction lists into its own row; this adds the rows per target in piece
// order (deterministic), one target per thread (HBM-bound, coalesced).
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

}  // namespace

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
