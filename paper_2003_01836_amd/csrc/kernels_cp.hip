// kernels_cp.hip -- cluster-particle treecode: interpolation of the proxy
// potentials down to the targets.
//
// Proxy potentials (the sources of a batch summed at a target cluster's
// Chebyshev points) and direct sums reuse the interaction kernels: proxy
// points are just targets whose "batch" is their cluster.  What is new is the
// last step: every target receives, for each cluster on its root-to-leaf path
// that has proxy potentials, the barycentric interpolant (eq. 4, tensor
// product over x, y, z) of those potentials at its position:
//   phi(x) += sum_k L_k1(x1) L_k2(x2) L_k3(x3) phihat_k
//           = (sum_k a_1k1 a_2k2 a_3k3 phihat_k) / (D_1 D_2 D_3),
// with a_lk = w_k / (x_l - t_lk) and D_l = sum_k a_lk, or a one-hot row and
// D_l = 1 when x_l is within DBL_MIN of a node (eq. 5; the lowest such k).
// One target per lane, 256 targets of one target leaf per workgroup; the
// cluster grids and proxy potentials are wave-uniform (scalar loads).
#include <cfloat>

#include "kernels_cp.hpp"

namespace bltc {
namespace {

template <int NP>
__device__ __forceinline__ double interp_factors(double x, const double* __restrict__ t,
                                                 double (&a)[NP])
{
    int hit = -1;
#pragma unroll
    for (int k = NP - 1; k >= 0; --k)
        if (fabs(x - t[k]) < DBL_MIN)
            hit = k;
    if (hit >= 0) {
#pragma unroll
        for (int k = 0; k < NP; ++k)
            a[k] = k == hit ? 1.0 : 0.0;
        return 1.0;
    }
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const double w = ((k & 1) ? -1.0 : 1.0) * ((k == 0 || k == NP - 1) ? 0.5 : 1.0);
        a[k] = w / (x - t[k]);
        sum += a[k];
    }
    return sum;
}

template <int N>
__global__ __launch_bounds__(kGroupSize) void interpolate_targets(
    const double4* __restrict__ tgt, const int64_t* __restrict__ tgt_orig,
    const int32_t* __restrict__ group_batch, const int64_t* __restrict__ group_first,
    const int64_t* __restrict__ batch_end, const int32_t* __restrict__ path_off,
    const int32_t* __restrict__ path_slot, const double* __restrict__ slot_nodes,
    const double* __restrict__ phat, double* __restrict__ phi)
{
    constexpr int NP = N + 1;
    constexpr int P = NP * NP * NP;
    const int g = blockIdx.x;
    const int b = group_batch[g];
    if (b < 0)
        return;
    const int64_t first = group_first[g];
    const int64_t end = batch_end[b];
    if (first + (threadIdx.x & ~63) >= end)
        return;
    int64_t i = first + threadIdx.x;
    const bool valid = i < end;
    if (!valid)
        i = end - 1;
    const double4 t = tgt[i];
    double acc = 0.0;
    const int e_end = path_off[b + 1];
    for (int e = path_off[b]; e < e_end; ++e) {
        const int64_t sl = path_slot[e];
        const double* __restrict__ nd = slot_nodes + sl * 3 * NP;
        const double* __restrict__ ph = phat + sl * P;
        double a1[NP], a2[NP], a3[NP];
        const double D = interp_factors<NP>(t.x, nd, a1) * interp_factors<NP>(t.y, nd + NP, a2) *
                         interp_factors<NP>(t.z, nd + 2 * NP, a3);
        double s = 0.0;
#pragma unroll 1
        for (int k1 = 0; k1 < NP; ++k1) {
            double s1 = 0.0;
#pragma unroll
            for (int k2 = 0; k2 < NP; ++k2) {
                double s2 = 0.0;
#pragma unroll
                for (int k3 = 0; k3 < NP; ++k3)
                    s2 = __fma_rn(a3[k3], ph[(k1 * NP + k2) * NP + k3], s2);
                s1 = __fma_rn(a2[k2], s2, s1);
            }
            s = __fma_rn(a1[k1], s1, s);
        }
        acc += s / D;
    }
    if (valid)
        phi[tgt_orig[i]] += acc;
}

#define BLTC_DEGREE_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

}  // namespace

hipError_t launch_interpolate_targets(const DevicePlan& d, const int32_t* path_off,
                                      const int32_t* path_slot, const double* slot_nodes,
                                      const double* phat, double* phi, hipStream_t s)
{
    if (d.ngroups == 0)
        return hipSuccess;
    const dim3 grid(static_cast<unsigned>(d.ngroups));
    switch (d.degree) {
#define X(n)                                                                                  \
    case n:                                                                                   \
        hipLaunchKernelGGL(interpolate_targets<n>, grid, dim3(d.group_threads), 0, s, d.tgt,  \
                           d.tgt_orig, d.group_batch, d.group_first, d.batch_end, path_off,   \
                           path_slot, slot_nodes, phat, phi);                                 \
        return hipGetLastError();
        BLTC_DEGREE_CASES(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace bltc
