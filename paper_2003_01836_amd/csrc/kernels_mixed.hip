// kernels_mixed.hip -- FP32-mixed batch/cluster interactions (eqs. 9 and 11).
//
// Same mapping as the FP64 kernel (one target per lane, wave-uniform lists and
// sources through the scalar cache), with the kernel evaluations in FP32:
//  * direct sums (eq. 9): local coordinates and an FP64 branch for close
//    pairs (device_mixed.hpp);
//  * approximations (eq. 11) use FP32 squared 1-D distances (formed in FP64,
//    rounded once per target and pair) and FP32 modified charges;
//  * FP32 partial sums cover at most kMixedFlush sources or (n+1)^2 proxy
//    points before they are added to the lane's FP64 accumulator.
#include "device_common.hpp"
#include "device_mixed.hpp"
#include "kernels.hpp"

namespace bltc {
namespace {

using namespace dev;

template <int N, int KER>
__device__ __forceinline__ double far_sum_mixed(double xt, double yt, double zt,
                                                const double* __restrict__ nd,
                                                const float* __restrict__ qh,
                                                const KernelArg32& nk)
{
    constexpr int NP = N + 1;
    float b2[NP], c2[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const float dy = static_cast<float>(yt - nd[NP + k]);
        const float dz = static_cast<float>(zt - nd[2 * NP + k]);
        b2[k] = dy * dy;
        c2[k] = dz * dz;
    }
    double acc = 0.0;
#pragma unroll 1
    for (int k1 = 0; k1 < NP; ++k1) {
        const float dx = static_cast<float>(xt - nd[k1]);
        const float a2 = dx * dx;
        const float* __restrict__ q1 = qh + k1 * NP * NP;
        float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
        for (int k2 = 0; k2 < NP; ++k2) {
            const float ab = a2 + b2[k2];
#pragma unroll
            for (int k3 = 0; k3 < NP; ++k3) {
                const float r2 = ab + c2[k3];
                const float g = green_f32<KER>(r2, nk);
                if ((k2 + k3) & 1)
                    s1 = __fmaf_rn(g, q1[k2 * NP + k3], s1);
                else
                    s0 = __fmaf_rn(g, q1[k2 * NP + k3], s0);
            }
        }
        acc += static_cast<double>(s0 + s1);
    }
    return acc;
}

// LDS staging of a cluster's modified charges up to n = 10 (5.3 KB per
// one-wave workgroup, about 30 workgroups per CU); above, the LDS would cut
// the occupancy and the charges come through the scalar cache
template <int N>
constexpr bool kStageCharges = N <= 10;

// eight waves per SIMD: the register allocation fits without spills and the
// far-field loop's scalar loads are better hidden than at the six waves the
// default allocation allows
template <int N, int KER>
__global__ __launch_bounds__(kGroupSize) __attribute__((amdgpu_waves_per_eu(8, 8))) void interact_mixed(
    const double4* __restrict__ tgt, const int64_t* __restrict__ tgt_orig,
    const double4* __restrict__ src, const float4* __restrict__ src32,
    const double4* __restrict__ node_info, const double4* __restrict__ batch_info,
    const int32_t* __restrict__ group_batch, const int64_t* __restrict__ group_first,
    const int64_t* __restrict__ batch_end, const int32_t* __restrict__ far_off,
    const int32_t* __restrict__ far_slot, const int32_t* __restrict__ near_off,
    const int64_t* __restrict__ near_begin, const int64_t* __restrict__ near_count,
    const int32_t* __restrict__ near_leaf, const double* __restrict__ slot_nodes,
    const float* __restrict__ qhat32,
    const int32_t* __restrict__ pc_off, const int64_t* __restrict__ pc_base,
    const double* __restrict__ pair_out, const int64_t* __restrict__ batch_begin,
    double* __restrict__ phi, KernelConst kc)
{
    constexpr int NP = N + 1;
    constexpr int P = NP * NP * NP;
    __shared__ double exp_tab[64];
    if constexpr (KER == 1)
        fill_exp2_table(exp_tab);
    const KernelArg kappa{kc.kappa, kc.delta2, exp_tab};
    const int g = blockIdx.x;
    const int b = group_batch[g];
    if (b < 0)
        return;  // empty slot of the per-die schedule
    const int64_t first = group_first[g];
    const int64_t end = batch_end[b];
    // (one-vector plans launch one wave per workgroup, so every wave of a
    // workgroup reaches the barriers of the far-field loop below; a wave
    // past the batch end evaluates its clamped targets and stores nothing)
    int64_t i = first + threadIdx.x;
    const bool valid = i < end;
    if (!valid)
        i = end - 1;
    const double4 t = tgt[i];
    const KernelArg32 nk = kernel_arg32(kc.kappa, kc.delta2);
    double acc = 0.0;

    const int f_end = far_off[b + 1];
    if constexpr (kStageCharges<N>) {
        // the cluster's modified charges staged in LDS (coalesced loads, one
        // copy per workgroup, read back as broadcasts): 5% faster at n = 8
        // than the wave-uniform scalar loads, whose latency the waves of a
        // SIMD did not hide
        extern __shared__ float qs[];
        for (int f = far_off[b]; f < f_end; ++f) {
            const int64_t slot = far_slot[f];
            const float* __restrict__ qg = qhat32 + slot * P;
            __syncthreads();   // the previous cluster's charges are read
            for (int k = threadIdx.x; k < P; k += blockDim.x)
                qs[k] = qg[k];
            __syncthreads();
            acc += far_sum_mixed<N, KER>(t.x, t.y, t.z, slot_nodes + slot * 3 * NP, qs, nk);
        }
    } else {
        for (int f = far_off[b]; f < f_end; ++f) {
            const int64_t slot = far_slot[f];
            acc += far_sum_mixed<N, KER>(t.x, t.y, t.z, slot_nodes + slot * 3 * NP,
                                         qhat32 + slot * P, nk);
        }
    }
    const double4 bi = batch_info[b];
    const int n_end = near_off[b + 1];
    for (int e = near_off[b]; e < n_end; ++e) {
        const double4 li = node_info[near_leaf[e]];
        const double dx = bi.x - li.x, dy = bi.y - li.y, dz = bi.z - li.z;
        const double dist = sqrt(dx * dx + dy * dy + dz * dz);
        const double extent = dist + bi.w + 2.0 * li.w;
        const double tau = kMixedTauRel * extent;
        const float tau2 = static_cast<float>(tau * tau);
        const int64_t nb = near_begin[e];
        const int32_t nc = static_cast<int32_t>(near_count[e]);
        // bounding spheres further apart than tau: no pair needs the FP64 branch
        if (dist - bi.w - li.w > 1.0625 * tau)
            acc += near_sum_mixed<KER, false>(t.x, t.y, t.z, src32 + nb, src + nb, nc, li, tau2,
                                              nk, kappa);
        else
            acc += near_sum_mixed<KER, true>(t.x, t.y, t.z, src32 + nb, src + nb, nc, li, tau2,
                                             nk, kappa);
    }
    if (pc_off) {
        // mutual leaf pairs: this target's row or column sums of each unit
        const int64_t pos = i - batch_begin[b];
        const int pc_end = pc_off[b + 1];
        for (int e = pc_off[b]; e < pc_end; ++e)
            acc += pair_out[pc_base[e] + pos];
    }
    if (valid)
        phi[tgt_orig[i]] = acc;
}

template <int N, int KER>
hipError_t run_interact_mixed(const DevicePlan& d, double* phi, KernelConst kc, hipStream_t s)
{
    if (d.ngroups == 0)
        return hipSuccess;
    const NearLists nl = near_lists(d);
    const size_t lds = kStageCharges<N> ? sizeof(float) * (N + 1) * (N + 1) * (N + 1) : 0;
    hipLaunchKernelGGL((interact_mixed<N, KER>), dim3(static_cast<unsigned>(d.ngroups)),
                       dim3(d.group_threads), lds, s, d.tgt, d.tgt_orig, d.src, d.src32, d.node_info,
                       d.batch_info, d.group_batch, d.group_first, d.batch_end, d.far_off,
                       d.far_slot, nl.off, nl.begin, nl.count, nl.leaf, d.slot_nodes, d.qhat32,
                       nl.pc_off, nl.pc_base, nl.pair_out, nl.batch_begin, phi, kc);
    return hipGetLastError();
}

#define BLTC_DEGREE_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

}  // namespace

hipError_t launch_interact_mixed(const DevicePlan& d, const KernelParams& kp, double* phi,
                                 hipStream_t s)
{
    if (!d.src32 || !d.node_info || !d.batch_info || !d.qhat32)
        return hipErrorInvalidValue;
    const KernelConst kc = kp.kconst();
    switch (d.degree) {
#define X(n)                                                                   \
    case n:                                                                    \
        return kp.kernel == 1 ? run_interact_mixed<n, 1>(d, phi, kc, s)        \
             : kp.kernel == 2 ? run_interact_mixed<n, 2>(d, phi, kc, s)        \
                              : run_interact_mixed<n, 0>(d, phi, kc, s);
        BLTC_DEGREE_CASES(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace bltc
