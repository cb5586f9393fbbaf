// device_mixed.hpp -- the FP32-mixed direct sum (eq. 9) of a lane's target
// over a wave-uniform source range, shared by the FP32-mixed interaction
// kernels of the BLTC and of the Hermite treecode.
//
//  * Local coordinates: sources are stored relative to the center of their
//    leaf; each lane forms its target's offset from that center once per
//    batch/leaf pair, in FP64, and rounds it to FP32, so the FP32 differences
//    carry relative rounding errors of the local extent, not of the domain;
//  * pairs with r^2 <= tau^2, tau = kMixedTauRel * (local extent) -- this
//    includes pairs at zero distance even when the extent is zero (a
//    one-particle batch against its own one-particle leaf) -- take an FP64
//    branch (exact coordinates, FP64 kernel), so the coordinate rounding never
//    exceeds about 2^-24 / kMixedTauRel (a few 1e-6) of a term, and the
//    aggregate coordinate error, which is dominated by the closest pairs,
//    scales as kMixedTauRel^-1/2;
//  * FP32 partial sums cover at most kMixedFlush sources before they are
//    added to the FP64 result.
#pragma once

#include "device_common.hpp"
#include "kernels.hpp"

namespace bltc {
namespace dev {

constexpr int kMixedFlush = 128;

// FP32 kernel value of one source for a lane's local target coordinates.
template <int KER>
__device__ __forceinline__ float near_value_f32(float x, float y, float z, const float4 p,
                                                const KernelArg32& nk, float& r2)
{
    const float dx = x - p.x;
    const float dy = y - p.y;
    const float dz = z - p.z;
    r2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
    return green_f32<KER>(r2, nk);
}

// Sources [j, j+4): FP32 values; if any of them is closer than tau (rare, one
// branch per 4 sources), those terms are redone in FP64 into `acc` and their
// FP32 values are zeroed.
template <int KER, bool CHECK>
__device__ __forceinline__ void near_quad_mixed(float x, float y, float z,
                                                const float4* __restrict__ s32,
                                                const double4* __restrict__ s64, float tau2,
                                                const KernelArg32& nk, double xt, double yt,
                                                double zt,
                                                const KernelArg& kappa, double& acc, float& a0, float& a1,
                                                float& a2, float& a3)
{
    const float4 p0 = s32[0], p1 = s32[1], p2 = s32[2], p3 = s32[3];
    float r0, r1, r2, r3;
    float g0 = near_value_f32<KER>(x, y, z, p0, nk, r0);
    float g1 = near_value_f32<KER>(x, y, z, p1, nk, r1);
    float g2 = near_value_f32<KER>(x, y, z, p2, nk, r2);
    float g3 = near_value_f32<KER>(x, y, z, p3, nk, r3);
    if (CHECK && fminf(fminf(r0, r1), fminf(r2, r3)) <= tau2) {
        if (r0 <= tau2) { acc += near_term_f64<KER>(xt, yt, zt, s64[0], kappa); g0 = 0.0f; }
        if (r1 <= tau2) { acc += near_term_f64<KER>(xt, yt, zt, s64[1], kappa); g1 = 0.0f; }
        if (r2 <= tau2) { acc += near_term_f64<KER>(xt, yt, zt, s64[2], kappa); g2 = 0.0f; }
        if (r3 <= tau2) { acc += near_term_f64<KER>(xt, yt, zt, s64[3], kappa); g3 = 0.0f; }
    }
    a0 = __fmaf_rn(g0, p0.w, a0);
    a1 = __fmaf_rn(g1, p1.w, a1);
    a2 = __fmaf_rn(g2, p2.w, a2);
    a3 = __fmaf_rn(g3, p3.w, a3);
}

// CHECK = false: the caller has shown that no pair is closer than tau
template <int KER, bool CHECK>
__device__ __forceinline__ double near_sum_mixed(double xt, double yt, double zt,
                                                 const float4* __restrict__ s32,
                                                 const double4* __restrict__ s64, int32_t cnt,
                                                 const double4 leaf, float tau2,
                                                 const KernelArg32& nk,
                                                 const KernelArg& kappa)
{
    const float x = static_cast<float>(xt - leaf.x);
    const float y = static_cast<float>(yt - leaf.y);
    const float z = static_cast<float>(zt - leaf.z);
    double acc = 0.0;
    for (int32_t j0 = 0; j0 < cnt; j0 += kMixedFlush) {
        const int32_t j1 = (cnt - j0 < kMixedFlush) ? cnt : j0 + kMixedFlush;
        float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
        int32_t j = j0;
        for (; j + 4 <= j1; j += 4)
            near_quad_mixed<KER, CHECK>(x, y, z, s32 + j, s64 + j, tau2, nk, xt, yt, zt, kappa,
                                        acc, a0, a1, a2, a3);
        for (; j < j1; ++j) {
            float r;
            float g = near_value_f32<KER>(x, y, z, s32[j], nk, r);
            if (CHECK && r <= tau2) {
                acc += near_term_f64<KER>(xt, yt, zt, s64[j], kappa);
                g = 0.0f;
            }
            a0 = __fmaf_rn(g, s32[j].w, a0);
        }
        acc += static_cast<double>((a0 + a1) + (a2 + a3));
    }
    return acc;
}

// One direct list entry: batch b's target against the sources of leaf li
// (center and radius; bi: the batch's).  Bounding spheres further apart than
// tau: no pair needs the FP64 branch.
template <int KER>
__device__ __forceinline__ double near_entry_mixed(double xt, double yt, double zt,
                                                   const double4 bi, const double4 li,
                                                   const float4* __restrict__ s32,
                                                   const double4* __restrict__ s64, int32_t cnt,
                                                   const KernelArg32& nk,
                                                   const KernelArg& kappa)
{
    const double dx = bi.x - li.x, dy = bi.y - li.y, dz = bi.z - li.z;
    const double dist = sqrt(dx * dx + dy * dy + dz * dz);
    const double extent = dist + bi.w + 2.0 * li.w;
    const double tau = kMixedTauRel * extent;
    const float tau2 = static_cast<float>(tau * tau);
    if (dist - bi.w - li.w > 1.0625 * tau)
        return near_sum_mixed<KER, false>(xt, yt, zt, s32, s64, cnt, li, tau2, nk, kappa);
    return near_sum_mixed<KER, true>(xt, yt, zt, s32, s64, cnt, li, tau2, nk, kappa);
}

}  // namespace dev
}  // namespace bltc
