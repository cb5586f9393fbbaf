// device_common.hpp -- FP64 device helpers shared by the kernel files:
// reciprocal square roots, the kernels G of eq. 2, and the direct
// batch/cluster sum of eq. 9 over a wave-uniform source range.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bltc {
namespace dev {

// ---------------------------------------------------------------------------
// FP64 reciprocal square root from the hardware estimate y0 = v_rsq_f64(r2)
// (relative error below 2^-22 on this device) and one Newton step in the form
//   2/sqrt(r2) ~ y0 (3 - r2 y0^2),
// three instructions (r2 y0, the fused 3 - (r2 y0) y0, the product with y0).
// The step's truncation error is -(3/8) e^2 relative with e = 1 - r2 y0^2, at
// most a few 1e-15 and of one sign; the interaction kernels accumulate the
// doubled values and halve each sum once.  rsqrt2_f64_or_zero returns +0 for
// r2 == 0: the estimate of 0 is +inf, whose low word is zero, so clearing its
// high word gives y0 = +0 and then 0 (pairs at zero distance contribute
// nothing, eq. 9).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double newton2(double r2, double y)
{
    const double u = r2 * y;
    return y * __fma_rn(-u, y, 3.0);
}

__device__ __forceinline__ double rsqrt2_f64(double r2)
{
    return newton2(r2, __builtin_amdgcn_rsq(r2));
}

__device__ __forceinline__ double rsqrt2_f64_or_zero(double r2)
{
    const double y = __builtin_amdgcn_rsq(r2);
    const int lo = __double2loint(y);
    const int hi = r2 > 0.0 ? __double2hiint(y) : 0;
    return newton2(r2, __hiloint2double(hi, lo));
}

__device__ __forceinline__ double rsqrt_f64_newton(double r2)
{
    return 0.5 * rsqrt2_f64(r2);
}

// ---------------------------------------------------------------------------
// exp(x) for x <= 0 in FP64 (x = -kappa r in the Yukawa kernel), from
// exp(x) = 2^(n/64) e^u with n = rint(64 x / ln 2) and u = x - n ln2/64
// (Cody-Waite: ln2/64 split into a 32-bit head, so n * head is exact for
// |n| < 2^21, and a tail), |u| <= ln2/128; e^u by its Taylor polynomial of
// degree 5 (remainder below 4e-17); 2^(j/64) from a 64-entry table that each
// workgroup fills in LDS with exp2 (fill_exp2_table).
// ---------------------------------------------------------------------------
constexpr double kLn2Over64Hi = 0x1.62e42fee00000p-7;
constexpr double kLn2Over64Lo = 0x1.a39ef35793c76p-39;
constexpr double k64OverLn2 = 92.33248261689366;

struct KernelArg {
    double kappa;        // Yukawa
    double delta2;       // regularized Coulomb: delta^2
    const double* tab;   // 2^(j/64), j < 64 (LDS; Yukawa)
};

__device__ __forceinline__ void fill_exp2_table(double* tab)
{
    if (threadIdx.x < 64)
        tab[threadIdx.x] = exp2(static_cast<double>(threadIdx.x) / 64.0);
    __syncthreads();
}

__device__ __forceinline__ double exp_f64(double x, const double* __restrict__ tab)
{
    const double nd = __builtin_rint(x * k64OverLn2);
    const int n = static_cast<int>(nd);
    double u = __fma_rn(-nd, kLn2Over64Hi, x);
    u = __fma_rn(-nd, kLn2Over64Lo, u);
    double p = __fma_rn(u, 1.0 / 120.0, 1.0 / 24.0);
    p = __fma_rn(u, p, 1.0 / 6.0);
    p = __fma_rn(u, p, 0.5);
    p = __fma_rn(u, p, 1.0);
    p = __fma_rn(u, p, 1.0);
    return ldexp(tab[n & 63] * p, n >> 6);
}

// G as a function of r^2 (eq. 2; KER 0 Coulomb 1/r, 1 Yukawa exp(-kappa r)/r,
// 2 regularized Coulomb (r^2 + delta^2)^(-1/2)), doubled: green_far2_f64 for
// well-separated points (r > 0), green_near2_f64 for any pair, zero at r = 0
// (pairs at zero distance are skipped).  With h = 2/r from rsqrt2, Yukawa's
// exponent -kappa r is -(kappa / 2) r^2 h.  green_far_f64 / green_near_f64 are
// the plain values.
template <int KER>
__device__ __forceinline__ double green_far2_f64(double r2, const KernelArg& ka)
{
    if constexpr (KER == 0) {
        return rsqrt2_f64(r2);
    } else if constexpr (KER == 1) {
        const double h = rsqrt2_f64(r2);
        return exp_f64(-0.5 * ka.kappa * (r2 * h), ka.tab) * h;
    } else {
        return rsqrt2_f64(r2 + ka.delta2);
    }
}

template <int KER>
__device__ __forceinline__ double green_near2_f64(double r2, const KernelArg& ka)
{
    if constexpr (KER == 0) {
        return rsqrt2_f64_or_zero(r2);
    } else if constexpr (KER == 1) {
        const double h = rsqrt2_f64_or_zero(r2);
        return exp_f64(-0.5 * ka.kappa * (r2 * h), ka.tab) * h;
    } else {
        const double g = rsqrt2_f64(r2 + ka.delta2);
        return r2 == 0.0 ? 0.0 : g;
    }
}

template <int KER>
__device__ __forceinline__ double green_far_f64(double r2, const KernelArg& ka)
{
    return 0.5 * green_far2_f64<KER>(r2, ka);
}

template <int KER>
__device__ __forceinline__ double green_near_f64(double r2, const KernelArg& ka)
{
    return 0.5 * green_near2_f64<KER>(r2, ka);
}

// FP32 kernel values (FP32-mixed path): nk = -kappa log2(e); r^2 > 0 (pairs at
// zero distance take the FP64 branch of the mixed near field).
struct KernelArg32 {
    float nk;
    float delta2;
};

__device__ __forceinline__ KernelArg32 kernel_arg32(double kappa, double delta2)
{
    return KernelArg32{static_cast<float>(-kappa * 1.4426950408889634), static_cast<float>(delta2)};
}

template <int KER>
__device__ __forceinline__ float green_f32(float r2, const KernelArg32& ka)
{
    if constexpr (KER == 0) {
        return __builtin_amdgcn_rsqf(r2);
    } else if constexpr (KER == 1) {
        const float rinv = __builtin_amdgcn_rsqf(r2);
        return __builtin_amdgcn_exp2f(ka.nk * (r2 * rinv)) * rinv;
    } else {
        return __builtin_amdgcn_rsqf(r2 + ka.delta2);
    }
}

// ---------------------------------------------------------------------------
// Direct batch/cluster sum over a contiguous source range (eq. 9), pairs at
// zero distance skipped.  `s` is wave-uniform.  The four partial sums hold
// doubled terms and are halved once.
// ---------------------------------------------------------------------------
template <int KER>
__device__ __forceinline__ double near_term2_f64(double x, double y, double z, const double4 p,
                                                 const KernelArg& kappa)
{
    const double dx = x - p.x;
    const double dy = y - p.y;
    const double dz = z - p.z;
    const double r2 = __fma_rn(dz, dz, __fma_rn(dy, dy, dx * dx));
    return green_near2_f64<KER>(r2, kappa) * p.w;
}

template <int KER>
__device__ __forceinline__ double near_term_f64(double x, double y, double z, const double4 p,
                                                const KernelArg& kappa)
{
    return 0.5 * near_term2_f64<KER>(x, y, z, p, kappa);
}

template <int KER>
__device__ __forceinline__ double near_sum_f64(double x, double y, double z,
                                               const double4* __restrict__ s, int32_t cnt,
                                               const KernelArg& kappa)
{
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int32_t j = 0;
    for (; j + 4 <= cnt; j += 4) {
        a0 += near_term2_f64<KER>(x, y, z, s[j], kappa);
        a1 += near_term2_f64<KER>(x, y, z, s[j + 1], kappa);
        a2 += near_term2_f64<KER>(x, y, z, s[j + 2], kappa);
        a3 += near_term2_f64<KER>(x, y, z, s[j + 3], kappa);
    }
    for (; j < cnt; ++j)
        a0 += near_term2_f64<KER>(x, y, z, s[j], kappa);
    return 0.5 * ((a0 + a1) + (a2 + a3));
}

}  // namespace dev
}  // namespace bltc
