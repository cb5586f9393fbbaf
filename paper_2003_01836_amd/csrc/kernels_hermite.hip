// kernels_hermite.hip -- batch/cluster interactions of the barycentric Hermite
// treecode (the Hermite variant that the paper's outlook, Sec. V, names).
//
// A cluster's grid point s_k carries eight modified charges Q_a, one per
// derivative multi-index a = (a1, a2, a3) in {0,1}^3 of the tensor-product
// Hermite interpolant in the source variable, and the approximation of a
// batch/cluster pair is sum_k sum_a d^a_y G(x, s_k) Q_a(k).  For a radial
// kernel with d = x - s_k, g1 = G'(r)/r, g2 = g1'(r)/r, g3 = g2'(r)/r:
//     d_yi G = -d_i g1,  d_yi d_yj G = d_i d_j g2 (i != j),
//     d_y1 d_y2 d_y3 G = -d_1 d_2 d_3 g3,
// so one grid point costs one reciprocal square root (and for Yukawa one
// exponential), the recurrences for g1..g3 and eight products with its
// charges.  Mapping as in the BLTC interaction kernel: one target per lane,
// 256 targets of one batch per workgroup, wave-uniform lists, grid nodes and
// charges through the scalar cache (the eight charges of a grid point are
// contiguous: one 64-byte load), phi written once per target in caller order.
// An FP32-mixed form follows the FP64 kernel.
#include "kernels.hpp"
#include "device_common.hpp"
#include "device_mixed.hpp"

namespace bltc {
namespace {

using namespace dev;

// G, g1, g2, g3 at r^2 > 0 (well-separated points; 1/sqrt by one Newton step)
template <int KER>
__device__ __forceinline__ void green_derivatives(double r2, const KernelArg& ka, double& g0,
                                                  double& g1, double& g2, double& g3)
{
    if constexpr (KER == 1) {
        // G = e/r, e = exp(-kappa r): g1 = -G (1 + kr)/r^2,
        // g2 = G (3 + 3 kr + (kr)^2)/r^4, g3 = -G (15 + 15 kr + 6 (kr)^2 + (kr)^3)/r^6
        const double ri = rsqrt_f64_newton(r2);
        const double ri2 = ri * ri;
        const double kr = ka.kappa * (r2 * ri);
        g0 = exp_f64(-kr, ka.tab) * ri;
        const double kr2 = kr * kr;
        const double h1 = g0 * ri2;
        const double h2 = h1 * ri2;
        g1 = -h1 * (1.0 + kr);
        g2 = h2 * __fma_rn(3.0, kr, 3.0 + kr2);
        g3 = -(h2 * ri2) * __fma_rn(kr2, kr + 6.0, __fma_rn(15.0, kr, 15.0));
    } else {
        // Coulomb (u = r^2) and regularized Coulomb (u = r^2 + delta^2):
        // G = u^(-1/2), g1 = -u^(-3/2), g2 = 3 u^(-5/2), g3 = -15 u^(-7/2)
        const double ri = rsqrt_f64_newton(KER == 2 ? r2 + ka.delta2 : r2);
        const double ri2 = ri * ri;
        g0 = ri;
        g1 = -ri * ri2;
        g2 = -3.0 * g1 * ri2;
        g3 = -5.0 * g2 * ri2;
    }
}

// sum over the (n+1)^3 grid of one cluster; nd = [3][n+1] nodes, qh = [(n+1)^3][8]
template <int N, int KER>
__device__ __forceinline__ double far_sum_hermite(double x, double y, double z,
                                                  const double* __restrict__ nd,
                                                  const double* __restrict__ qh,
                                                  const KernelArg& ka)
{
    constexpr int NP = N + 1;
    double e2[NP], e3[NP], b2[NP], c2[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        e2[k] = y - nd[NP + k];
        e3[k] = z - nd[2 * NP + k];
        b2[k] = e2[k] * e2[k];
        c2[k] = e3[k] * e3[k];
    }
    double acc0 = 0.0, acc1 = 0.0;
#pragma unroll 1
    for (int k1 = 0; k1 < NP; ++k1) {
        const double d1 = x - nd[k1];
        const double a2 = d1 * d1;
        const double* __restrict__ q1 = qh + k1 * NP * NP * 8;
#pragma unroll
        for (int k2 = 0; k2 < NP; ++k2) {
            const double d2 = e2[k2];
            const double ab = a2 + b2[k2];
            const double d12 = d1 * d2;
#pragma unroll
            for (int k3 = 0; k3 < NP; ++k3) {
                const double d3 = e3[k3];
                double g0, g1, g2, g3;
                green_derivatives<KER>(ab + c2[k3], ka, g0, g1, g2, g3);
                const double* __restrict__ Q = q1 + (k2 * NP + k3) * 8;
                // a = 4 a1 + 2 a2 + a3
                const double s1 = __fma_rn(d1, Q[4], __fma_rn(d2, Q[2], d3 * Q[1]));
                const double s2 = __fma_rn(d12, Q[6], d3 * __fma_rn(d1, Q[5], d2 * Q[3]));
                const double s3 = d12 * d3 * Q[7];
                double t = g0 * Q[0];
                t = __fma_rn(-g1, s1, t);
                t = __fma_rn(g2, s2, t);
                t = __fma_rn(-g3, s3, t);
                if ((k2 + k3) & 1)
                    acc1 += t;
                else
                    acc0 += t;
            }
        }
    }
    return acc0 + acc1;
}

template <int N, int KER>
__global__ __launch_bounds__(kGroupSize) void interact_hermite_f64(
    const double4* __restrict__ tgt, const int64_t* __restrict__ tgt_orig,
    const double4* __restrict__ src, const int32_t* __restrict__ group_batch,
    const int64_t* __restrict__ group_first, const int64_t* __restrict__ batch_end,
    const int32_t* __restrict__ far_off, const int32_t* __restrict__ far_slot,
    const int32_t* __restrict__ near_off, const int64_t* __restrict__ near_begin,
    const int64_t* __restrict__ near_count, const double* __restrict__ slot_nodes,
    const double* __restrict__ qh,
    const int32_t* __restrict__ pc_off, const int64_t* __restrict__ pc_base,
    const double* __restrict__ pair_out, const int64_t* __restrict__ batch_begin,
    double* __restrict__ phi, KernelConst kc)
{
    constexpr int NP = N + 1;
    constexpr int P8 = 8 * NP * NP * NP;
    __shared__ double exp_tab[64];
    if constexpr (KER == 1)
        fill_exp2_table(exp_tab);
    const KernelArg ka{kc.kappa, kc.delta2, exp_tab};
    const int g = blockIdx.x;
    const int b = group_batch[g];
    if (b < 0)
        return;  // empty slot of the per-die schedule
    const int64_t first = group_first[g];
    const int64_t end = batch_end[b];
    if (first + (threadIdx.x & ~63) >= end)
        return;  // the whole wave lies past the batch end
    int64_t i = first + threadIdx.x;
    const bool valid = i < end;
    if (!valid)
        i = end - 1;
    const double4 t = tgt[i];
    double acc = 0.0;
    const int f_end = far_off[b + 1];
    for (int f = far_off[b]; f < f_end; ++f) {
        const int64_t slot = far_slot[f];
        acc += far_sum_hermite<N, KER>(t.x, t.y, t.z, slot_nodes + slot * 3 * NP, qh + slot * P8,
                                       ka);
    }
    const int n_end = near_off[b + 1];
    for (int e = near_off[b]; e < n_end; ++e)
        acc += near_sum_f64<KER>(t.x, t.y, t.z, src + near_begin[e],
                                 static_cast<int32_t>(near_count[e]), ka);
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

// ---------------------------------------------------------------------------
// FP32-mixed form.  With u = r^2 (u = r^2 + delta^2 for the regularized
// kernel), ri = u^(-1/2) and the direction cosines f = d ri (|f_i| <= 1),
// the term of one grid point is
//     G [ Q_0 + ri (p1 S1 + ri (p2 S2 + ri p3 S3)) ]
// with S1 = f1 Q_4 + f2 Q_2 + f3 Q_1, S2 = f1 f2 Q_6 + f3 (f1 Q_5 + f2 Q_3),
// S3 = f1 f2 f3 Q_7 and p1, p2, p3 = 1, 3, 15 (Coulomb forms) or
// 1 + kr, 3 + 3 kr + (kr)^2, 15 + 15 kr + 6 (kr)^2 + (kr)^3 (Yukawa, k = kappa):
// the same sum as above, ordered so that no intermediate grows like a power
// of 1/r beyond the first (FP32 range).  Squared 1-D distances are formed in
// FP64 and rounded once per target and cluster; FP32 partial sums cover
// (n+1)^2 grid points; direct sums as in the FP32-mixed BLTC.
// ---------------------------------------------------------------------------
// one grid point: r2 = |d|^2, d = x - s_k in FP32, Q its eight charges
template <int KER>
__device__ __forceinline__ float hermite_term_f32(float r2, float d1, float d2, float d3,
                                                  const float* __restrict__ Q,
                                                  const KernelArg32& nk, float kf)
{
    const float u = KER == 2 ? r2 + nk.delta2 : r2;
    const float ri = __builtin_amdgcn_rsqf(u);
    const float e1 = d1 * ri, e2 = d2 * ri, e3 = d3 * ri;   // direction cosines f
    const float S1 = __fmaf_rn(e1, Q[4], __fmaf_rn(e2, Q[2], e3 * Q[1]));
    const float e12 = e1 * e2;
    const float S2 = __fmaf_rn(e12, Q[6], e3 * __fmaf_rn(e1, Q[5], e2 * Q[3]));
    const float S3 = e12 * e3 * Q[7];
    if constexpr (KER == 1) {
        const float r = u * ri;
        const float kr = kf * r;
        const float g = __builtin_amdgcn_exp2f(nk.nk * r) * ri;
        const float p1 = 1.0f + kr;
        const float p2 = __fmaf_rn(kr, kr + 3.0f, 3.0f);
        const float p3 = __fmaf_rn(kr, __fmaf_rn(kr, kr + 6.0f, 15.0f), 15.0f);
        const float h = __fmaf_rn(ri, __fmaf_rn(p2, S2, ri * (p3 * S3)), p1 * S1);
        return g * __fmaf_rn(ri, h, Q[0]);
    } else {
        const float h = __fmaf_rn(ri, __fmaf_rn(3.0f, S2, ri * (15.0f * S3)), S1);
        return ri * __fmaf_rn(ri, h, Q[0]);
    }
}

// sum over the (n+1)^3 grid of one cluster in FP32-mixed; qh = [(n+1)^3][8] FP32
template <int N, int KER>
__device__ __forceinline__ double far_sum_hermite_f32(double x, double y, double z,
                                                      const double* __restrict__ nd,
                                                      const float* __restrict__ qh,
                                                      const KernelArg32& nk, float kf)
{
    constexpr int NP = N + 1;
    float e2[NP], e3[NP], b2[NP], c2[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        e2[k] = static_cast<float>(y - nd[NP + k]);
        e3[k] = static_cast<float>(z - nd[2 * NP + k]);
        b2[k] = e2[k] * e2[k];
        c2[k] = e3[k] * e3[k];
    }
    double acc = 0.0;
#pragma unroll 1
    for (int k1 = 0; k1 < NP; ++k1) {
        const float d1 = static_cast<float>(x - nd[k1]);
        const float a2 = d1 * d1;
        const float* __restrict__ q1 = qh + k1 * NP * NP * 8;
        float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
        for (int k2 = 0; k2 < NP; ++k2) {
            const float ab = a2 + b2[k2];
#pragma unroll
            for (int k3 = 0; k3 < NP; ++k3) {
                const float t = hermite_term_f32<KER>(ab + c2[k3], d1, e2[k2], e3[k3],
                                                      q1 + (k2 * NP + k3) * 8, nk, kf);
                if ((k2 + k3) & 1)
                    s1 += t;
                else
                    s0 += t;
            }
        }
        acc += static_cast<double>(s0 + s1);
    }
    return acc;
}

// LDS staging of the FP32 modified charges at n = 4 (1000 values, 4 KB per
// one-wave workgroup): 4% faster there; at n = 2 and 3 the two barriers per
// cluster cost more than the scalar loads save, and at n = 6 the LDS size
// costs occupancy, so the other degrees read the charges through the scalar
// cache
template <int N>
constexpr bool kStageHermite = N == 4;

template <int N, int KER>
__global__ __launch_bounds__(kGroupSize) void interact_hermite_mixed(
    const double4* __restrict__ tgt, const int64_t* __restrict__ tgt_orig,
    const double4* __restrict__ src, const float4* __restrict__ src32,
    const double4* __restrict__ node_info, const double4* __restrict__ batch_info,
    const int32_t* __restrict__ group_batch, const int64_t* __restrict__ group_first,
    const int64_t* __restrict__ batch_end, const int32_t* __restrict__ far_off,
    const int32_t* __restrict__ far_slot, const int32_t* __restrict__ near_off,
    const int64_t* __restrict__ near_begin, const int64_t* __restrict__ near_count,
    const int32_t* __restrict__ near_leaf, const double* __restrict__ slot_nodes,
    const float* __restrict__ qh32,
    const int32_t* __restrict__ pc_off, const int64_t* __restrict__ pc_base,
    const double* __restrict__ pair_out, const int64_t* __restrict__ batch_begin,
    double* __restrict__ phi, KernelConst kc)
{
    constexpr int NP = N + 1;
    constexpr int P8 = 8 * NP * NP * NP;
    __shared__ double exp_tab[64];
    if constexpr (KER == 1)
        fill_exp2_table(exp_tab);
    const KernelArg ka{kc.kappa, kc.delta2, exp_tab};
    const KernelArg32 nk = kernel_arg32(kc.kappa, kc.delta2);
    const float kf = static_cast<float>(kc.kappa);
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
    double acc = 0.0;
    const int f_end = far_off[b + 1];
    if constexpr (kStageHermite<N>) {
        // the cluster's 8 (n+1)^3 modified charges staged in LDS, as in the
        // FP32-mixed BLTC kernel
        extern __shared__ float qs[];
        for (int f = far_off[b]; f < f_end; ++f) {
            const int64_t slot = far_slot[f];
            const float* __restrict__ qg = qh32 + slot * P8;
            __syncthreads();   // the previous cluster's charges are read
            for (int k = threadIdx.x; k < P8; k += blockDim.x)
                qs[k] = qg[k];
            __syncthreads();
            acc += far_sum_hermite_f32<N, KER>(t.x, t.y, t.z, slot_nodes + slot * 3 * NP, qs,
                                               nk, kf);
        }
    } else {
        for (int f = far_off[b]; f < f_end; ++f) {
            const int64_t slot = far_slot[f];
            acc += far_sum_hermite_f32<N, KER>(t.x, t.y, t.z, slot_nodes + slot * 3 * NP,
                                               qh32 + slot * P8, nk, kf);
        }
    }
    const double4 bi = batch_info[b];
    const int n_end = near_off[b + 1];
    for (int e = near_off[b]; e < n_end; ++e) {
        const int64_t nb = near_begin[e];
        acc += near_entry_mixed<KER>(t.x, t.y, t.z, bi, node_info[near_leaf[e]], src32 + nb,
                                     src + nb, static_cast<int32_t>(near_count[e]), nk, ka);
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
hipError_t run_interact_hermite_mixed(const DevicePlan& d, double* phi, KernelConst kc,
                                      hipStream_t s)
{
    if (d.ngroups == 0)
        return hipSuccess;
    const NearLists nl = near_lists(d);
    const size_t lds = kStageHermite<N> ? sizeof(float) * 8 * (N + 1) * (N + 1) * (N + 1) : 0;
    hipLaunchKernelGGL((interact_hermite_mixed<N, KER>), dim3(static_cast<unsigned>(d.ngroups)),
                       dim3(d.group_threads), lds, s, d.tgt, d.tgt_orig, d.src, d.src32,
                       d.node_info, d.batch_info, d.group_batch, d.group_first, d.batch_end,
                       d.far_off, d.far_slot, nl.off, nl.begin, nl.count, nl.leaf, d.slot_nodes,
                       d.qhat32, nl.pc_off, nl.pc_base, nl.pair_out, nl.batch_begin, phi, kc);
    return hipGetLastError();
}

template <int N, int KER>
hipError_t run_interact_hermite(const DevicePlan& d, double* phi, KernelConst kc, hipStream_t s)
{
    if (d.ngroups == 0)
        return hipSuccess;
    const NearLists nl = near_lists(d);
    hipLaunchKernelGGL((interact_hermite_f64<N, KER>), dim3(static_cast<unsigned>(d.ngroups)),
                       dim3(d.group_threads), 0, s, d.tgt, d.tgt_orig, d.src, d.group_batch,
                       d.group_first, d.batch_end, d.far_off, d.far_slot, nl.off, nl.begin,
                       nl.count, d.slot_nodes, d.qhat_h, nl.pc_off, nl.pc_base, nl.pair_out,
                       nl.batch_begin, phi, kc);
    return hipGetLastError();
}

#define BLTC_HERMITE_DEGREE_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10)

}  // namespace

hipError_t launch_interact_hermite(const DevicePlan& d, const KernelParams& kp, double* phi,
                                   hipStream_t s)
{
    static_assert(kMaxHermiteDegree == 10, "degree cases below");
    if (!d.hermite || !d.qhat_h)
        return hipErrorInvalidValue;
    const KernelConst kc = kp.kconst();
    if (kp.precision == 1) {
        if (!d.src32 || !d.node_info || !d.batch_info || !d.qhat32)
            return hipErrorInvalidValue;
        switch (d.degree) {
#define X(n)                                                                         \
    case n:                                                                          \
        return kp.kernel == 1 ? run_interact_hermite_mixed<n, 1>(d, phi, kc, s)      \
             : kp.kernel == 2 ? run_interact_hermite_mixed<n, 2>(d, phi, kc, s)      \
                              : run_interact_hermite_mixed<n, 0>(d, phi, kc, s);
            BLTC_HERMITE_DEGREE_CASES(X)
#undef X
        default:
            return hipErrorInvalidValue;
        }
    }
    switch (d.degree) {
#define X(n)                                                                   \
    case n:                                                                    \
        return kp.kernel == 1 ? run_interact_hermite<n, 1>(d, phi, kc, s)      \
             : kp.kernel == 2 ? run_interact_hermite<n, 2>(d, phi, kc, s)      \
                              : run_interact_hermite<n, 0>(d, phi, kc, s);
        BLTC_HERMITE_DEGREE_CASES(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace bltc
