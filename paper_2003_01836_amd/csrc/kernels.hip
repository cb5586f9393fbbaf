// kernels.hip -- gfx950 kernels of the barycentric Lagrange treecode.
//
// Mapping (CDNA4, wave64):
//  * interactions: one target per lane, 256 targets of one batch per
//    workgroup; every lane of a wave walks the same interaction list (the MAC
//    is applied per batch, Sec. III-B), so source particles, Chebyshev points
//    and modified charges are wave-uniform and are read through the scalar
//    data cache into SGPRs -- no LDS staging and no barriers.  Each lane owns
//    its target's accumulator, so phi is written exactly once, in caller
//    order, without atomics.
//  * the upward pass lives in kernels_upward.hip (matrix cores).
#include "kernels.hpp"
#include "device_common.hpp"

namespace bltc {
namespace {

using namespace dev;

// ---------------------------------------------------------------------------
// Batch/cluster approximation (eq. 11): sum_k G(x, s_k) qhat_k over the
// (n+1)^3 tensor grid.  With the grid separable, r^2 = a_k1 + b_k2 + c_k3
// where a, b, c are the squared 1-D distances, formed once per target.
// `nd` ([3][n+1] points) and `qh` ([P] charges) are wave-uniform.
// ---------------------------------------------------------------------------
template <int N, int KER>
__device__ __forceinline__ double far_sum_f64(double x, double y, double z,
                                              const double* __restrict__ nd,
                                              const double* __restrict__ qh, const KernelArg& kappa)
{
    constexpr int NP = N + 1;
    double b2[NP], c2[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const double dy = y - nd[NP + k];
        const double dz = z - nd[2 * NP + k];
        b2[k] = dy * dy;
        c2[k] = dz * dz;
    }
    double acc0 = 0.0, acc1 = 0.0;
#pragma unroll 1
    for (int k1 = 0; k1 < NP; ++k1) {
        const double dx = x - nd[k1];
        const double a2 = dx * dx;
        const double* __restrict__ q1 = qh + k1 * NP * NP;
#pragma unroll
        for (int k2 = 0; k2 < NP; ++k2) {
            const double ab = a2 + b2[k2];
#pragma unroll
            for (int k3 = 0; k3 < NP; ++k3) {
                const double r2 = ab + c2[k3];
                const double g = green_far2_f64<KER>(r2, kappa);
                if ((k2 + k3) & 1)
                    acc1 = __fma_rn(g, q1[k2 * NP + k3], acc1);
                else
                    acc0 = __fma_rn(g, q1[k2 * NP + k3], acc0);
            }
        }
    }
    return 0.5 * (acc0 + acc1);   // the terms are doubled (green_far2_f64)
}

// ---------------------------------------------------------------------------
// Interactions of one workgroup: 256 consecutive targets of one batch.
// ---------------------------------------------------------------------------
template <int N, int KER>
__global__ __launch_bounds__(kGroupSize) void interact_f64(
    const double4* __restrict__ tgt, const int64_t* __restrict__ tgt_orig,
    const double4* __restrict__ src, const int32_t* __restrict__ group_batch,
    const int64_t* __restrict__ group_first, const int64_t* __restrict__ batch_end,
    const int32_t* __restrict__ far_off, const int32_t* __restrict__ far_slot,
    const int32_t* __restrict__ near_off, const int64_t* __restrict__ near_begin,
    const int64_t* __restrict__ near_count, const double* __restrict__ slot_nodes,
    const double* __restrict__ qhat,
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
    const int64_t wave_first = first + (threadIdx.x & ~63);
    if (wave_first >= end)
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
        acc += far_sum_f64<N, KER>(t.x, t.y, t.z, slot_nodes + slot * 3 * NP, qhat + slot * P,
                                   kappa);
    }
    const int n_end = near_off[b + 1];
    for (int e = near_off[b]; e < n_end; ++e)
        acc += near_sum_f64<KER>(t.x, t.y, t.z, src + near_begin[e],
                                 static_cast<int32_t>(near_count[e]), kappa);

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

__global__ __launch_bounds__(256) void gather_charges(double4* __restrict__ src,
                                                      float4* __restrict__ src32,
                                                      const int64_t* __restrict__ order,
                                                      const double* __restrict__ q, int64_t ns)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j < ns) {
        const double v = q[order[j]];
        src[j].w = v;
        if (src32)
            src32[j].w = static_cast<float>(v);
    }
}

__global__ __launch_bounds__(256) void pack_sources(int64_t ns, const double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    const double* __restrict__ z,
                                                    const double* __restrict__ q,
                                                    double4* __restrict__ out)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j < ns)
        out[j] = make_double4(x[j], y[j], z[j], q[j]);
}

template <int KER>
__global__ __launch_bounds__(256) void direct_f64(int64_t nt, const double* __restrict__ tx,
                                                  const double* __restrict__ ty,
                                                  const double* __restrict__ tz, int64_t ns,
                                                  const double4* __restrict__ src,
                                                  double* __restrict__ phi, KernelConst kc)
{
    __shared__ double exp_tab[64];
    if constexpr (KER == 1)
        fill_exp2_table(exp_tab);
    const KernelArg kappa{kc.kappa, kc.delta2, exp_tab};
    const int64_t base = static_cast<int64_t>(blockIdx.x) * blockDim.x;
    if (base + (threadIdx.x & ~63) >= nt)
        return;
    int64_t i = base + threadIdx.x;
    const bool valid = i < nt;
    if (!valid)
        i = nt - 1;
    double acc = 0.0;
    for (int64_t j0 = 0; j0 < ns; j0 += (int64_t(1) << 30)) {
        const int64_t left = ns - j0;
        const int32_t cnt = static_cast<int32_t>(left < (int64_t(1) << 30) ? left : (int64_t(1) << 30));
        acc += near_sum_f64<KER>(tx[i], ty[i], tz[i], src + j0, cnt, kappa);
    }
    if (valid)
        phi[i] = acc;
}

// ---------------------------------------------------------------------------
// dispatch over the interpolation degree
// ---------------------------------------------------------------------------

template <int N, int KER>
hipError_t run_interact(const DevicePlan& d, double* phi, KernelConst kc, hipStream_t s)
{
    if (d.ngroups == 0)
        return hipSuccess;
    const NearLists nl = near_lists(d);
    hipLaunchKernelGGL((interact_f64<N, KER>), dim3(static_cast<unsigned>(d.ngroups)),
                       dim3(d.group_threads), 0, s, d.tgt, d.tgt_orig, d.src, d.group_batch,
                       d.group_first, d.batch_end, d.far_off, d.far_slot, nl.off, nl.begin,
                       nl.count, d.slot_nodes, d.qhat, nl.pc_off, nl.pc_base, nl.pair_out,
                       nl.batch_begin, phi, kc);
    return hipGetLastError();
}

#define BLTC_DEGREE_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

}  // namespace

hipError_t launch_gather_charges(const DevicePlan& d, const double* q, hipStream_t s)
{
    if (d.ns == 0)
        return hipSuccess;
    hipLaunchKernelGGL(gather_charges, dim3(static_cast<unsigned>((d.ns + 255) / 256)), dim3(256),
                       0, s, d.src, d.src32, d.src_order, q, d.ns);
    return hipGetLastError();
}

hipError_t launch_interact(const DevicePlan& d, const KernelParams& kp, double* phi,
                           hipStream_t s)
{
    const KernelConst kc = kp.kconst();
    switch (d.degree) {
#define X(n)                                                                   \
    case n:                                                                    \
        return kp.kernel == 1 ? run_interact<n, 1>(d, phi, kc, s)              \
             : kp.kernel == 2 ? run_interact<n, 2>(d, phi, kc, s)              \
                              : run_interact<n, 0>(d, phi, kc, s);
        BLTC_DEGREE_CASES(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_pack_sources(int64_t ns, const double* x, const double* y, const double* z,
                               const double* q, double4* out, hipStream_t s)
{
    if (ns == 0)
        return hipSuccess;
    hipLaunchKernelGGL(pack_sources, dim3(static_cast<unsigned>((ns + 255) / 256)), dim3(256), 0,
                       s, ns, x, y, z, q, out);
    return hipGetLastError();
}

hipError_t launch_direct(int64_t nt, const double* tx, const double* ty, const double* tz,
                         int64_t ns, const double4* src, const KernelParams& kp, double* phi,
                         hipStream_t s)
{
    if (nt == 0)
        return hipSuccess;
    const dim3 grid(static_cast<unsigned>((nt + 255) / 256));
    const KernelConst kc = kp.kconst();
    if (kp.kernel == 1)
        hipLaunchKernelGGL(direct_f64<1>, grid, dim3(256), 0, s, nt, tx, ty, tz, ns, src, phi, kc);
    else if (kp.kernel == 2)
        hipLaunchKernelGGL(direct_f64<2>, grid, dim3(256), 0, s, nt, tx, ty, tz, ns, src, phi, kc);
    else
        hipLaunchKernelGGL(direct_f64<0>, grid, dim3(256), 0, s, nt, tx, ty, tz, ns, src, phi, kc);
    return hipGetLastError();
}

}  // namespace bltc
