// kernels_cp.hip -- cluster-particle treecode: proxy potentials at the
// target clusters' Chebyshev points, and their interpolation down to the
// targets.
//
// Direct sums reuse the interaction kernels.  The proxy potentials have their
// own kernel (below), which uses the tensor-product form of each cluster's
// grid.  The last step: every target receives, for each cluster on its
// root-to-leaf path that has proxy potentials, the barycentric interpolant
// (eq. 4, tensor product over x, y, z) of those potentials at its position:
//   phi(x) += sum_k L_k1(x1) L_k2(x2) L_k3(x3) phihat_k
//           = (sum_k a_1k1 a_2k2 a_3k3 phihat_k) / (D_1 D_2 D_3),
// with a_lk = w_k / (x_l - t_lk) and D_l = sum_k a_lk, or a one-hot row and
// D_l = 1 when x_l is within DBL_MIN of a node (eq. 5; the lowest such k).
// One target per lane, 256 targets of one target leaf per workgroup; the
// cluster grids and proxy potentials are wave-uniform (scalar loads).
#include <cfloat>

#include "device_common.hpp"
#include "kernels_cp.hpp"

namespace bltc {
namespace {

using namespace dev;

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

// ---------------------------------------------------------------------------
// Proxy potentials: for every target cluster B (a slot) and every source
// batch C approximated with it, phat_B[k] += sum_{j in C} G(t_k, y_j) q_j at
// B's Chebyshev points t_k = (t_1k1, t_2k2, t_3k3).  The grid is a tensor
// product, so r^2 = (t_1k1 - y_1)^2 + [(t_2k2 - y_2)^2 + (t_3k3 - y_3)^2]:
// a lane owns one (k2, k3) and three consecutive k1 and forms the bracket
// once for its three terms.  Sources are wave-uniform (scalar loads).  The
// pair is approximated, so r >= R - r_B - r_C > 0 (no zero-distance case).
//
// A slot's list is cut into pieces of at most a few thousand sources (runs of
// whole list entries; d.chunk_* on the host side), one wave per (piece, part):
// part w holds lane items 64 w .. 64 w + 63 of the slot's G (n+1)^2 items,
// G = ceil((n+1)/3), item l = (g (n+1) + k2) (n+1) + k3 with k1 = 3 g + u,
// u < 3.  A piece writes its sums to row piece_row of `out` (the caller adds
// up the rows of a slot in piece order).  Workgroup b runs on die b mod 8;
// all parts of a piece take the same die (they read the same sources).
//
// FP32-mixed: points and sources relative to the source batch's center, FP32
// terms summed in FP32 for at most kProxyFlush sources, then in FP64; a batch
// whose bounding sphere comes closer to B's than the close-pair cut-off of
// the mixed near field (tau) takes FP64 terms instead.
// ---------------------------------------------------------------------------
constexpr int kProxyK1 = 3;
constexpr int kProxyFlush = 32;

template <int N>
constexpr int proxy_parts()
{
    return (((N + 1 + kProxyK1 - 1) / kProxyK1) * (N + 1) * (N + 1) + 63) / 64;
}

template <int N, int KER, bool MIXED>
__global__ __launch_bounds__(64) void proxy_potentials(
    int64_t npieces, const int32_t* __restrict__ piece_slot,
    const int64_t* __restrict__ piece_entry, const int64_t* __restrict__ piece_entries,
    const int64_t* __restrict__ piece_row, const double* __restrict__ slot_nodes,
    const double4* __restrict__ src, const float4* __restrict__ src32,
    const double4* __restrict__ node_info, const double4* __restrict__ batch_info,
    const int64_t* __restrict__ near_begin, const int64_t* __restrict__ near_count,
    const int32_t* __restrict__ near_leaf, double* __restrict__ out, KernelConst kc)
{
    constexpr int NP = N + 1;
    constexpr int NP2 = NP * NP;
    constexpr int P = NP2 * NP;
    constexpr int G = (NP + kProxyK1 - 1) / kProxyK1;
    constexpr int parts = proxy_parts<N>();
    __shared__ double exp_tab[64];
    if constexpr (KER == 1)
        fill_exp2_table(exp_tab);
    const KernelArg ka{kc.kappa, kc.delta2, exp_tab};
    const KernelArg32 nk = kernel_arg32(kc.kappa, kc.delta2);

    const int64_t b = blockIdx.x;
    const int64_t kd = b >> 3;
    const int64_t piece = (kd / parts) * 8 + (b & 7);
    if (piece >= npieces)
        return;
    const int64_t slot = piece_slot[piece];
    const int lane = threadIdx.x;
    const int item = static_cast<int>(kd % parts) * 64 + lane;
    const bool live = item < G * NP2;
    const int it = live ? item : 0;
    const int g = it / NP2;
    const int k2 = (it - g * NP2) / NP;
    const int k3 = it - g * NP2 - k2 * NP;
    const double* __restrict__ nd = slot_nodes + slot * 3 * NP;
    double t1[kProxyK1];
#pragma unroll
    for (int u = 0; u < kProxyK1; ++u)
        t1[u] = nd[kProxyK1 * g + u < NP ? kProxyK1 * g + u : NP - 1];
    const double t2 = nd[NP + k2], t3 = nd[2 * NP + k3];

    double acc[kProxyK1];
#pragma unroll
    for (int u = 0; u < kProxyK1; ++u)
        acc[u] = 0.0;
    const double4 bi = MIXED ? batch_info[slot] : double4{0.0, 0.0, 0.0, 0.0};
    const int64_t e_end = piece_entry[piece] + piece_entries[piece];
    for (int64_t e = piece_entry[piece]; e < e_end; ++e) {
        const int64_t jb = near_begin[e];
        const int32_t nc = static_cast<int32_t>(near_count[e]);
        bool fast = false;
        double4 li = double4{0.0, 0.0, 0.0, 0.0};
        if constexpr (MIXED) {
            li = node_info[near_leaf[e]];
            const double dx = bi.x - li.x, dy = bi.y - li.y, dz = bi.z - li.z;
            const double dist = sqrt(dx * dx + dy * dy + dz * dz);
            const double tau = kMixedTauRel * (dist + bi.w + 2.0 * li.w);
            fast = dist - bi.w - li.w > 1.0625 * tau;
        }
        if (fast) {
            float l1[kProxyK1];
#pragma unroll
            for (int u = 0; u < kProxyK1; ++u)
                l1[u] = static_cast<float>(t1[u] - li.x);
            const float l2 = static_cast<float>(t2 - li.y), l3 = static_cast<float>(t3 - li.z);
            const float4* __restrict__ S = src32 + jb;
            for (int j0 = 0; j0 < nc; j0 += kProxyFlush) {
                const int j1 = nc - j0 < kProxyFlush ? nc : j0 + kProxyFlush;
                float ra[kProxyK1];
#pragma unroll
                for (int u = 0; u < kProxyK1; ++u)
                    ra[u] = 0.0f;
#pragma unroll 2
                for (int j = j0; j < j1; ++j) {
                    const float4 p = S[j];
                    const float d2 = l2 - p.y, d3 = l3 - p.z;
                    const float bc = __fmaf_rn(d2, d2, d3 * d3);
#pragma unroll
                    for (int u = 0; u < kProxyK1; ++u) {
                        const float d1 = l1[u] - p.x;
                        ra[u] = __fmaf_rn(green_f32<KER>(__fmaf_rn(d1, d1, bc), nk), p.w, ra[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < kProxyK1; ++u)
                    acc[u] += static_cast<double>(ra[u]);
            }
        } else {
            const double4* __restrict__ S = src + jb;
#pragma unroll 2
            for (int j = 0; j < nc; ++j) {
                const double4 p = S[j];
                const double d2 = t2 - p.y, d3 = t3 - p.z;
                const double bc = __fma_rn(d2, d2, d3 * d3);
#pragma unroll
                for (int u = 0; u < kProxyK1; ++u) {
                    const double d1 = t1[u] - p.x;
                    const double r2 = __fma_rn(d1, d1, bc);
                    // FP64 plans sum 2 G (the Newton step's factor, halved at
                    // the store: the same sums exactly); here the FP32-mixed
                    // plans' FP64 terms are added to FP32 partial sums
                    const double gv = MIXED ? green_far_f64<KER>(r2, ka) : green_far2_f64<KER>(r2, ka);
                    acc[u] = __fma_rn(gv, p.w, acc[u]);
                }
            }
        }
    }
    if (live) {
        double* __restrict__ dst = out + piece_row[piece] * P + k2 * NP + k3;
#pragma unroll
        for (int u = 0; u < kProxyK1; ++u)
            if (kProxyK1 * g + u < NP)
                dst[(kProxyK1 * g + u) * NP2] = MIXED ? acc[u] : 0.5 * acc[u];
    }
}

template <int N, int KER>
hipError_t run_proxy(const DevicePlan& d, const double* slot_nodes, bool mixed, double* out,
                     KernelConst kc, hipStream_t s)
{
    const int64_t blocks = ((d.nchunks + 7) / 8) * 8 * proxy_parts<N>();
    if (mixed)
        hipLaunchKernelGGL((proxy_potentials<N, KER, true>), dim3(static_cast<unsigned>(blocks)),
                           dim3(64), 0, s, d.nchunks, d.chunk_slot, d.chunk_begin, d.chunk_count,
                           d.chunk_dst, slot_nodes, d.src, d.src32, d.node_info, d.batch_info,
                           d.near_begin, d.near_count, d.near_leaf, out, kc);
    else
        hipLaunchKernelGGL((proxy_potentials<N, KER, false>), dim3(static_cast<unsigned>(blocks)),
                           dim3(64), 0, s, d.nchunks, d.chunk_slot, d.chunk_begin, d.chunk_count,
                           d.chunk_dst, slot_nodes, d.src, d.src32, d.node_info, d.batch_info,
                           d.near_begin, d.near_count, d.near_leaf, out, kc);
    return hipGetLastError();
}

#define BLTC_DEGREE_CASES(X) \
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16)

}  // namespace

hipError_t launch_proxy_potentials(const DevicePlan& d, const double* slot_nodes,
                                   const KernelParams& kp, double* out, hipStream_t s)
{
    if (d.nchunks == 0)
        return hipSuccess;
    const bool mixed = kp.precision == 1;
    if (mixed && (!d.src32 || !d.node_info || !d.batch_info))
        return hipErrorInvalidValue;
    const KernelConst kc = kp.kconst();
    hipError_t e = hipErrorInvalidValue;
    switch (d.degree) {
#define X(n)                                                                        \
    case n:                                                                         \
        e = kp.kernel == 1 ? run_proxy<n, 1>(d, slot_nodes, mixed, out, kc, s)      \
          : kp.kernel == 2 ? run_proxy<n, 2>(d, slot_nodes, mixed, out, kc, s)      \
                           : run_proxy<n, 0>(d, slot_nodes, mixed, out, kc, s);     \
        break;
        BLTC_DEGREE_CASES(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
    return e;
}

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
