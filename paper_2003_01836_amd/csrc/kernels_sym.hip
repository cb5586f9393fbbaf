// kernels_sym.hip -- the near field (eq. 9) of mutual leaf pairs when the
// targets are the sources.
//
// G(x, y) = G(y, x): for two different leaves B and C that are in each
// other's direct lists, every kernel value serves both directions.  One wave
// per sub-unit: up to kChunks x 64 of B's particles as targets (one per lane
// and chunk, all in registers) against all of C's particles, which stream
// through the scalar cache as wave-uniform sources in blocks of kBlk.  Per
// pair the wave forms one kernel value g, adds the row term g q_j to the
// lane's sum for that target and the column term g q_i to the lane's column
// register of that source.  After a block, a butterfly over the lanes
// (log2 kBlk xor-shuffle stages inside each group of kBlk lanes, then
// log2(64 / kBlk) across the groups) leaves in lane l the sum over the
// sub-unit's targets of column l mod kBlk, which lanes 0..kBlk-1 store; the
// butterfly's cost is shared by the kChunks targets of a lane.  Every sum has
// a fixed order, so the results are deterministic.
//
// FP32-mixed rounding: a column sum covers up to 512 target terms, but as 64
// lane sums of at most kChunks = 8 terms combined by the butterfly's 6 levels
// of pairwise additions, so its rounding error is at most (8 + 6) eps32 times
// the sum of the magnitudes of its terms -- that of a 14-term sequential sum,
// below the row sums' (at most kFlushEvery = 128 FP32 terms, then FP64).  A
// close pair's kernel value comes from the FP64 coordinates and is rounded
// once to FP32 like every other value: the FP64 branch removes the coordinate
// rounding that 1/r amplifies for close pairs, and what is left is one FP32
// rounding of the value and one of its product with the charge.
#include "kernels.hpp"
#include "device_common.hpp"

namespace bltc {
namespace {

using namespace dev;

constexpr int kBlk = 8;           // sources per butterfly block
constexpr int kChunks = 8;        // 64-target chunks held in registers (FP32-mixed)
constexpr int kChunks64 = 8;      // the same for the FP64 kernel
static_assert(kSymTargetsMixed == 64 * kChunks && kSymTargetsF64 == 64 * kChunks64,
              "sub-unit sizes");

constexpr double kTauRel = kMixedTauRel;   // the mixed interaction kernel's cut-off
constexpr int kFlushEvery = 128;           // FP32 row sums span at most this many sources

// lane l returns the sum over the wave's 64 lanes of v[l % kBlk] (v is consumed)
template <typename T>
__device__ __forceinline__ T column_sums(T (&v)[kBlk], int lane)
{
#pragma unroll
    for (int d = kBlk / 2; d >= 1; d >>= 1) {
        const bool up = (lane & d) != 0;
#pragma unroll
        for (int k = 0; k < d; ++k) {
            // lanes with bit d clear keep column k, the others column k + d
            const T x = v[k], y = v[k + d];
            const T sx = __shfl_xor(x, d), sy = __shfl_xor(y, d);
            v[k] = up ? y + sy : x + sx;
        }
    }
    T r = v[0];
#pragma unroll
    for (int d = kBlk; d < 64; d <<= 1)
        r += __shfl_xor(r, d);
    return r;
}

// ---------------------------------------------------------------------------
// FP64
// ---------------------------------------------------------------------------
// One mutual pair: the doubled kernel value serves the row term (into the
// target's sum `row`) and the column term (into the source's column `col`).
// CHECK = false: the unit's leaves are apart (r^2 > 0 for every pair), so the
// zero-distance test of green_near2_f64 is left out.
template <int KER, bool CHECK>
__device__ __forceinline__ void pair_term_f64(double tx, double ty, double tz, double tq,
                                              const double4 p, const KernelArg& ka, double& row,
                                              double& col)
{
    const double dx = tx - p.x;
    const double dy = ty - p.y;
    const double dz = tz - p.z;
    const double r2 = __fma_rn(dz, dz, __fma_rn(dy, dy, dx * dx));
    const double g = CHECK ? green_near2_f64<KER>(r2, ka) : green_far2_f64<KER>(r2, ka);  // 2 G
    row = __fma_rn(g, p.w, row);
    col = __fma_rn(g, tq, col);
}

template <int KER, bool CHECK>
__device__ __forceinline__ void pairs_unit_f64(const SymUnit& u, const double4* __restrict__ src,
                                               double* __restrict__ out, const KernelArg& ka)
{
    const int lane = threadIdx.x;
    const double4* __restrict__ S = src + u.sb;
    const int nch = (u.nb + 63) / 64;   // uniform, <= kChunks64 by construction
    double tx[kChunks64], ty[kChunks64], tz[kChunks64], tq[kChunks64], a0[kChunks64],
        a1[kChunks64];
#pragma unroll
    for (int k = 0; k < kChunks64; ++k) {
        const int i = 64 * k + lane;
        const double4 t = src[u.tb + (i < u.nb ? i : u.nb - 1)];
        tx[k] = t.x;
        ty[k] = t.y;
        tz[k] = t.z;
        tq[k] = i < u.nb ? t.w : 0.0;   // no column terms from lanes past the end
        a0[k] = 0.0;
        a1[k] = 0.0;
    }
    // full blocks: the kBlk sources are loaded once (wave-uniform, into SGPRs)
    // and serve every chunk of targets
    int s0 = 0;
    for (; s0 + kBlk <= u.nc; s0 += kBlk) {
        double4 p[kBlk];
#pragma unroll
        for (int m = 0; m < kBlk; ++m)
            p[m] = S[s0 + m];
        double v[kBlk];
#pragma unroll
        for (int m = 0; m < kBlk; ++m)
            v[m] = 0.0;
#pragma unroll
        for (int k = 0; k < kChunks64; ++k) {
            if (k >= nch)
                break;
#pragma unroll
            for (int m = 0; m < kBlk; ++m)
                pair_term_f64<KER, CHECK>(tx[k], ty[k], tz[k], tq[k], p[m], ka,
                                          (m & 1) ? a1[k] : a0[k], v[m]);
        }
        const double cs = column_sums(v, lane);
        out[u.coff + s0 + (lane & (kBlk - 1))] = 0.5 * cs;   // lanes l, l + kBlk, ... agree
    }
    if (s0 < u.nc) {
        // the last, partial block
        const int cnt = u.nc - s0;   // uniform, < kBlk
        double v[kBlk];
#pragma unroll
        for (int m = 0; m < kBlk; ++m)
            v[m] = 0.0;
#pragma unroll
        for (int k = 0; k < kChunks64; ++k) {
            if (k >= nch)
                break;
#pragma unroll
            for (int m = 0; m < kBlk; ++m) {
                if (m >= cnt)
                    break;
                pair_term_f64<KER, CHECK>(tx[k], ty[k], tz[k], tq[k], S[s0 + m], ka,
                                          (m & 1) ? a1[k] : a0[k], v[m]);
            }
        }
        const double cs = column_sums(v, lane);
        if (lane < cnt)
            out[u.coff + s0 + lane] = 0.5 * cs;
    }
#pragma unroll
    for (int k = 0; k < kChunks64; ++k) {
        const int i = 64 * k + lane;
        if (k < nch && i < u.nb)
            out[u.roff + i] = 0.5 * (a0[k] + a1[k]);
    }
}

// Two waves per SIMD: 8 chunks of targets and a source block in flight take
// about 250 VGPRs (one wave per SIMD when left to the compiler, or spills at
// three); measured on 10^6 particles, 19.2 ms against 24.9 ms (one wave) and
// 20.5 ms (4 chunks, three waves).
template <int KER>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void near_pairs_f64(
    const SymUnit* __restrict__ units, const double4* __restrict__ src, double* __restrict__ out,
    KernelConst kc)
{
    __shared__ double exp_tab[64];
    if constexpr (KER == 1)
        fill_exp2_table(exp_tab);
    const KernelArg ka{kc.kappa, kc.delta2, exp_tab};
    const SymUnit u = units[blockIdx.x];
    if (u.apart)
        pairs_unit_f64<KER, false>(u, src, out, ka);
    else
        pairs_unit_f64<KER, true>(u, src, out, ka);
}

// ---------------------------------------------------------------------------
// FP32-mixed: FP32 kernel values on coordinates local to C's center (sources
// as stored for the mixed path, targets rounded once).  A pair with
// r^2 <= tau^2 takes its kernel value from the FP64 coordinates (computed in
// FP64, rounded once), so coordinate rounding never enters a close pair; the
// value then serves the row and the column term like any other.  FP32 row
// sums over at most kFlushEvery sources go into the lane's FP64 sums.
// ---------------------------------------------------------------------------
template <int KER>
__device__ __forceinline__ float value_f32(float x, float y, float z, const float4 p,
                                           const KernelArg32& nk, float& r2)
{
    const float dx = x - p.x;
    const float dy = y - p.y;
    const float dz = z - p.z;
    r2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
    return green_f32<KER>(r2, nk);
}

// one block of sources [s0, s0 + cnt) (cnt = kBlk when FULL) against the
// super-chunk's targets; column terms into v
template <int KER, bool FULL>
__device__ __forceinline__ void block_mixed(const float (&tx)[kChunks], const float (&ty)[kChunks],
                                            const float (&tz)[kChunks], const float (&tq)[kChunks],
                                            float (&ra)[kChunks], float (&v)[kBlk], int nch,
                                            const float4* __restrict__ s32,
                                            const double4* __restrict__ s64, int cnt,
                                            const double4* __restrict__ tgt64, int c0, int nb,
                                            float tau2, const KernelArg32& nk,
                                            const KernelArg& ka, int lane)
{
#pragma unroll
    for (int k = 0; k < kChunks; ++k) {
        if (k >= nch)
            break;
#pragma unroll
        for (int q = 0; q < kBlk / 4; ++q) {
            float g[4], r[4], w[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (FULL || 4 * q + m < cnt) {
                    const float4 p = s32[4 * q + m];
                    g[m] = value_f32<KER>(tx[k], ty[k], tz[k], p, nk, r[m]);
                    w[m] = p.w;
                } else {
                    g[m] = 0.0f;
                    r[m] = __builtin_inff();
                    w[m] = 0.0f;
                }
            }
            if (fminf(fminf(r[0], r[1]), fminf(r[2], r[3])) <= tau2) {
                // rare: kernel values of the close pairs from the FP64 coordinates
                // (straight-line over the quad, then one select per pair)
                const int i = c0 + 64 * k + lane;
                const double4 t = tgt64[i < nb ? i : nb - 1];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    if (FULL || 4 * q + m < cnt) {
                        const double4 p = s64[4 * q + m];
                        const double dx = t.x - p.x;
                        const double dy = t.y - p.y;
                        const double dz = t.z - p.z;
                        const double r2 = __fma_rn(dz, dz, __fma_rn(dy, dy, dx * dx));
                        const float gg = static_cast<float>(green_near_f64<KER>(r2, ka));
                        g[m] = r[m] <= tau2 ? gg : g[m];
                    }
                }
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                ra[k] = __fmaf_rn(g[m], w[m], ra[k]);
                v[4 * q + m] = __fmaf_rn(g[m], tq[k], v[4 * q + m]);
            }
        }
    }
}

// four waves per SIMD (128 VGPRs, no spills): 8% faster than the three the
// default allocation allows
template <int KER>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void near_pairs_mixed(
    const SymUnit* __restrict__ units, const double4* __restrict__ src,
    const float4* __restrict__ src32, const double4* __restrict__ node_info,
    const double4* __restrict__ batch_info, double* __restrict__ out, KernelConst kc)
{
    __shared__ double exp_tab[64];
    if constexpr (KER == 1)
        fill_exp2_table(exp_tab);
    const KernelArg ka{kc.kappa, kc.delta2, exp_tab};
    const KernelArg32 nk = kernel_arg32(kc.kappa, kc.delta2);
    const SymUnit u = units[blockIdx.x];
    const int lane = threadIdx.x;
    // tau of the pair: the larger of the two directions' values
    const double4 bi = batch_info[u.batch];
    const double4 li = node_info[u.leaf];
    const double ex = bi.x - li.x, ey = bi.y - li.y, ez = bi.z - li.z;
    const double extent = sqrt(ex * ex + ey * ey + ez * ez) +
                          fmax(bi.w + 2.0 * li.w, li.w + 2.0 * bi.w);
    const double tau = kTauRel * extent;
    const float tau2 = static_cast<float>(tau * tau);
    const float4* __restrict__ S32 = src32 + u.sb;
    const double4* __restrict__ S64 = src + u.sb;
    const double4* __restrict__ T64 = src + u.tb;
    const int nch = (u.nb + 63) / 64;   // uniform, <= kChunks by construction
    float tx[kChunks], ty[kChunks], tz[kChunks], tq[kChunks], ra[kChunks];
    double acc[kChunks];
#pragma unroll
    for (int k = 0; k < kChunks; ++k) {
        const int i = 64 * k + lane;
        const int pos = i < u.nb ? i : u.nb - 1;
        const double4 t = T64[pos];
        tx[k] = static_cast<float>(t.x - li.x);
        ty[k] = static_cast<float>(t.y - li.y);
        tz[k] = static_cast<float>(t.z - li.z);
        tq[k] = i < u.nb ? src32[u.tb + pos].w : 0.0f;   // no column terms past the end
        ra[k] = 0.0f;
        acc[k] = 0.0;
    }
    int s0 = 0;
    for (; s0 + kBlk <= u.nc; s0 += kBlk) {
        float v[kBlk];
#pragma unroll
        for (int m = 0; m < kBlk; ++m)
            v[m] = 0.0f;
        block_mixed<KER, true>(tx, ty, tz, tq, ra, v, nch, S32 + s0, S64 + s0, kBlk, T64, 0, u.nb,
                               tau2, nk, ka, lane);
        const float cs = column_sums(v, lane);
        if (lane < kBlk)
            out[u.coff + s0 + lane] = static_cast<double>(cs);
        if ((s0 + kBlk) % kFlushEvery == 0) {
#pragma unroll
            for (int k = 0; k < kChunks; ++k) {
                acc[k] += static_cast<double>(ra[k]);
                ra[k] = 0.0f;
            }
        }
    }
    if (s0 < u.nc) {
        const int cnt = u.nc - s0;
        float v[kBlk];
#pragma unroll
        for (int m = 0; m < kBlk; ++m)
            v[m] = 0.0f;
        block_mixed<KER, false>(tx, ty, tz, tq, ra, v, nch, S32 + s0, S64 + s0, cnt, T64, 0, u.nb,
                                tau2, nk, ka, lane);
        const float cs = column_sums(v, lane);
        if (lane < cnt)
            out[u.coff + s0 + lane] = static_cast<double>(cs);
    }
#pragma unroll
    for (int k = 0; k < kChunks; ++k) {
        const int i = 64 * k + lane;
        if (k < nch && i < u.nb)
            out[u.roff + i] = acc[k] + static_cast<double>(ra[k]);
    }
}

// One round of mutual-pair results into the per-target sums: one workgroup
// per batch, one target per lane, the batch's entries of the round in order.
__global__ __launch_bounds__(256) void fold_pairs(const int64_t* __restrict__ begin,
                                                  const int64_t* __restrict__ end,
                                                  const int32_t* __restrict__ off,
                                                  const int64_t* __restrict__ base,
                                                  const double* __restrict__ out,
                                                  double* __restrict__ acc, int first)
{
    const int b = blockIdx.x;
    const int64_t b0 = begin[b], b1 = end[b];
    const int e0 = off[b], e1 = off[b + 1];
    for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) {
        const int64_t p = i - b0;
        double v = first ? 0.0 : acc[i];
        for (int e = e0; e < e1; ++e)
            v += out[base[e] + p];
        acc[i] = v;
    }
}

}  // namespace

hipError_t launch_fold_pairs(int64_t nbatches, const int64_t* begin, const int64_t* end,
                             const int32_t* off, const int64_t* base, const double* out,
                             double* acc, bool first, hipStream_t s)
{
    if (nbatches == 0)
        return hipSuccess;
    if (!begin || !end || !off || !base || !out || !acc)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(fold_pairs, dim3(static_cast<unsigned>(nbatches)), dim3(256), 0, s, begin,
                       end, off, base, out, acc, first ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_near_pairs(const DevicePlan& d, int64_t first, int64_t count,
                             const KernelParams& kp, hipStream_t s)
{
    if (!d.sym || count == 0)
        return hipSuccess;
    if (!d.sym_unit || !d.sym_out || first < 0 || first + count > d.sym_units)
        return hipErrorInvalidValue;
    const KernelConst kc = kp.kconst();
    const dim3 grid(static_cast<unsigned>(count));
    const SymUnit* units = d.sym_unit + first;
    const size_t lds = 0;
    if (kp.precision == 1) {
        if (!d.src32 || !d.node_info || !d.batch_info)
            return hipErrorInvalidValue;
        if (kp.kernel == 1)
            hipLaunchKernelGGL(near_pairs_mixed<1>, grid, dim3(64), lds, s, units, d.src,
                               d.src32, d.node_info, d.batch_info, d.sym_out, kc);
        else if (kp.kernel == 2)
            hipLaunchKernelGGL(near_pairs_mixed<2>, grid, dim3(64), lds, s, units, d.src,
                               d.src32, d.node_info, d.batch_info, d.sym_out, kc);
        else
            hipLaunchKernelGGL(near_pairs_mixed<0>, grid, dim3(64), lds, s, units, d.src,
                               d.src32, d.node_info, d.batch_info, d.sym_out, kc);
    } else {
        if (kp.kernel == 1)
            hipLaunchKernelGGL(near_pairs_f64<1>, grid, dim3(64), lds, s, units, d.src,
                               d.sym_out, kc);
        else if (kp.kernel == 2)
            hipLaunchKernelGGL(near_pairs_f64<2>, grid, dim3(64), lds, s, units, d.src,
                               d.sym_out, kc);
        else
            hipLaunchKernelGGL(near_pairs_f64<0>, grid, dim3(64), lds, s, units, d.src,
                               d.sym_out, kc);
    }
    return hipGetLastError();
}

}  // namespace bltc
