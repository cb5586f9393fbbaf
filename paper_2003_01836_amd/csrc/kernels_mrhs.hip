// kernels_mrhs.hip -- batch/cluster interactions for up to 16 charge vectors
// at once (eqs. 9 and 11 with a matrix of charges).
//
// The kernel values G(x_i, y_j) do not depend on the charge vector, so a pair
// is evaluated once and contracted with all right-hand sides on the matrix
// cores:  Phi[i][m] += sum_j G[i][j] Q[j][m].  A wave owns 64 targets of one
// batch as four 16-target tiles.  Per step of 4 sources (or proxy points),
// lane l evaluates G for target row (l % 16) of each tile and source column
// (l / 16) on the VALU -- exactly the MFMA A-operand layout -- and loads
// Q[source l/16][rhs l%16] -- the B-operand layout -- so the G tile goes
// straight from the VALU into v_mfma_*_16x16x4 without any shuffle.  On
// gfx950 the matrix core and the VALU of a SIMD do not issue at the same time
// (measured: their costs add, within a wave and across waves), so a step costs
// its VALU work plus its MFMAs.
//
// Result layouts of the 16x16x4 MFMAs on gfx950 (checked on the device):
//   f64: lane l, register r holds D[4r + l/16][l % 16]
//   f32: lane l, register r holds D[4(l/16) + r][l % 16]
// Rows are targets, columns are right-hand sides.
#include "device_common.hpp"
#include "kernels.hpp"

namespace bltc {
namespace {

using namespace dev;

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kRhs = 16;
constexpr int kMixedFlushSteps = 32;   // FP32 MFMA partial sums cover <= 128 sources

constexpr double kTauRel = kMixedTauRel;

// Steps of 4 sources whose coordinates and charges are in flight ahead of the
// step being evaluated (a ring of registers per lane).  The FP32 path gains
// from a deep ring; the FP64 path is bound by its VALU and MFMA work, and more
// registers would cost it a wave per SIMD.
constexpr int kAheadF64 = 1;
constexpr int kAheadMixed = 3;
// FP32 partial sums are moved to FP64 after this many rounds of kAheadMixed steps
constexpr int kFlushRounds = kMixedFlushSteps / kAheadMixed;

// Loads and stores through the global address space: the descriptor's
// pointers are read from memory, so the compiler cannot prove that they are
// global, and a flat access in flight makes every wait cover all loads.
// Coordinates are loaded as 3-vectors: a dead 4th register would be reused at
// once and force a wait for the load.
typedef float f3v __attribute__((ext_vector_type(3)));
typedef double d3v __attribute__((ext_vector_type(3)));

template <typename T>
__device__ __forceinline__ T gload(const void* p)
{
    return *(const __attribute__((address_space(1))) T*)(p);
}

// values the whole wave shares, moved to scalar registers (vector loads of
// list entries are not known to be uniform)
__device__ __forceinline__ int32_t uniform32(int32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint64_t u = static_cast<uint64_t>(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
    return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

// the same from a uniform base and a 32-bit byte offset (the SGPR-base form
// of the load: no 64-bit address arithmetic per lane)
template <typename T>
__device__ __forceinline__ T gload_at(const void* base, uint32_t byte_off)
{
    return gload<T>(static_cast<const char*>(base) + byte_off);
}

template <typename T>
__device__ __forceinline__ void gstore(T* p, T v)
{
    *(__attribute__((address_space(1))) T*)(p) = v;
}

// Order of the far-field steps over a cluster's (n+1)^3 proxy points: the
// grid's (n+1)^2 lines (k1, k2) go to the four source columns of a step in
// rounds -- line 4R + c to column c in round R -- and a round takes n + 1
// steps, k3 = 0..n.  A lane thus keeps one line for n + 1 steps: the x- and
// y-part of its targets' squared distances is formed once per round, and a
// step forms one difference and one FMA per value (the separable grid of
// eq. 11).  Columns past the last line carry zero charges.  The cursor is
// the same in every lane (uniform).
struct GridWalk {
    int np, lines;   // n + 1, (n + 1)^2
    int round, k3;
    __device__ __forceinline__ GridWalk(int n1) : np(n1), lines(n1 * n1), round(0), k3(0) {}
    __device__ __forceinline__ void advance()
    {
        if (++k3 == np) {
            k3 = 0;
            ++round;
        }
    }
    __device__ __forceinline__ bool live(int col) const { return 4 * round + col < lines; }
    // proxy index of column col (the last point for columns past the end)
    __device__ __forceinline__ uint32_t point(int col) const
    {
        const int line = 4 * round + col;
        return static_cast<uint32_t>(line < lines ? line * np + k3 : lines * np - 1);
    }
    __device__ __forceinline__ int steps() const { return ((lines + 3) / 4) * np; }
};

// ---------------------------------------------------------------------------
// FP64: G in FP64 on the VALU, contraction on v_mfma_f64_16x16x4f64.
// ---------------------------------------------------------------------------
template <int KER>
__device__ __forceinline__ void group_mrhs_f64(const MrhsDesc& d, int g, const double* exp_tab)
{
    const double4* __restrict__ tgt = d.tgt;
    const int64_t* __restrict__ tgt_orig = d.tgt_orig;
    const double4* __restrict__ src = d.src;
    const double* __restrict__ qm = d.qm;
    const int32_t* __restrict__ far_off = d.far_off;
    const int32_t* __restrict__ far_slot = d.far_slot;
    const int32_t* __restrict__ near_off = d.near_off;
    const int64_t* __restrict__ near_begin = d.near_begin;
    const int64_t* __restrict__ near_count = d.near_count;
    const double4* __restrict__ proxies = d.proxies;
    const double* __restrict__ qhat16 = d.qhat16;
    double* __restrict__ phi = d.phi;
    const int32_t np = d.np;
    const int64_t phi_ld = d.phi_ld;
    const int32_t m_count = d.mc;
    const KernelArg kappa{d.kc.kappa, d.kc.delta2, exp_tab};
    const int b = gload<int32_t>(d.group_batch + g);
    if (b < 0)
        return;
    const int64_t first = gload<int64_t>(d.group_first + g);
    const int64_t end = gload<int64_t>(d.batch_end + b);
    const int64_t wave_first = first + (threadIdx.x & ~63);
    if (wave_first >= end)
        return;
    const int lane = threadIdx.x & 63;
    const int row = lane & 15;
    const int col = lane >> 4;

    double tx[4], ty[4], tz[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int64_t i = wave_first + 16 * t + row;
        i = i < end ? i : end - 1;
        const d3v v = gload<d3v>(tgt + i);
        tx[t] = v.x;
        ty[t] = v.y;
        tz[t] = v.z;
    }
    d4v acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        acc[t] = d4v{0.0, 0.0, 0.0, 0.0};

    const int P = np * np * np;
    const int f_end = gload<int32_t>(far_off + b + 1);
    for (int f = gload<int32_t>(far_off + b); f < f_end; ++f) {
        const int64_t slot = gload<int32_t>(far_slot + f);
        const double4* __restrict__ px = proxies + slot * P;
        const double* __restrict__ qh = qhat16 + slot * static_cast<int64_t>(P) * kRhs;
        // software pipeline: the proxy points and charges of kAheadF64 steps
        // are in flight; ring slot u serves steps u, u + kAheadF64, ... and is
        // reloaded once its step is evaluated.  Whole rounds of steps are
        // evaluated; steps past the end carry zero charges.
        GridWalk ld(np), ev(np);   // next step to load, next step to evaluate
        d3v pn[kAheadF64];
        double qn[kAheadF64];
#pragma unroll
        for (int a = 0; a < kAheadF64; ++a) {
            const uint32_t kk = ld.point(col);
            pn[a] = gload_at<d3v>(px, kk * 32u);
            qn[a] = gload_at<double>(qh, (kk * kRhs + row) * 8u);
            ld.advance();
            // slot 0 first: the loop's first wait then leaves the other slots in flight
            __builtin_amdgcn_sched_barrier(0);
        }
        double ab[4];   // (x - x_k1)^2 + (y - y_k2)^2 of the lane's line
        const int steps = ev.steps();
        for (int s1 = 0; s1 < steps; s1 += kAheadF64) {
#pragma unroll
            for (int u = 0; u < kAheadF64; ++u) {
                const double bq = ev.live(col) ? qn[u] : 0.0;
                if (ev.k3 == 0) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const double dx = tx[t] - pn[u].x, dy = ty[t] - pn[u].y;
                        ab[t] = __fma_rn(dy, dy, dx * dx);
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double dz = tz[t] - pn[u].z;
                    const double r2 = __fma_rn(dz, dz, ab[t]);
                    const double gv = green_far2_f64<KER>(r2, kappa);   // 2 G
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(gv, bq, acc[t], 0, 0, 0);
                }
                ev.advance();
                const uint32_t kk = ld.point(col);
                pn[u] = gload_at<d3v>(px, kk * 32u);
                qn[u] = gload_at<double>(qh, (kk * kRhs + row) * 8u);
                ld.advance();
                // keep the step's order: its reload is issued after its MFMAs
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    const int n_end = gload<int32_t>(near_off + b + 1);
    for (int e = gload<int32_t>(near_off + b); e < n_end; ++e) {
        const int64_t nb = uniform64(gload<int64_t>(near_begin + e));
        const int32_t cnt = uniform32(static_cast<int32_t>(gload<int64_t>(near_count + e)));
        const double4* sp = src + nb;
        const double* qp = qm + nb * kRhs;
        d3v pn[kAheadF64];
        double qn[kAheadF64];
#pragma unroll
        for (int a = 0; a < kAheadF64; ++a) {
            const uint32_t jj = 4 * a + col < cnt ? 4 * a + col : cnt - 1;
            pn[a] = gload_at<d3v>(sp, jj * 32u);
            qn[a] = gload_at<double>(qp, (jj * kRhs + row) * 8u);
            // slot 0 first: the loop's first wait then leaves the other slots in flight
            __builtin_amdgcn_sched_barrier(0);
        }
        for (int32_t j1 = 0; j1 < cnt; j1 += 4 * kAheadF64) {
#pragma unroll
            for (int u = 0; u < kAheadF64; ++u) {
                const int32_t j0 = j1 + 4 * u;
                const double bq = (j0 + col < cnt) ? qn[u] : 0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double dx = tx[t] - pn[u].x, dy = ty[t] - pn[u].y, dz = tz[t] - pn[u].z;
                    const double r2 = __fma_rn(dz, dz, __fma_rn(dy, dy, dx * dx));
                    const double gv = green_near2_f64<KER>(r2, kappa);   // 2 G
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(gv, bq, acc[t], 0, 0, 0);
                }
                const int32_t jn = j0 + 4 * kAheadF64 + col;
                const uint32_t jj = jn < cnt ? jn : cnt - 1;
                pn[u] = gload_at<d3v>(sp, jj * 32u);
                qn[u] = gload_at<double>(qp, (jj * kRhs + row) * 8u);
                // keep the step's order: its reload is issued after its MFMAs
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    if (row < m_count) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = wave_first + 16 * t + 4 * r + col;
                if (i < end)   // the kernel values were doubled (green_*2_f64)
                    gstore(phi + row * phi_ld + gload<int64_t>(tgt_orig + i), 0.5 * acc[t][r]);
            }
    }
}

// ---------------------------------------------------------------------------
// FP32-mixed: G in FP32 on local coordinates (close pairs from FP64
// coordinates), contraction on v_mfma_f32_16x16x4f32, FP32 partial sums over
// <= kMixedFlushSteps steps, accumulated per target and right-hand side in FP64.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void flush_f32(f4v (&part)[4], double (&acc)[4][4])
{
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            acc[t][r] += static_cast<double>(part[t][r]);
        part[t] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
    }
}

template <int KER>
__device__ __forceinline__ void group_mrhs_mixed(const MrhsDesc& d, int g, const double* exp_tab,
                                                 double* __restrict__ tl)
{
    const double4* __restrict__ tgt = d.tgt;
    const int64_t* __restrict__ tgt_orig = d.tgt_orig;
    const double4* __restrict__ src = d.src;
    const float4* __restrict__ src32 = d.src32;
    const float* __restrict__ qm32 = d.qm32;
    const double4* __restrict__ node_info = d.node_info;
    const double4* __restrict__ batch_info = d.batch_info;
    const int32_t* __restrict__ far_off = d.far_off;
    const int32_t* __restrict__ far_slot = d.far_slot;
    const int32_t* __restrict__ near_off = d.near_off;
    const int64_t* __restrict__ near_begin = d.near_begin;
    const int64_t* __restrict__ near_count = d.near_count;
    const int32_t* __restrict__ near_leaf = d.near_leaf;
    const int32_t* __restrict__ slot_cluster = d.slot_cluster;
    const float4* __restrict__ proxies32 = d.proxies32;
    const float* __restrict__ qhat16 = d.qhat16f;
    double* __restrict__ phi = d.phi;
    const int32_t np = d.np;
    const int64_t phi_ld = d.phi_ld;
    const int32_t m_count = d.mc;
    const KernelArg kappa{d.kc.kappa, d.kc.delta2, exp_tab};
    const int b = gload<int32_t>(d.group_batch + g);
    if (b < 0)
        return;
    const int64_t first = gload<int64_t>(d.group_first + g);
    const int64_t end = gload<int64_t>(d.batch_end + b);
    const int64_t wave_first = first + (threadIdx.x & ~63);
    if (wave_first >= end)
        return;
    const int lane = threadIdx.x & 63;
    const int row = lane & 15;
    const int col = lane >> 4;
    const KernelArg32 nk = kernel_arg32(d.kc.kappa, d.kc.delta2);

    // The targets' FP64 coordinates wait in LDS, in slots of this lane only
    // (no barrier): held in registers they would take 24 VGPRs for the whole
    // group and keep the kernel from four waves per SIMD.  The accesses are
    // volatile, or the compiler forwards the stored values and keeps them in
    // registers after all.
    volatile double* tl_lane = tl + threadIdx.x;
    auto tc = [tl_lane](int t, int l) -> volatile double& {
        return tl_lane[(3 * t + l) * kGroupSize];
    };
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        int64_t i = wave_first + 16 * t + row;
        i = i < end ? i : end - 1;
        const d3v v = gload<d3v>(tgt + i);
        tc(t, 0) = v.x;
        tc(t, 1) = v.y;
        tc(t, 2) = v.z;
    }
    double acc[4][4];
    f4v part[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        part[t] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int r = 0; r < 4; ++r)
            acc[t][r] = 0.0;
    }

    const int P = np * np * np;
    const int f_end = gload<int32_t>(far_off + b + 1);
    for (int f = gload<int32_t>(far_off + b); f < f_end; ++f) {
        const int64_t slot = gload<int32_t>(far_slot + f);
        const d4v ci = gload<d4v>(node_info + gload<int32_t>(slot_cluster + slot));
        // targets relative to the cluster center (proxy points are stored so)
        float ux[4], uy[4], uz[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            ux[t] = static_cast<float>(tc(t, 0) - ci.x);
            uy[t] = static_cast<float>(tc(t, 1) - ci.y);
            uz[t] = static_cast<float>(tc(t, 2) - ci.z);
        }
        const float4* __restrict__ px = proxies32 + slot * P;
        const float* __restrict__ qh = qhat16 + slot * static_cast<int64_t>(P) * kRhs;
        GridWalk ld(np), ev(np);   // next step to load, next step to evaluate
        f3v pn[kAheadMixed];
        float qn[kAheadMixed];
#pragma unroll
        for (int a = 0; a < kAheadMixed; ++a) {
            const uint32_t kk = ld.point(col);
            pn[a] = gload_at<f3v>(px, kk * 16u);
            qn[a] = gload_at<float>(qh, (kk * kRhs + row) * 4u);
            ld.advance();
            // slot 0 first: the loop's first wait then leaves the other slots in flight
            __builtin_amdgcn_sched_barrier(0);
        }
        float ab[4];   // (x - x_k1)^2 + (y - y_k2)^2 of the lane's line
        int rounds = 0;
        const int steps = ev.steps();
        for (int s1 = 0; s1 < steps; s1 += kAheadMixed) {
#pragma unroll
            for (int u = 0; u < kAheadMixed; ++u) {
                const float bq = ev.live(col) ? qn[u] : 0.0f;
                if (ev.k3 == 0) {
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float dx = ux[t] - pn[u].x, dy = uy[t] - pn[u].y;
                        ab[t] = __fmaf_rn(dy, dy, dx * dx);
                    }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float dz = uz[t] - pn[u].z;
                    const float r2 = __fmaf_rn(dz, dz, ab[t]);
                    const float gv = green_f32<KER>(r2, nk);
                    part[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv, bq, part[t], 0, 0, 0);
                }
                ev.advance();
                const uint32_t kk = ld.point(col);
                pn[u] = gload_at<f3v>(px, kk * 16u);
                qn[u] = gload_at<float>(qh, (kk * kRhs + row) * 4u);
                ld.advance();
                // keep the step's order: its reload is issued after its MFMAs
                __builtin_amdgcn_sched_barrier(0);
            }
            if (++rounds == kFlushRounds) {
                flush_f32(part, acc);
                rounds = 0;
            }
        }
        flush_f32(part, acc);
    }

    const d4v bi = gload<d4v>(batch_info + b);
    const int n_end = gload<int32_t>(near_off + b + 1);
    for (int e = gload<int32_t>(near_off + b); e < n_end; ++e) {
        const d4v li = gload<d4v>(node_info + gload<int32_t>(near_leaf + e));
        const double ddx = bi.x - li.x, ddy = bi.y - li.y, ddz = bi.z - li.z;
        const double extent = sqrt(ddx * ddx + ddy * ddy + ddz * ddz) + bi.w + 2.0 * li.w;
        const double tau = kTauRel * extent;
        const float tau2 = static_cast<float>(tau * tau);
        float ux[4], uy[4], uz[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            ux[t] = static_cast<float>(tc(t, 0) - li.x);
            uy[t] = static_cast<float>(tc(t, 1) - li.y);
            uz[t] = static_cast<float>(tc(t, 2) - li.z);
        }
        const int64_t nb = uniform64(gload<int64_t>(near_begin + e));
        const int32_t cnt = uniform32(static_cast<int32_t>(gload<int64_t>(near_count + e)));
        const float4* sp = src32 + nb;
        const float* qp = qm32 + nb * kRhs;
        f3v pn[kAheadMixed];
        float qn[kAheadMixed];
#pragma unroll
        for (int a = 0; a < kAheadMixed; ++a) {
            const uint32_t jj = 4 * a + col < cnt ? 4 * a + col : cnt - 1;
            pn[a] = gload_at<f3v>(sp, jj * 16u);
            qn[a] = gload_at<float>(qp, (jj * kRhs + row) * 4u);
            // slot 0 first: the loop's first wait then leaves the other slots in flight
            __builtin_amdgcn_sched_barrier(0);
        }
        int rounds = 0;
        for (int32_t j1 = 0; j1 < cnt; j1 += 4 * kAheadMixed) {
#pragma unroll
            for (int u = 0; u < kAheadMixed; ++u) {
                const int32_t j0 = j1 + 4 * u;
                const float bq = (j0 + col < cnt) ? qn[u] : 0.0f;
                float gv[4], r2v[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float dx = ux[t] - pn[u].x, dy = uy[t] - pn[u].y, dz = uz[t] - pn[u].z;
                    r2v[t] = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, dx * dx));
                    gv[t] = green_f32<KER>(r2v[t], nk);
                }
                if (fminf(fminf(r2v[0], r2v[1]), fminf(r2v[2], r2v[3])) <= tau2) {
                    // close pairs: the kernel value from the exact coordinates, in FP64
                    const d3v p64 = gload<d3v>(src + nb + (j0 + col < cnt ? j0 + col : cnt - 1));
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (r2v[t] <= tau2) {
                            const double dx = tc(t, 0) - p64.x;
                            const double dy = tc(t, 1) - p64.y;
                            const double dz = tc(t, 2) - p64.z;
                            const double r2 = __fma_rn(dz, dz, __fma_rn(dy, dy, dx * dx));
                            gv[t] = static_cast<float>(green_near_f64<KER>(r2, kappa));
                        }
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    part[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[t], bq, part[t], 0, 0, 0);
                const int32_t jn = j0 + 4 * kAheadMixed + col;
                const uint32_t jj = jn < cnt ? jn : cnt - 1;
                pn[u] = gload_at<f3v>(sp, jj * 16u);
                qn[u] = gload_at<float>(qp, (jj * kRhs + row) * 4u);
                // keep the step's order: its reload is issued after its MFMAs
                __builtin_amdgcn_sched_barrier(0);
            }
            if (++rounds == kFlushRounds) {
                flush_f32(part, acc);
                rounds = 0;
            }
        }
        flush_f32(part, acc);
    }
    if (row < m_count) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = wave_first + 16 * t + 4 * col + r;
                if (i < end)
                    gstore(phi + row * phi_ld + gload<int64_t>(tgt_orig + i), acc[t][r]);
            }
    }
}

// four waves per SIMD on the FP32-mixed form, as for the work queue below
template <int KER, int PREC>
__global__ __launch_bounds__(kGroupSize) __attribute__((amdgpu_waves_per_eu(PREC == 1 ? 4 : 1)))
void interact_mrhs(MrhsDesc d)
{
    __shared__ double exp_tab[64];
    __shared__ double tlds[PREC == 0 ? 1 : 12 * kGroupSize];
    if constexpr (KER == 1)
        fill_exp2_table(exp_tab);
    if constexpr (PREC == 0)
        group_mrhs_f64<KER>(d, blockIdx.x, exp_tab);
    else
        group_mrhs_mixed<KER>(d, blockIdx.x, exp_tab, tlds);
}

// Persistent work queue over the groups of many systems: every workgroup
// repeatedly takes the next unit (system, group) -- heaviest first -- until
// the queue is empty.  The counter is reset by reset_counter before a launch.
template <int KER, int PREC>
// The FP32-mixed form is held to four waves per SIMD (the compiler then keeps
// 128 VGPRs and spills a few to scratch; measured faster than three waves
// without spills).
__global__ __launch_bounds__(kGroupSize) __attribute__((amdgpu_waves_per_eu(PREC == 1 ? 4 : 1)))
void interact_queue(const MrhsDesc* __restrict__ descs, const int2* __restrict__ units,
                    int32_t nunits, int32_t* __restrict__ counter)
{
    __shared__ int32_t next;
    __shared__ double exp_tab[64];
    __shared__ double tlds[PREC == 0 ? 1 : 12 * kGroupSize];
    if constexpr (KER == 1)
        fill_exp2_table(exp_tab);
    for (;;) {
        if (threadIdx.x == 0)
            next = atomicAdd(counter, 1);
        __syncthreads();
        const int32_t u = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
        if (u >= nunits)
            break;
        const int2 w = units[u];
        const int32_t sys = __builtin_amdgcn_readfirstlane(w.x);
        const int32_t g = __builtin_amdgcn_readfirstlane(w.y);
        if constexpr (PREC == 0)
            group_mrhs_f64<KER>(descs[sys], g, exp_tab);
        else
            group_mrhs_mixed<KER>(descs[sys], g, exp_tab, tlds);
    }
}

__global__ void reset_counter(int32_t* counter)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        counter[0] = 0;
}

// charges of up to 16 vectors into tree order, padded with zeros:
// qm[j][m] = q[(m0 + m) * q_ld + order[j]] for m < mc
__global__ __launch_bounds__(256) void gather_charges16(double* __restrict__ qm,
                                                        float* __restrict__ qm32,
                                                        const int64_t* __restrict__ order,
                                                        const double* __restrict__ q, int64_t q_ld,
                                                        int32_t mc, int64_t ns)
{
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= ns * kRhs)
        return;
    const int64_t j = idx / kRhs;
    const int m = static_cast<int>(idx - j * kRhs);
    const double v = m < mc ? q[m * q_ld + order[j]] : 0.0;
    qm[idx] = v;
    if (qm32)
        qm32[idx] = static_cast<float>(v);
}

}  // namespace

hipError_t launch_gather_charges16(const DevicePlan& d, const double* q, int64_t q_ld, int32_t mc,
                                   hipStream_t s)
{
    if (d.ns == 0)
        return hipSuccess;
    const int64_t total = d.ns * kRhs;
    hipLaunchKernelGGL(gather_charges16, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256),
                       0, s, d.qm, d.qm32, d.src_order, q, q_ld, mc, d.ns);
    return hipGetLastError();
}

MrhsDesc make_mrhs_desc(const DevicePlan& d, const KernelParams& kp, double* phi, int64_t phi_ld,
                        int32_t mc)
{
    MrhsDesc m;
    m.tgt = d.tgt;
    m.tgt_orig = d.tgt_orig;
    m.src = d.src;
    m.src32 = d.src32;
    m.qm = d.qm;
    m.qm32 = d.qm32;
    m.node_info = d.node_info;
    m.batch_info = d.batch_info;
    m.group_batch = d.group_batch;
    m.group_first = d.group_first;
    m.batch_end = d.batch_end;
    m.far_off = d.far_off;
    m.far_slot = d.far_slot;
    m.near_off = d.near_off;
    m.near_begin = d.near_begin;
    m.near_count = d.near_count;
    m.near_leaf = d.near_leaf;
    m.slot_cluster = d.slot_cluster;
    m.proxies = d.proxies;
    m.proxies32 = d.proxies32;
    m.qhat16 = d.qhat16;
    m.qhat16f = d.qhat16f;
    m.phi = phi;
    m.phi_ld = phi_ld;
    m.np = d.degree + 1;
    m.mc = mc;
    m.kc = kp.kconst();
    return m;
}

static bool mrhs_tables_ok(const DevicePlan& d, int32_t precision)
{
    if (precision == 1)
        return d.src32 && d.qm32 && d.qhat16f && d.proxies32 && d.node_info && d.batch_info;
    return d.qm && d.qhat16 && d.proxies;
}

hipError_t launch_interact_mrhs(const DevicePlan& d, const KernelParams& kp, double* phi,
                                int64_t phi_ld, int32_t mc, hipStream_t s)
{
    if (d.ngroups == 0)
        return hipSuccess;
    if (!mrhs_tables_ok(d, kp.precision))
        return hipErrorInvalidValue;
    const MrhsDesc m = make_mrhs_desc(d, kp, phi, phi_ld, mc);
    const dim3 grid(static_cast<unsigned>(d.ngroups)), block(kGroupSize);
    void (*fn)(MrhsDesc) = nullptr;
    if (kp.precision == 1)
        fn = kp.kernel == 1 ? interact_mrhs<1, 1> : kp.kernel == 2 ? interact_mrhs<2, 1>
                                                                   : interact_mrhs<0, 1>;
    else
        fn = kp.kernel == 1 ? interact_mrhs<1, 0> : kp.kernel == 2 ? interact_mrhs<2, 0>
                                                                   : interact_mrhs<0, 0>;
    hipLaunchKernelGGL(fn, grid, block, 0, s, m);
    return hipGetLastError();
}

using QueueKernel = void (*)(const MrhsDesc*, const int2*, int32_t, int32_t*);

static QueueKernel queue_kernel(const KernelParams& kp)
{
    if (kp.precision == 1)
        return kp.kernel == 1 ? interact_queue<1, 1> : kp.kernel == 2 ? interact_queue<2, 1>
                                                                      : interact_queue<0, 1>;
    return kp.kernel == 1 ? interact_queue<1, 0> : kp.kernel == 2 ? interact_queue<2, 0>
                                                                  : interact_queue<0, 0>;
}

hipError_t launch_reset_counter(int32_t* counter, hipStream_t s)
{
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_interact_queue(const MrhsDesc* descs, const int2* units, int32_t nunits,
                                 int32_t* counter, const KernelParams& kp, int32_t workgroups,
                                 hipStream_t s)
{
    if (nunits == 0)
        return hipSuccess;
    const dim3 grid(static_cast<unsigned>(workgroups)), block(kGroupSize);
    hipLaunchKernelGGL(queue_kernel(kp), grid, block, 0, s, descs, units, nunits, counter);
    return hipGetLastError();
}

const void* interact_queue_symbol(const KernelParams& kp)
{
    return reinterpret_cast<const void*>(queue_kernel(kp));
}

}  // namespace bltc
