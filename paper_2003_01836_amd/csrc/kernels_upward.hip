// kernels_upward.hip -- the upward pass (eqs. 14-15) as a dense contraction on
// the matrix cores.
//
// For the sources j of one cluster, with the 1-D barycentric factors
// a_l[j][k] = w_k / (y_jl - s_lk) (one-hot when the coordinate coincides with a
// node, eq. 5) and q~_jm = q_jm / (D_1 D_2 D_3) (eq. 14), eq. 15 reads
//     Qhat[(k1, m)][(k2, k3)] = sum_j (a_1[j][k1] q~_jm) * (a_2[j][k2] a_3[j][k3])
// i.e. the product (a_1 o q~)^T (a_2 (.) a_3) of an N_C x (n+1)M and an
// N_C x (n+1)^2 matrix (o: outer product per row, (.): row-wise Kronecker
// product).  One workgroup takes a chunk of a cluster's sources and a set of
// 16x16 output tiles; the factors of 128 sources at a time are formed in FP64
// in LDS, and each wave accumulates its tiles with v_mfma_f64_16x16x4f64,
// K = 4 sources per instruction.  Chunks of the same cluster are summed in a
// fixed order by a second kernel (deterministic).
//
// The Hermite variant has 2(n+1) factors per dimension -- A_k then B_k, the
// Hermite basis on the same nodes -- and hence 8 (n+1)^3 outputs per cluster
// in the layout ((a1 (n+1) + k1) 2(n+1) + a2 (n+1) + k2) 2(n+1) + a3 (n+1) + k3.
#include <cfloat>

#include "kernels.hpp"

#include <type_traits>

namespace bltc {
namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int kTile = 128;          // sources staged in LDS at a time
constexpr int kTilesPerWave = 8;    // 16x16 output tiles accumulated per wave
constexpr int kTilesPerGroup = 4 * kTilesPerWave;

// 1-D factors of one coordinate (eqs. 4-5, 14), FP64; returns D_l.
__device__ __forceinline__ double factors_rt(double yv, const double* __restrict__ s, int np,
                                             double* __restrict__ a)
{
    const int n = np - 1;
    int hit = -1;
    for (int k = np - 1; k >= 0; --k)
        if (fabs(yv - s[k]) < DBL_MIN)
            hit = k;
    if (hit >= 0) {
        for (int k = 0; k < np; ++k)
            a[k] = (k == hit) ? 1.0 : 0.0;
        return 1.0;
    }
    double sum = 0.0;
    for (int k = 0; k < np; ++k) {
        const double w = ((k & 1) ? -1.0 : 1.0) * ((k == 0 || k == n) ? 0.5 : 1.0);
        const double v = w / (yv - s[k]);
        a[k] = v;
        sum += v;
    }
    return sum;
}

// Hermite factors of one coordinate: a[k] = A_k(y) = (1 - 2 c_k (y - s_k)) L_k(y)^2,
// a[np + k] = B_k(y) = (y - s_k) L_k(y)^2 with L_k from eq. 4 and c_k = L_k'(s_k)
// (given); one-hot A and zero B at a node (eq. 5).  Returns 1 (the factors are
// normalized).
__device__ __forceinline__ double factors_hermite(double yv, const double* __restrict__ s,
                                                  const double* __restrict__ c, int np,
                                                  double* __restrict__ a)
{
    const int n = np - 1;
    int hit = -1;
    for (int k = np - 1; k >= 0; --k)
        if (fabs(yv - s[k]) < DBL_MIN)
            hit = k;
    if (hit >= 0) {
        for (int k = 0; k < np; ++k) {
            a[k] = (k == hit) ? 1.0 : 0.0;
            a[np + k] = 0.0;
        }
        return 1.0;
    }
    double sum = 0.0;
    for (int k = 0; k < np; ++k) {
        const double w = ((k & 1) ? -1.0 : 1.0) * ((k == 0 || k == n) ? 0.5 : 1.0);
        const double v = w / (yv - s[k]);
        a[k] = v;
        sum += v;
    }
    const double inv = 1.0 / sum;
    for (int k = 0; k < np; ++k) {
        const double d = yv - s[k];
        const double l = a[k] * inv;
        const double l2 = l * l;
        a[k] = (1.0 - 2.0 * c[k] * d) * l2;
        a[np + k] = d * l2;
    }
    return 1.0;
}

// grid: x = chunk, y = tile pass.  mw = 1 (one charge vector, taken from
// src[j].w) or 16 (charges from qm[j][16]).  Output of a chunk: dst[k * mw + m]
// with dst = out + chunk_dst[c] * P * mw (rows below nslots are the final
// modified charges of single-chunk clusters, the others partial sums).
// Tiles are dealt round-robin to the 4 waves: wave w of tile pass p owns
// tiles p * 32 + w + 4u, u < 8.
__device__ __forceinline__ void upward_chunk(
    const double4* __restrict__ src, const double* __restrict__ qm, int32_t mw,
    const int32_t* __restrict__ chunk_slot, const int64_t* __restrict__ chunk_begin,
    const int64_t* __restrict__ chunk_count, const int64_t* __restrict__ chunk_dst,
    const double* __restrict__ slot_nodes, int32_t np, int32_t nf, double* __restrict__ out,
    int c, int pass, double* __restrict__ lds)
{
    // nf factors per dimension: np (Lagrange) or 2 np (Hermite)
    const bool hermite = nf != np;
    const int nf2 = nf * nf;
    const int P = nf2 * nf;
    double* __restrict__ A1 = lds;                   // [kTile][nf]
    double* __restrict__ A2 = A1 + kTile * nf;       // [kTile][nf]
    double* __restrict__ A3 = A2 + kTile * nf;       // [kTile][nf]
    double* __restrict__ SQ = A3 + kTile * nf;       // [kTile][mw]  q~
    double* __restrict__ SN = SQ + kTile * mw;       // [3][np]      nodes
    double* __restrict__ SC = SN + 3 * np;           // [3][np]      c_k (Hermite)

    const int64_t slot = chunk_slot[c];
    const int64_t begin = chunk_begin[c];
    const int64_t count = chunk_count[c];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    if (tid < 3 * np)
        SN[tid] = slot_nodes[slot * 3 * np + tid];
    if (hermite) {
        __syncthreads();
        if (tid < 3 * np) {
            // c_k = L_k'(s_k) = sum_{j != k} 1 / (s_k - s_j) of dimension tid / np
            const double* sd = SN + (tid / np) * np;
            const int k = tid % np;
            double cs = 0.0;
            for (int j = 0; j < np; ++j)
                if (j != k)
                    cs += 1.0 / (sd[k] - sd[j]);
            SC[tid] = cs;
        }
    }

    const int R = nf * mw;                  // rows (k1, m)
    const int RT = (R + 15) / 16;
    const int CT = (nf2 + 15) / 16;         // columns (k2, k3)
    const int T = RT * CT;
    const int tbase = pass * kTilesPerGroup + wave;

    // per owned tile: LDS offsets of this lane's row factor and column factors
    int rk1[kTilesPerWave], rm[kTilesPerWave], ck2[kTilesPerWave], ck3[kTilesPerWave];
    bool live[kTilesPerWave];
    d4v acc[kTilesPerWave];
#pragma unroll
    for (int u = 0; u < kTilesPerWave; ++u) {
        const int t = tbase + 4 * u;
        live[u] = t < T;
        const int rt = live[u] ? t / CT : 0;
        const int ct = live[u] ? t - rt * CT : 0;
        const int r = rt * 16 + (lane & 15);
        const int cc = ct * 16 + (lane & 15);
        // rows/cols past the end get index -1: their operand is zero
        rk1[u] = r < R ? r / mw : -1;
        rm[u] = r < R ? r - (r / mw) * mw : 0;
        ck2[u] = cc < nf2 ? cc / nf : -1;
        ck3[u] = cc < nf2 ? cc - (cc / nf) * nf : 0;
        acc[u] = d4v{0.0, 0.0, 0.0, 0.0};
    }
    __syncthreads();

    for (int64_t t0 = 0; t0 < count; t0 += kTile) {
        const int tn = static_cast<int>(count - t0 < kTile ? count - t0 : kTile);
        if (tid < kTile) {
            if (tid < tn) {
                const int64_t j = begin + t0 + tid;
                const double4 p = src[j];
                const double D =
                    hermite ? factors_hermite(p.x, SN, SC, np, A1 + tid * nf) *
                                  factors_hermite(p.y, SN + np, SC + np, np, A2 + tid * nf) *
                                  factors_hermite(p.z, SN + 2 * np, SC + 2 * np, np, A3 + tid * nf)
                            : factors_rt(p.x, SN, np, A1 + tid * nf) *
                                  factors_rt(p.y, SN + np, np, A2 + tid * nf) *
                                  factors_rt(p.z, SN + 2 * np, np, A3 + tid * nf);
                const double inv = 1.0 / D;
                if (mw == 1) {
                    SQ[tid] = p.w * inv;
                } else {
                    for (int m = 0; m < mw; ++m)
                        SQ[tid * mw + m] = qm[j * 16 + m] * inv;
                }
            } else {
                // zero rows: the partial last step of the tile contributes nothing
                for (int k = 0; k < nf; ++k) {
                    A1[tid * nf + k] = 0.0;
                    A2[tid * nf + k] = 0.0;
                    A3[tid * nf + k] = 0.0;
                }
                for (int m = 0; m < mw; ++m)
                    SQ[tid * mw + m] = 0.0;
            }
        }
        __syncthreads();
        if (tbase < T) {
            const int steps = (tn + 3) / 4;
            for (int st = 0; st < steps; ++st) {
                const int j = 4 * st + (lane >> 4);
#pragma unroll
                for (int u = 0; u < kTilesPerWave; ++u) {
                    if (!live[u])
                        continue;
                    const double av = rk1[u] >= 0 ? A1[j * nf + rk1[u]] * SQ[j * mw + rm[u]] : 0.0;
                    const double bv = ck2[u] >= 0 ? A2[j * nf + ck2[u]] * A3[j * nf + ck3[u]] : 0.0;
                    acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }

    // f64 result layout: lane l, register r holds D[4r + l/16][l % 16]
    double* __restrict__ dst = out + chunk_dst[c] * static_cast<int64_t>(P) * mw;
#pragma unroll
    for (int u = 0; u < kTilesPerWave; ++u) {
        if (!live[u])
            continue;
        const int t = tbase + 4 * u;
        const int rt = t / CT;
        const int ct = t - rt * CT;
        const int cc = ct * 16 + (lane & 15);
        if (cc >= nf2)
            continue;
        const int k2 = cc / nf, k3 = cc - (cc / nf) * nf;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = rt * 16 + 4 * r + (lane >> 4);
            if (row < R) {
                const int k1 = row / mw, m = row - (row / mw) * mw;
                dst[static_cast<int64_t>((k1 * nf + k2) * nf + k3) * mw + m] = acc[u][r];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// One charge vector, Lagrange factors, n + 1 = NP <= 16 nodes per dimension:
// the output Qhat[k1][(k2, k3)] has one row tile (k1 < NP <= 16) and
// CT = ceil(NP^2 / 16) column tiles.  Every wave accumulates all CT tiles over
// a quarter of the sources (wave w takes the steps of 4 sources st = w mod 4),
// and the four partial tiles are summed in LDS in the fixed order
// (w0 + w2) + (w1 + w3).  The factors of 128 sources at a time are formed by
// two of the waves, in turns, with the degree known at compile time (the 3 NP
// reciprocals of a source are independent and pipeline); the row operand
// a_1[j][k1] q~_j is stored ready for the matrix core.  Factor rows have one
// zero entry past the last node, which the lanes of rows k1 >= NP and of
// columns past NP^2 read instead of branching.

// |d| < DBL_MIN: zero or subnormal (class bits of -/+ zero and -/+ subnormal)
__device__ __forceinline__ bool below_normal(double d)
{
    return __builtin_amdgcn_class(d, 0x0F0);
}

// The 1-D factors a_k = w_k / (y - s_k) of eq. 14 without the coincidence
// rule, and D = sum_k a_k; `tiny` tells whether some |y - s_k| < DBL_MIN (then
// these values are not used: the caller applies eq. 5).
template <int NP>
__device__ __forceinline__ double factors_np(double yv, const double* __restrict__ s,
                                             double* __restrict__ a, bool& tiny)
{
    double sum = 0.0;
    bool t = false;
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const double d = yv - s[k];
        t |= below_normal(d);
        // 1/d: hardware estimate refined by two Newton steps r <- r + r (1 - d r)
        double r = __builtin_amdgcn_rcp(d);
        r = fma(fma(-d, r, 1.0), r, r);
        r = fma(fma(-d, r, 1.0), r, r);
        const double v = ((k & 1) ? -1.0 : 1.0) * ((k == 0 || k == NP - 1) ? 0.5 : 1.0) * r;
        a[k] = v;
        sum += v;
    }
    tiny = t;
    return sum;
}

// eq. 5: the row of a coordinate that coincides with a node is one-hot at the
// lowest such node, times `scale`
template <int NP>
__device__ __forceinline__ void one_hot_row(double yv, const double* __restrict__ s, double scale,
                                            double* __restrict__ row)
{
    int hit = NP;
#pragma unroll
    for (int k = NP - 1; k >= 0; --k)
        if (below_normal(yv - s[k]))
            hit = k;
#pragma unroll
    for (int k = 0; k < NP; ++k)
        row[k] = (k == hit) ? scale : 0.0;
}

// Hermite factors of one coordinate for the single-vector kernel: row[k] =
// scale A_k(y), row[NP + k] = scale B_k(y), A_k = (1 - 2 c_k (y - s_k)) L_k^2,
// B_k = (y - s_k) L_k^2 with L_k of eq. 4 from the same reciprocals; a
// coordinate on a node (eq. 5) gives a one-hot A and zero B.
template <int NP>
__device__ __forceinline__ void hermite_row(double yv, const double* __restrict__ s,
                                            const double* __restrict__ cs, double scale,
                                            double* __restrict__ row)
{
    double a[NP];
    bool tiny;
    const double inv = 1.0 / factors_np<NP>(yv, s, a, tiny);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const double d = yv - s[k];
        const double l = a[k] * inv;
        const double l2 = l * l;
        row[k] = scale * (__fma_rn(-2.0 * cs[k], d, 1.0) * l2);
        row[NP + k] = scale * (d * l2);
    }
    if (tiny) {
        // rare: the coordinate is on a node
        one_hot_row<NP>(yv, s, scale, row);
#pragma unroll
        for (int k = 0; k < NP; ++k)
            row[NP + k] = 0.0;
    }
}

// FP32-mixed rows of one source: the factors are formed in FP64 as above and
// normalized per dimension before rounding -- L_k = a_k / D_l (eq. 4), or
// A_k, B_k -- so that every stored value is O(1) and the charge multiplies
// the x row: r1 = q L1, r2 = L2, r3 = L3.  A coordinate on a node gives the
// one-hot row of eq. 5.
template <int NP, bool HERM>
__device__ __forceinline__ void rows_f32(const double4 p, bool live, const double* __restrict__ sn,
                                         const double* __restrict__ sc, float* __restrict__ r1,
                                         float* __restrict__ r2, float* __restrict__ r3)
{
    constexpr int NF = HERM ? 2 * NP : NP;
    const double q = live ? p.w : 0.0;
    const double yv[3] = {p.x, p.y, p.z};
    float* const rows[3] = {r1, r2, r3};
#pragma unroll
    for (int l = 2; l >= 0; --l) {
        double a[NF];
        const double scale = l == 0 ? q : 1.0;
        if constexpr (HERM) {
            hermite_row<NP>(yv[l], sn + l * NP, sc + l * NP, scale, a);
        } else {
            bool tiny;
            const double D = factors_np<NP>(yv[l], sn + l * NP, a, tiny);
            if (tiny) {
                one_hot_row<NP>(yv[l], sn + l * NP, scale, a);
            } else {
                const double f = scale / D;
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    a[k] *= f;
            }
        }
#pragma unroll
        for (int k = 0; k < NF; ++k)
            rows[l][k] = static_cast<float>(a[k]);
        rows[l][NF] = 0.0f;
    }
}

// NF factors per dimension: NP Lagrange factors or 2 NP Hermite factors
template <int NP, bool HERM>
constexpr int single_nf()
{
    return HERM ? 2 * NP : NP;
}

template <int NP, bool HERM>
constexpr int single_lds_doubles()
{
    // factor rows [kTile][NF + 1] x 3 (+ c_k of the Hermite factors), or two
    // waves' partial tiles [CT][4][64]
    constexpr int NF = single_nf<NP, HERM>();
    constexpr int rows = 3 * kTile * (NF + 1) + (HERM ? 3 * NP : 0);
    constexpr int parts = 2 * ((NF * NF + 15) / 16) * 256;
    return rows > parts ? rows : parts;
}

// HERM: the Hermite charges (8 (n+1)^3 per cluster, blocked layout
// (f1 NF + f2) NF + f3 with f = a (n+1) + k): rows f1 = 2 NP <= 16, columns
// (f2, f3), factors normalized (q instead of q~).
//
// F32 (FP32-mixed plans): the rows are rounded to FP32 after their FP64
// formation (rows_f32), the products run on v_mfma_f32_16x16x4f32, and each
// wave's FP32 partial tiles -- at most 32 sources of one 128-source tile --
// are added to its FP64 tiles after every tile; outputs stay FP64.
template <int NP, bool HERM, bool F32>
__global__ __launch_bounds__(256) void upward_single(
    const double4* __restrict__ src, const int32_t* __restrict__ chunk_slot,
    const int64_t* __restrict__ chunk_begin, const int64_t* __restrict__ chunk_count,
    const int64_t* __restrict__ chunk_dst, const double* __restrict__ slot_nodes,
    double* __restrict__ out)
{
    constexpr int NF = single_nf<NP, HERM>();
    constexpr int NF2 = NF * NF;
    constexpr int CT = (NF2 + 15) / 16;
    constexpr int SP = NF + 1;                      // row stride: NF factors and a zero
    static_assert(NF <= 16, "one row tile");
    using R = typename std::conditional<F32, float, double>::type;
    __shared__ double lds[single_lds_doubles<NP, HERM>()];
    R* __restrict__ A1 = reinterpret_cast<R*>(lds); // [kTile][SP]  x factors times q~ (q)
    R* __restrict__ A2 = A1 + kTile * SP;           // [kTile][SP]
    R* __restrict__ A3 = A2 + kTile * SP;           // [kTile][SP]
    double* __restrict__ SC = lds + 3 * kTile * SP; // [3][NP] c_k (Hermite)

    const int c = blockIdx.x;
    const int64_t slot = chunk_slot[c];
    const int64_t begin = chunk_begin[c];
    const int64_t count = chunk_count[c];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double* __restrict__ sn = slot_nodes + slot * 3 * NP;   // wave-uniform
    if constexpr (HERM) {
        // c_k = L_k'(s_k) = sum_{j != k} 1 / (s_k - s_j) of dimension tid / NP
        if (tid < 3 * NP) {
            const double* sd = sn + (tid / NP) * NP;
            const int k = tid % NP;
            double cs = 0.0;
            for (int j = 0; j < NP; ++j)
                if (j != k)
                    cs += 1.0 / (sd[k] - sd[j]);
            SC[tid] = cs;
        }
        __syncthreads();
    }

    // this lane's operand offsets: row f1 = lane % 16, columns ct * 16 + lane % 16
    // (rows and columns past the end point at the zero entry)
    const int k1 = lane & 15;
    const int off1 = (lane >> 4) * SP + (k1 < NF ? k1 : NF);
    int off2[CT], off3[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        const int cc = ct * 16 + (lane & 15);
        off2[ct] = (lane >> 4) * SP + (cc < NF2 ? cc / NF : 0);
        off3[ct] = (lane >> 4) * SP + (cc < NF2 ? cc - (cc / NF) * NF : NF);
    }
    d4v acc[CT];
    f4v acc32[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
        acc[ct] = d4v{0.0, 0.0, 0.0, 0.0};
        acc32[ct] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
    }

    for (int64_t t0 = 0; t0 < count; t0 += kTile) {
        const int tn = static_cast<int>(count - t0 < kTile ? count - t0 : kTile);
        // waves 0-1 and 2-3 take turns forming the factors (two SIMDs each)
        const int ft = tid - ((static_cast<int>(t0 / kTile) & 1) ? kTile : 0);
        if (ft >= 0 && ft < kTile) {
            // Rows past the chunk's end get charge 0 (their x row is zero).
            double4 p = double4{0.0, 0.0, 0.0, 0.0};
            const bool live = ft < tn;
            if (live)
                p = src[begin + t0 + ft];
            if constexpr (F32) {
                rows_f32<NP, HERM>(p, live, sn, SC, reinterpret_cast<float*>(A1) + ft * SP,
                                   reinterpret_cast<float*>(A2) + ft * SP,
                                   reinterpret_cast<float*>(A3) + ft * SP);
            } else if constexpr (HERM) {
                hermite_row<NP>(p.z, sn + 2 * NP, SC + 2 * NP, 1.0, A3 + ft * SP);
                hermite_row<NP>(p.y, sn + NP, SC + NP, 1.0, A2 + ft * SP);
                hermite_row<NP>(p.x, sn, SC, live ? p.w : 0.0, A1 + ft * SP);
                A1[ft * SP + NF] = 0.0;
                A2[ft * SP + NF] = 0.0;
                A3[ft * SP + NF] = 0.0;
            } else {
                // z and y factors go to LDS as they are formed; x waits for q~
                double a[NP];
                bool tz, ty, tx;
                const double Dz = factors_np<NP>(p.z, sn + 2 * NP, a, tz);
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    A3[ft * SP + k] = a[k];
                A3[ft * SP + NP] = 0.0;
                const double Dy = factors_np<NP>(p.y, sn + NP, a, ty);
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    A2[ft * SP + k] = a[k];
                A2[ft * SP + NP] = 0.0;
                const double Dx = factors_np<NP>(p.x, sn, a, tx);
                const double D = (tx ? 1.0 : Dx) * (ty ? 1.0 : Dy) * (tz ? 1.0 : Dz);
                const double qt = live ? p.w / D : 0.0;
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    A1[ft * SP + k] = a[k] * qt;
                A1[ft * SP + NP] = 0.0;
                if (tx || ty || tz) {
                    // rare: a coordinate on a node (eq. 5)
                    if (tz)
                        one_hot_row<NP>(p.z, sn + 2 * NP, 1.0, A3 + ft * SP);
                    if (ty)
                        one_hot_row<NP>(p.y, sn + NP, 1.0, A2 + ft * SP);
                    if (tx)
                        one_hot_row<NP>(p.x, sn, qt, A1 + ft * SP);
                }
            }
        }
        __syncthreads();
        const int steps = (tn + 3) / 4;
        for (int st = wave; st < steps; st += 4) {
            const int jb = 4 * st * SP;
            const R av = A1[jb + off1];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const R bv = A2[jb + off2[ct]] * A3[jb + off3[ct]];
                if constexpr (F32)
                    acc32[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc32[ct], 0, 0, 0);
                else
                    acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ct], 0, 0, 0);
            }
        }
        if constexpr (F32) {
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[ct][r] += static_cast<double>(acc32[ct][r]);
                acc32[ct] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
            }
        }
        __syncthreads();
    }

    // (w0 + w2) + (w1 + w3) through LDS; lane l, register r holds D[4r + l/16][l % 16]
    // (f64 MFMA) or D[4 (l/16) + r][l % 16] (f32 MFMA)
    if (wave >= 2) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                lds[(((wave - 2) * CT + ct) * 4 + r) * 64 + lane] = acc[ct][r];
    }
    __syncthreads();
    if (wave < 2) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[ct][r] += lds[((wave * CT + ct) * 4 + r) * 64 + lane];
    }
    __syncthreads();
    if (wave == 1) {
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                lds[(ct * 4 + r) * 64 + lane] = acc[ct][r];
    }
    __syncthreads();
    if (wave == 0) {
        double* __restrict__ dst = out + chunk_dst[c] * static_cast<int64_t>(NF2) * NF;
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int cc = ct * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = F32 ? 4 * (lane >> 4) + r : 4 * r + (lane >> 4);
                if (row < NF && cc < NF2)
                    dst[row * NF2 + cc] = acc[ct][r] + lds[(ct * 4 + r) * 64 + lane];
            }
        }
    }
}

template <int NP, bool HERM = false>
hipError_t launch_single_np(const DevicePlan& d, double* buf, hipStream_t s)
{
    // FP32-mixed plans (they hold FP32 source copies): FP32 matrix-core products
    if (d.src32)
        hipLaunchKernelGGL((upward_single<NP, HERM, true>), dim3(static_cast<unsigned>(d.nchunks)),
                           dim3(256), 0, s, d.src, d.chunk_slot, d.chunk_begin, d.chunk_count,
                           d.chunk_dst, d.slot_nodes, buf);
    else
        hipLaunchKernelGGL((upward_single<NP, HERM, false>), dim3(static_cast<unsigned>(d.nchunks)),
                           dim3(256), 0, s, d.src, d.chunk_slot, d.chunk_begin, d.chunk_count,
                           d.chunk_dst, d.slot_nodes, buf);
    return hipGetLastError();
}

// n + 1 <= 16 nodes (Hermite: n + 1 <= 8): the single-vector kernel; returns
// false for other degrees
bool launch_single(const DevicePlan& d, double* buf, hipStream_t s, hipError_t* err)
{
    if (d.hermite) {
        switch (d.degree + 1) {
        case 2: *err = launch_single_np<2, true>(d, buf, s); return true;
        case 3: *err = launch_single_np<3, true>(d, buf, s); return true;
        case 4: *err = launch_single_np<4, true>(d, buf, s); return true;
        case 5: *err = launch_single_np<5, true>(d, buf, s); return true;
        case 6: *err = launch_single_np<6, true>(d, buf, s); return true;
        case 7: *err = launch_single_np<7, true>(d, buf, s); return true;
        case 8: *err = launch_single_np<8, true>(d, buf, s); return true;
        default: return false;
        }
    }
    switch (d.degree + 1) {
    case 2: *err = launch_single_np<2>(d, buf, s); return true;
    case 3: *err = launch_single_np<3>(d, buf, s); return true;
    case 4: *err = launch_single_np<4>(d, buf, s); return true;
    case 5: *err = launch_single_np<5>(d, buf, s); return true;
    case 6: *err = launch_single_np<6>(d, buf, s); return true;
    case 7: *err = launch_single_np<7>(d, buf, s); return true;
    case 8: *err = launch_single_np<8>(d, buf, s); return true;
    case 9: *err = launch_single_np<9>(d, buf, s); return true;
    case 10: *err = launch_single_np<10>(d, buf, s); return true;
    case 11: *err = launch_single_np<11>(d, buf, s); return true;
    case 12: *err = launch_single_np<12>(d, buf, s); return true;
    case 13: *err = launch_single_np<13>(d, buf, s); return true;
    case 14: *err = launch_single_np<14>(d, buf, s); return true;
    case 15: *err = launch_single_np<15>(d, buf, s); return true;
    case 16: *err = launch_single_np<16>(d, buf, s); return true;
    default: return false;
    }
}

// ---------------------------------------------------------------------------
// 16 charge vectors, Lagrange factors, n + 1 = NP <= 9 nodes per dimension.
// Output tile (k1, ct) is Qhat[k1][m][(k2, k3)] for the 16 vectors m (rows)
// and the 16 columns ct*16 .. ct*16 + 15 of (k2, k3): A[m][j] = L1[j][k1]
// q[j][m] and B[j][(k2, k3)] = L2[j][k2] L3[j][k3], with the factors
// normalized per dimension (L_l = a_l / D_l, eq. 4, so q~ of eq. 14 is the
// charge itself).  The NP * ceil(NP^2 / 16) tiles of a chunk are dealt
// round-robin to the 8 waves of a workgroup and each wave runs over all of
// the chunk's sources, so the factors are formed once per chunk, 128 sources
// at a time: the four quarters of the workgroup take the x, y and z factors
// and the charges (16 per source) of the same 128 sources into LDS, with the
// degree known at compile time.  F32: the rows and charges are rounded to
// FP32 after their FP64 formation, the products run on v_mfma_f32_16x16x4f32,
// and every wave adds its FP32 tiles -- 128 sources -- to FP64 tiles after
// each round.
// ---------------------------------------------------------------------------
constexpr int kMultiTile = 128;
constexpr int kMultiWaves = 8;
constexpr int kMultiMaxNP = 9;
// LDS of one round: three factor rows of kMultiMaxNP + 1 and 16 charges per source
constexpr int kMultiLds = kMultiTile * (3 * (kMultiMaxNP + 1) + 16);

template <int NP>
constexpr int multi_tiles_per_wave()
{
    return (NP * ((NP * NP + 15) / 16) + kMultiWaves - 1) / kMultiWaves;
}

template <int NP, bool F32>
__device__ __forceinline__ void multi_chunk(const double4* __restrict__ src,
                                            const double* __restrict__ qm,
                                            const float* __restrict__ qm32,
                                            const int32_t* __restrict__ chunk_slot,
                                            const int64_t* __restrict__ chunk_begin,
                                            const int64_t* __restrict__ chunk_count,
                                            const int64_t* __restrict__ chunk_dst,
                                            const double* __restrict__ slot_nodes,
                                            double* __restrict__ out, int c, double* lds)
{
    constexpr int NP2 = NP * NP;
    constexpr int CT = (NP2 + 15) / 16;
    constexpr int T = NP * CT;
    constexpr int TW = multi_tiles_per_wave<NP>();
    constexpr int SP = NP + 1;                      // row stride: NP factors and a zero
    using R = typename std::conditional<F32, float, double>::type;
    R* __restrict__ L1 = reinterpret_cast<R*>(lds);
    R* __restrict__ L2 = L1 + kMultiTile * SP;
    R* __restrict__ L3 = L2 + kMultiTile * SP;
    R* __restrict__ SQ = L3 + kMultiTile * SP;      // [kMultiTile][16] charges

    const int64_t slot = chunk_slot[c];
    const int64_t begin = chunk_begin[c];
    const int64_t count = chunk_count[c];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const double* __restrict__ sn = slot_nodes + slot * 3 * NP;   // wave-uniform

    // this wave's tiles t = wave + 8u: row tile k1 = t / CT, column tile t % CT;
    // columns past NP^2 read the zero entry of the rows
    int ok1[TW], ok2[TW], ok3[TW];
    d4v acc[TW];
    f4v acc32[TW];
#pragma unroll
    for (int u = 0; u < TW; ++u) {
        const int t = wave + kMultiWaves * u;
        const bool live = t < T;
        const int k1 = live ? t / CT : 0;
        const int cc = (live ? t - (t / CT) * CT : 0) * 16 + (lane & 15);
        ok1[u] = k1;
        ok2[u] = cc < NP2 ? cc / NP : NP;
        ok3[u] = cc < NP2 ? cc - (cc / NP) * NP : NP;
        acc[u] = d4v{0.0, 0.0, 0.0, 0.0};
        acc32[u] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
    }
    const int m = lane & 15;
    const int jl = lane >> 4;
    const int js = tid & (kMultiTile - 1);          // this thread's source of a round
    const int role = tid / kMultiTile;              // 0, 1, 2: x, y, z factors; 3: charges

    for (int64_t t0 = 0; t0 < count; t0 += kMultiTile) {
        const int tn = static_cast<int>(count - t0 < kMultiTile ? count - t0 : kMultiTile);
        {
            // rows and charges past the chunk's end are zero
            const bool on = js < tn;
            const int64_t j = begin + t0 + (on ? js : 0);
            if (role < 3) {
                const double4 p = src[j];
                const double yv = role == 0 ? p.x : role == 1 ? p.y : p.z;
                double a[NP];
                bool tiny;
                const double D = factors_np<NP>(yv, sn + role * NP, a, tiny);
                const double f = on ? 1.0 : 0.0;
                if (tiny) {
                    one_hot_row<NP>(yv, sn + role * NP, f, a);
                } else {
                    const double g = f / D;
#pragma unroll
                    for (int k = 0; k < NP; ++k)
                        a[k] *= g;
                }
                R* __restrict__ row = (role == 0 ? L1 : role == 1 ? L2 : L3) + js * SP;
#pragma unroll
                for (int k = 0; k < NP; ++k)
                    row[k] = static_cast<R>(a[k]);
                row[NP] = R(0);
            } else {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    R qv;
                    if constexpr (F32)
                        qv = on ? qm32[j * 16 + v] : 0.0f;
                    else
                        qv = on ? qm[j * 16 + v] : 0.0;
                    SQ[js * 16 + v] = qv;
                }
            }
        }
        __syncthreads();
        const int steps = (tn + 3) / 4;
        for (int st = 0; st < steps; ++st) {
            const int j = 4 * st + jl;
            const R qv = SQ[j * 16 + m];
            const int jb = j * SP;
#pragma unroll
            for (int u = 0; u < TW; ++u) {
                if (wave + kMultiWaves * u >= T)   // uniform: past this wave's last tile
                    continue;
                const R av = L1[jb + ok1[u]] * qv;
                const R bv = L2[jb + ok2[u]] * L3[jb + ok3[u]];
                if constexpr (F32)
                    acc32[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc32[u], 0, 0, 0);
                else
                    acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
            }
        }
        if constexpr (F32) {
#pragma unroll
            for (int u = 0; u < TW; ++u) {
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[u][r] += static_cast<double>(acc32[u][r]);
                acc32[u] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
            }
        }
        __syncthreads();
    }

    // lane l, register r: row m = 4r + l/16 (f64) or 4 (l/16) + r (f32), column l % 16
    double* __restrict__ dst = out + chunk_dst[c] * static_cast<int64_t>(NP2) * NP * 16;
#pragma unroll
    for (int u = 0; u < TW; ++u) {
        if (wave + kMultiWaves * u >= T || ok2[u] == NP)
            continue;
        const int64_t kb = static_cast<int64_t>((ok1[u] * NP + ok2[u]) * NP + ok3[u]) * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int mo = F32 ? 4 * (lane >> 4) + r : 4 * r + (lane >> 4);
            dst[kb + mo] = acc[u][r];
        }
    }
}

template <int NP, bool F32>
__global__ __launch_bounds__(64 * kMultiWaves) void upward_multi(
    const double4* __restrict__ src, const double* __restrict__ qm, const float* __restrict__ qm32,
    const int32_t* __restrict__ chunk_slot, const int64_t* __restrict__ chunk_begin,
    const int64_t* __restrict__ chunk_count, const int64_t* __restrict__ chunk_dst,
    const double* __restrict__ slot_nodes, double* __restrict__ out)
{
    __shared__ double lds[kMultiLds];
    multi_chunk<NP, F32>(src, qm, qm32, chunk_slot, chunk_begin, chunk_count, chunk_dst,
                         slot_nodes, out, blockIdx.x, lds);
}

// the chunks of many systems (all of degree NP - 1) in one launch
template <int NP, bool F32>
__global__ __launch_bounds__(64 * kMultiWaves) void upward_multi_many(
    const UpwardDesc* __restrict__ descs, const int2* __restrict__ units)
{
    __shared__ double lds[kMultiLds];
    const int2 w = units[blockIdx.x];
    const UpwardDesc& d = descs[__builtin_amdgcn_readfirstlane(w.x)];
    multi_chunk<NP, F32>(d.src, d.qm, d.qm32, d.chunk_slot, d.chunk_begin, d.chunk_count,
                         d.chunk_dst, d.slot_nodes, d.buf, __builtin_amdgcn_readfirstlane(w.y),
                         lds);
}

#define BLTC_MULTI_NP(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9)

// 16-vector Lagrange upward pass of one plan (n + 1 <= 9); false for other degrees
bool launch_multi(const DevicePlan& d, double* buf, bool f32, hipStream_t s, hipError_t* err)
{
    switch (d.degree + 1) {
#define X(np)                                                                                  \
    case np:                                                                                   \
        if (f32)                                                                               \
            hipLaunchKernelGGL((upward_multi<np, true>), dim3(static_cast<unsigned>(d.nchunks)), \
                               dim3(64 * kMultiWaves), 0, s, d.src, d.qm, d.qm32, d.chunk_slot, d.chunk_begin, \
                               d.chunk_count, d.chunk_dst, d.slot_nodes, buf);                 \
        else                                                                                   \
            hipLaunchKernelGGL((upward_multi<np, false>), dim3(static_cast<unsigned>(d.nchunks)), \
                               dim3(64 * kMultiWaves), 0, s, d.src, d.qm, d.qm32, d.chunk_slot, d.chunk_begin, \
                               d.chunk_count, d.chunk_dst, d.slot_nodes, buf);                 \
        *err = hipGetLastError();                                                              \
        return true;
        BLTC_MULTI_NP(X)
#undef X
    default:
        return false;
    }
}

__global__ __launch_bounds__(256) void upward_mfma_f64(
    const double4* __restrict__ src, const double* __restrict__ qm, int32_t mw,
    const int32_t* __restrict__ chunk_slot, const int64_t* __restrict__ chunk_begin,
    const int64_t* __restrict__ chunk_count, const int64_t* __restrict__ chunk_dst,
    const double* __restrict__ slot_nodes, int32_t np, int32_t nf, double* __restrict__ out)
{
    extern __shared__ double lds[];
    upward_chunk(src, qm, mw, chunk_slot, chunk_begin, chunk_count, chunk_dst, slot_nodes, np, nf,
                 out, blockIdx.x, blockIdx.y, lds);
}

// the chunks of many systems in one launch: unit = (system, chunk)
__global__ __launch_bounds__(256) void upward_mfma_f64_many(const UpwardDesc* __restrict__ descs,
                                                            const int2* __restrict__ units,
                                                            int32_t mw)
{
    extern __shared__ double lds[];
    const int2 w = units[blockIdx.x];
    const UpwardDesc& d = descs[__builtin_amdgcn_readfirstlane(w.x)];
    const int32_t np2 = d.np * d.np;
    const int32_t tiles = ((d.np * mw + 15) / 16) * ((np2 + 15) / 16);
    if (static_cast<int32_t>(blockIdx.y) * kTilesPerGroup >= tiles)
        return;  // this system needs fewer tile passes (uniform over the workgroup)
    upward_chunk(d.src, d.qm, mw, d.chunk_slot, d.chunk_begin, d.chunk_count, d.chunk_dst,
                 d.slot_nodes, d.np, d.np, d.buf, __builtin_amdgcn_readfirstlane(w.y), blockIdx.y,
                 lds);
}

// qhat (and its FP32 copy) of every slot: the chunk result already in place
// for single-chunk clusters, else the sum of the partials in chunk order
__global__ __launch_bounds__(256) void upward_mfma_reduce(
    const int32_t* __restrict__ slot_chunk_off, const int64_t* __restrict__ chunk_dst,
    double* __restrict__ buf, float* __restrict__ qhat32, int64_t nslots, int64_t per_slot)
{
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= nslots * per_slot)
        return;
    const int64_t slot = idx / per_slot;
    const int64_t k = idx - slot * per_slot;
    const int32_t c0 = slot_chunk_off[slot], c1 = slot_chunk_off[slot + 1];
    double s;
    if (c1 - c0 == 1) {
        s = buf[idx];
    } else {
        s = 0.0;
        for (int32_t c = c0; c < c1; ++c)
            s += buf[chunk_dst[c] * per_slot + k];
        buf[idx] = s;
    }
    if (qhat32)
        qhat32[idx] = static_cast<float>(s);
}

// Hermite modified charges of every slot (and their FP32 copy), regrouped per
// grid point:
// qh[slot][k][a] (k = (k1 (n+1) + k2) (n+1) + k3, a = 4 a1 + 2 a2 + a3) is the
// sum over the slot's chunks, in chunk order, of the blocked chunk result
// buf[row][((a1 np + k1) nf + a2 np + k2) nf + a3 np + k3], nf = 2 np.  The
// eight values of one grid point are then one 64-byte wave-uniform load.
__global__ __launch_bounds__(256) void upward_reduce_hermite(
    const int32_t* __restrict__ slot_chunk_off, const int64_t* __restrict__ chunk_dst,
    const double* __restrict__ buf, double* __restrict__ qh, float* __restrict__ qh32,
    int64_t nslots, int32_t np)
{
    const int64_t P = static_cast<int64_t>(np) * np * np;
    const int64_t per_slot = 8 * P;
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= nslots * per_slot)
        return;
    const int64_t slot = idx / per_slot;
    const int64_t r = idx - slot * per_slot;
    const int32_t k = static_cast<int32_t>(r >> 3), a = static_cast<int32_t>(r & 7);
    const int32_t k1 = k / (np * np), k2 = (k / np) % np, k3 = k % np;
    const int32_t nf = 2 * np;
    const int64_t kb = ((((a >> 2) * np + k1) * nf + ((a >> 1) & 1) * np + k2) * nf) +
                       (a & 1) * np + k3;
    const int32_t c0 = slot_chunk_off[slot], c1 = slot_chunk_off[slot + 1];
    double s = 0.0;
    for (int32_t c = c0; c < c1; ++c)
        s += buf[chunk_dst[c] * per_slot + kb];
    qh[idx] = s;
    if (qh32)
        qh32[idx] = static_cast<float>(s);
}

}  // namespace

size_t upward_lds_bytes(int32_t np, int32_t mw, int32_t nf)
{
    return sizeof(double) *
           (static_cast<size_t>(3) * kTile * nf + static_cast<size_t>(kTile) * mw + 6 * np);
}

int32_t upward_passes(int32_t nf, int32_t mw)
{
    const int32_t T = ((nf * mw + 15) / 16) * ((nf * nf + 15) / 16);
    return (T + kTilesPerGroup - 1) / kTilesPerGroup;
}

hipError_t upward_prepare(size_t lds)
{
    if (lds <= 65536)
        return hipSuccess;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(upward_mfma_f64),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(lds));
    if (e != hipSuccess)
        return e;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(upward_mfma_f64_many),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
}

hipError_t launch_upward_reduce(const DevicePlan& d, int32_t mw, double* buf, float* qhat32,
                                hipStream_t s)
{
    const int32_t nf = d.hermite ? 2 * (d.degree + 1) : d.degree + 1;
    const int64_t per_slot = static_cast<int64_t>(nf) * nf * nf * mw;
    const int64_t total = d.nslots * per_slot;
    if (total == 0)
        return hipSuccess;
    if (d.hermite) {
        if (mw != 1 || !d.qhat_h)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(upward_reduce_hermite, dim3(static_cast<unsigned>((total + 255) / 256)),
                           dim3(256), 0, s, d.slot_chunk_off, d.chunk_dst, buf, d.qhat_h, qhat32,
                           d.nslots, d.degree + 1);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(upward_mfma_reduce, dim3(static_cast<unsigned>((total + 255) / 256)),
                       dim3(256), 0, s, d.slot_chunk_off, d.chunk_dst, buf, qhat32, d.nslots,
                       per_slot);
    return hipGetLastError();
}

hipError_t launch_upward_mfma(const DevicePlan& d, int32_t mw, double* buf, float* qhat32,
                              hipStream_t s)
{
    if (d.nchunks == 0)
        return hipSuccess;
    hipError_t e = hipSuccess;
    if (mw == 1 && launch_single(d, buf, s, &e)) {
        if (e != hipSuccess)
            return e;
        return launch_upward_reduce(d, mw, buf, qhat32, s);
    }
    if (mw == 16 && !d.hermite && launch_multi(d, buf, d.src32 != nullptr, s, &e)) {
        if (e != hipSuccess)
            return e;
        return launch_upward_reduce(d, mw, buf, qhat32, s);
    }
    const int32_t np = d.degree + 1;
    const int32_t nf = d.hermite ? 2 * np : np;
    const size_t lds = upward_lds_bytes(np, mw, nf);
    e = upward_prepare(lds);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(upward_mfma_f64, dim3(static_cast<unsigned>(d.nchunks), upward_passes(nf, mw)),
                       dim3(256), lds, s, d.src, d.qm, mw, d.chunk_slot, d.chunk_begin,
                       d.chunk_count, d.chunk_dst, d.slot_nodes, np, nf, buf);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_upward_reduce(d, mw, buf, qhat32, s);
}

bool upward_many_multi(int32_t np, int32_t mw)
{
    return mw == 16 && np >= 2 && np <= kMultiMaxNP;
}

hipError_t launch_upward_many_multi(const UpwardDesc* descs, const int2* units, int32_t nunits,
                                    int32_t np, bool f32, hipStream_t s)
{
    if (nunits == 0)
        return hipSuccess;
    switch (np) {
#define X(n)                                                                                   \
    case n:                                                                                    \
        if (f32)                                                                               \
            hipLaunchKernelGGL((upward_multi_many<n, true>), dim3(static_cast<unsigned>(nunits)), \
                               dim3(64 * kMultiWaves), 0, s, descs, units);                                 \
        else                                                                                   \
            hipLaunchKernelGGL((upward_multi_many<n, false>), dim3(static_cast<unsigned>(nunits)), \
                               dim3(64 * kMultiWaves), 0, s, descs, units);                                 \
        return hipGetLastError();
        BLTC_MULTI_NP(X)
#undef X
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_upward_many(const UpwardDesc* descs, const int2* units, int32_t nunits,
                              int32_t mw, int32_t passes, size_t lds, hipStream_t s)
{
    if (nunits == 0)
        return hipSuccess;
    hipLaunchKernelGGL(upward_mfma_f64_many, dim3(static_cast<unsigned>(nunits), passes), dim3(256),
                       lds, s, descs, units, mw);
    return hipGetLastError();
}

}  // namespace bltc
