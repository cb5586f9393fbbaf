// microbench.hip -- instruction-cost probes behind the issue-rate model of the
// interaction kernels (a standalone program, not part of libbltc.so).
//
//  1. SIMD-cycles per wave instruction for the VALU operations the kernels
//     use: 8 independent chains per lane, 16 waves per SIMD, timed with HIP
//     events and priced at the nominal 2.4 GHz (a counter run of this program
//     gives each dispatch's clock, hence its core cycles).
//  2. Relative error of the v_rsq_f64 / v_rsq_f32 estimates and of one FP64
//     Newton step, against 1/sqrtl on the host, over 2^22 arguments spread
//     log-uniformly over 2^-20 .. 2^20.
//  3. Whether matrix-core (MFMA) and VALU work overlap: waves running only
//     v_mfma_f32_16x16x4f32, only FP32 FMAs, half of the waves each (twice the
//     work each), and both interleaved in every wave.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

namespace {

constexpr int kChains = 8;
constexpr double kClockHz = 2.4e9;
constexpr int kSimds = 1024;

#define CHECK(call)                                                                   \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            std::fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));           \
            std::exit(1);                                                             \
        }                                                                             \
    } while (0)

// ---------------------------------------------------------------------------
// 1. issue costs
// ---------------------------------------------------------------------------
template <int OP>
__global__ __launch_bounds__(256) void chains(double* out, int iters, double seed)
{
    double a[kChains];
    float f[kChains];
    for (int c = 0; c < kChains; ++c) {
        a[c] = seed + 0.001 * c + 1e-9 * threadIdx.x;
        f[c] = static_cast<float>(a[c]);
    }
    const double b = 0.9999999, cc = 1e-7;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if constexpr (OP == 0) a[c] = __fma_rn(a[c], b, cc);
            if constexpr (OP == 1) a[c] = a[c] * b;
            if constexpr (OP == 2) a[c] = a[c] + cc;
            if constexpr (OP == 3) a[c] = __builtin_amdgcn_rsq(a[c]);
            if constexpr (OP == 4) f[c] = __fmaf_rn(f[c], 0.9999f, 1e-4f);
            if constexpr (OP == 5) f[c] = __builtin_amdgcn_rsqf(f[c]);
            if constexpr (OP == 6) f[c] = __builtin_amdgcn_exp2f(-f[c]);
        }
    }
    double s = 0;
    for (int c = 0; c < kChains; ++c)
        s += a[c] + f[c];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <int OP>
float time_chains(double* out, int blocks, int iters)
{
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(chains<OP>, dim3(blocks), dim3(256), 0, 0, out, iters, 1.3);
    CHECK(hipEventRecord(e0));
    hipLaunchKernelGGL(chains<OP>, dim3(blocks), dim3(256), 0, 0, out, iters, 1.3);
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return ms;
}

void issue_costs()
{
    const int blocks = kSimds * 4;   // 4 waves per block: 16 waves per SIMD
    const int iters = 2048;
    double* out = nullptr;
    CHECK(hipMalloc(&out, sizeof(double) * blocks * 256));
    const char* names[] = {"v_fma_f64", "v_mul_f64", "v_add_f64", "v_rsq_f64",
                           "v_fma_f32", "v_rsq_f32", "v_exp_f32"};
    float ms[7];
    ms[0] = time_chains<0>(out, blocks, iters);
    ms[1] = time_chains<1>(out, blocks, iters);
    ms[2] = time_chains<2>(out, blocks, iters);
    ms[3] = time_chains<3>(out, blocks, iters);
    ms[4] = time_chains<4>(out, blocks, iters);
    ms[5] = time_chains<5>(out, blocks, iters);
    ms[6] = time_chains<6>(out, blocks, iters);
    const double wave_insts_per_simd = blocks * 4.0 * iters * kChains / kSimds;
    std::printf("# issue cost: SIMD-cycles per wave instruction at the nominal %.1f GHz (times the\n"
                "# clock a counter run reports for the dispatch over 2.4 GHz gives core cycles)\n",
                kClockHz * 1e-9);
    for (int i = 0; i < 7; ++i)
        std::printf("cycles %-10s nominal %6.2f (%.3f ms)\n", names[i],
                    ms[i] * 1e-3 * kClockHz / wave_insts_per_simd, ms[i]);
    CHECK(hipFree(out));
}

// ---------------------------------------------------------------------------
// 2. reciprocal square root estimates
// ---------------------------------------------------------------------------
__global__ void rsq_estimates(const double* x, double* y64, double* yn, double* y32, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const double r2 = x[i];
    const double y = __builtin_amdgcn_rsq(r2);
    y64[i] = y;
    yn[i] = 0.5 * (y * __fma_rn(-(r2 * y), y, 3.0));
    y32[i] = __builtin_amdgcn_rsqf(static_cast<float>(r2));
}

void rsq_accuracy()
{
    const int n = 1 << 22;
    std::vector<double> x(n);
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> u(-20.0, 20.0);
    for (int i = 0; i < n; ++i)
        x[i] = std::exp2(u(g));
    double *dx, *a, *b, *c;
    CHECK(hipMalloc(&dx, n * sizeof(double)));
    CHECK(hipMalloc(&a, n * sizeof(double)));
    CHECK(hipMalloc(&b, n * sizeof(double)));
    CHECK(hipMalloc(&c, n * sizeof(double)));
    CHECK(hipMemcpy(dx, x.data(), n * sizeof(double), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(rsq_estimates, dim3(n / 256), dim3(256), 0, 0, dx, a, b, c, n);
    CHECK(hipDeviceSynchronize());
    std::vector<double> A(n), B(n), C(n);
    CHECK(hipMemcpy(A.data(), a, n * sizeof(double), hipMemcpyDeviceToHost));
    CHECK(hipMemcpy(B.data(), b, n * sizeof(double), hipMemcpyDeviceToHost));
    CHECK(hipMemcpy(C.data(), c, n * sizeof(double), hipMemcpyDeviceToHost));
    double ea = 0, eb = 0, ec = 0, mb = 0;
    for (int i = 0; i < n; ++i) {
        const long double t = 1.0L / sqrtl(static_cast<long double>(x[i]));
        const double ra = static_cast<double>((A[i] - t) / t);
        const double rb = static_cast<double>((B[i] - t) / t);
        const double rc = static_cast<double>((C[i] - t) / t);
        ea = std::fmax(ea, std::fabs(ra));
        eb = std::fmax(eb, std::fabs(rb));
        ec = std::fmax(ec, std::fabs(rc));
        mb += rb;
    }
    std::printf("# relative error of 1/sqrt over %d arguments in [2^-20, 2^20]\n", n);
    std::printf("rsq_f64_estimate max %.3e\n", ea);
    std::printf("rsq_f64_newton   max %.3e mean %.3e\n", eb, mb / n);
    std::printf("rsq_f32_estimate max %.3e\n", ec);
    CHECK(hipFree(dx));
    CHECK(hipFree(a));
    CHECK(hipFree(b));
    CHECK(hipFree(c));
}

// ---------------------------------------------------------------------------
// 3. MFMA and VALU overlap
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float mfma_work(int iters)
{
    v4f c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
    const float a = 1.0f + threadIdx.x * 1e-6f, b = 0.5f;
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c3, 0, 0, 0);
    }
    return c0[0] + c1[1] + c2[2] + c3[3];
}

__device__ __forceinline__ float valu_work(int iters)
{
    float f[kChains];
    for (int c = 0; c < kChains; ++c)
        f[c] = 1.0f + c * 1e-3f + threadIdx.x * 1e-7f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c)
            f[c] = __fmaf_rn(f[c], 0.9999f, 1e-4f);
    }
    float s = 0;
    for (int c = 0; c < kChains; ++c)
        s += f[c];
    return s;
}

// mode 0: every wave MFMA; 1: every wave VALU; 2: even waves MFMA, odd VALU;
// 3: waves 0-3 MFMA, 4-7 VALU (workgroups of 8 waves)
__global__ __launch_bounds__(512) void split_waves(float* out, int mode, int mi, int vi)
{
    const int w = threadIdx.x / 64;
    const bool mf = mode == 0 || (mode == 2 && (w % 2) == 0) || (mode == 3 && w < 4);
    out[blockIdx.x * blockDim.x + threadIdx.x] = mf ? mfma_work(mi) : valu_work(vi);
}

// every wave: per step 4 MFMAs, then k x 8 independent FP32 FMAs
__global__ __launch_bounds__(512) void interleaved(float* out, int iters, int k)
{
    v4f c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
    const float a = 1.0f + threadIdx.x * 1e-6f, b = 0.5f;
    float f[kChains];
    for (int c = 0; c < kChains; ++c)
        f[c] = 1.0f + c * 1e-3f + threadIdx.x * 1e-7f;
    for (int i = 0; i < iters; ++i) {
        c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
        c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c1, 0, 0, 0);
        c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c2, 0, 0, 0);
        c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c3, 0, 0, 0);
        for (int j = 0; j < k; ++j) {
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                f[c] = __fmaf_rn(f[c], 0.9999f, 1e-4f);
        }
    }
    float s = c0[0] + c1[1] + c2[2] + c3[3];
    for (int c = 0; c < kChains; ++c)
        s += f[c];
    out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

void mfma_valu_overlap()
{
    const int blocks = 256 * 2;   // two workgroups of 8 waves per CU: 4 waves per SIMD
    float* out = nullptr;
    CHECK(hipMalloc(&out, sizeof(float) * blocks * 512));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    auto timed = [&](auto launch) {
        launch();
        CHECK(hipEventRecord(e0));
        launch();
        CHECK(hipEventRecord(e1));
        CHECK(hipEventSynchronize(e1));
        float ms = 0;
        CHECK(hipEventElapsedTime(&ms, e0, e1));
        return ms;
    };
    const int mi = 4096, vi = 4096;
    auto split = [&](int mode, int m_it, int v_it) {
        return timed([&] {
            hipLaunchKernelGGL(split_waves, dim3(blocks), dim3(512), 0, 0, out, mode, m_it, v_it);
        });
    };
    const float t_m = split(0, mi, vi), t_v = split(1, mi, vi);
    const float t_2 = split(2, 2 * mi, 2 * vi), t_3 = split(3, 2 * mi, 2 * vi);
    std::printf("# MFMA and VALU overlap (4 waves per SIMD)\n");
    std::printf("mfma_only_ms %.3f\nvalu_only_ms %.3f\n", t_m, t_v);
    std::printf("split_even_odd_ms %.3f (serial %.3f, overlapped %.3f)\n", t_2, t_m + t_v,
                t_m > t_v ? t_m : t_v);
    std::printf("split_halves_ms %.3f\n", t_3);
    for (int k : {0, 2, 4, 8}) {
        const float t = timed([&] {
            hipLaunchKernelGGL(interleaved, dim3(blocks), dim3(512), 0, 0, out, mi, k);
        });
        std::printf("interleaved_k%d_ms %.3f (4 MFMA + %d x 8 FMA per step)\n", k, t, k);
    }
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    CHECK(hipFree(out));
}

}  // namespace

int main()
{
    issue_costs();
    rsq_accuracy();
    mfma_valu_overlap();
    return 0;
}
