// autotune.cpp -- the library's own tuner for the leaf size N_L and batch
// size N_B (kept equal, as in the paper's runs) and the threads per target,
// C ABI bltc_autotune.
//
// For a given geometry the tuner builds a plan for each candidate size, times
// one evaluation of each on the GPU (HIP events on the caller's stream, after
// one warm-up), and keeps the fastest; for one-vector BLTC and Hermite plans
// whose threads per target are left to it (0) it then times 2 and 4 lanes
// per target at that size and keeps the fastest of 1, 2, 4.  Choices are
// cached in a text file keyed by the problem class (method, log2 of the
// particle counts, theta, degree, kernel and its parameter, precision, one or
// several charge vectors), so later calls with a
// similar problem skip the search.  The accuracy of the treecode is set by
// theta and n; the leaf size changes which pairs are approximated and hence
// the error slightly, never the bound the MAC enforces.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <fstream>
#include <new>
#include <sstream>
#include <string>

#include "internal.hpp"

using bltc_detail::fail;

namespace {

std::string cache_path()
{
    const char* env = std::getenv("BLTC_TUNE_CACHE");
    if (env && *env)
        return env;
    const char* home = std::getenv("HOME");
    return std::string(home && *home ? home : "/tmp") + "/.bltc_tune_cache";
}

std::string class_key(const bltc_params* p, int64_t nt, int64_t ns, int32_t num_q)
{
    std::ostringstream k;
    k << "v2 nt2=" << (nt > 0 ? static_cast<int>(std::lround(std::log2(static_cast<double>(nt)))) : 0)
      << " ns2=" << (ns > 0 ? static_cast<int>(std::lround(std::log2(static_cast<double>(ns)))) : 0)
      << " theta=" << p->theta << " n=" << p->degree << " kernel=" << p->kernel
      << " prec=" << p->precision << " q=" << (num_q > 1 ? 16 : 1) << " method=" << p->method
      << " delta=" << p->delta << " kappa=" << p->kappa;
    return k.str();
}

bool cache_lookup(const std::string& key, int32_t* leaf, int32_t* tpt, double* ms)
{
    std::ifstream f(cache_path());
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        const size_t bar = line.rfind('|');
        if (bar == std::string::npos || line.substr(0, bar) != key)
            continue;
        std::istringstream v(line.substr(bar + 1));
        int32_t l = 0, tp = 0;
        double t = 0.0;
        if (v >> l >> t >> tp && l > 0 && (tp == 1 || tp == 2 || tp == 4)) {
            *leaf = l;
            *tpt = tp;
            *ms = t;
            found = true;   // the last entry of a key wins
        }
    }
    return found;
}

void cache_store(const std::string& key, int32_t leaf, int32_t tpt, double ms)
{
    std::ofstream f(cache_path(), std::ios::app);
    if (f) {
        f.precision(17);
        f << key << "|" << leaf << " " << ms << " " << tpt << "\n";
    }
}

}  // namespace

namespace {

// ncand = 0: the sizes of *p are kept and only the threads per target are
// searched (the caller checked that they are open and searchable)
int autotune_impl(const bltc_params* p, int64_t nt, const double* tx, const double* ty,
                  const double* tz, int64_t ns, const double* sx, const double* sy,
                  const double* sz, int32_t num_q, const int32_t* candidates, int32_t ncand,
                  int32_t use_cache, bltc_params* out, double* best_ms, void* stream)
{
    *out = *p;
    if (best_ms)
        *best_ms = 0.0;
    if (nt == 0 || ns == 0)
        return BLTC_OK;
    const bool fixed = ncand == 0;
    const int32_t fixed_size = p->leaf_size;
    if (fixed) {
        candidates = &fixed_size;
        ncand = 1;
    }
    // threads per target: searched for one-vector BLTC plans that leave it open
    const bool tune_tpt = p->threads_per_target == 0 && num_q == 1 &&
                          (p->method == BLTC_PARTICLE_CLUSTER || p->method == BLTC_HERMITE);
    std::string key = class_key(p, nt, ns, num_q) + " tpt=" +
                      std::to_string(tune_tpt ? 0 : std::max(1, p->threads_per_target));
    if (fixed)
        key += " sizes=" + std::to_string(p->leaf_size) + "," + std::to_string(p->batch_size);
    int32_t cached = 0, cached_tpt = 1;
    double cached_ms = 0.0;
    if (use_cache && cache_lookup(key, &cached, &cached_tpt, &cached_ms)) {
        if (!fixed) {
            out->leaf_size = cached;
            out->batch_size = cached;
        }
        if (tune_tpt)
            out->threads_per_target = cached_tpt;
        if (best_ms)
            *best_ms = cached_ms;
        return BLTC_OK;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // charges: ones (the timing does not depend on the values)
    double* q = nullptr;
    double* phi = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = BLTC_OK;
    int32_t best = -1, best_tpt = 1;
    double best_t = 0.0;
    std::vector<double> ones(static_cast<size_t>(ns) * num_q, 1.0);
    do {
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&q), ones.size() * sizeof(double));
        if (e == hipSuccess)
            e = hipMalloc(reinterpret_cast<void**>(&phi), static_cast<size_t>(nt) * num_q * sizeof(double));
        if (e == hipSuccess)
            e = hipMemcpyAsync(q, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipEventCreate(&e0);
        if (e == hipSuccess)
            e = hipEventCreate(&e1);
        if (e != hipSuccess) {
            rc = bltc_detail::hip_fail(e, "autotune setup");
            break;
        }
        // candidate sizes at the caller's threads per target, then (tune_tpt)
        // 2 and 4 lanes per target at the best size
        const int32_t nsteps = ncand + (tune_tpt ? 2 : 0);
        for (int32_t c = 0; c < nsteps && rc == BLTC_OK; ++c) {
            bltc_params trial = *p;
            const int32_t leaf = c < ncand ? candidates[c] : best;
            const int32_t tpt = c < ncand ? std::max(1, p->threads_per_target) : (c == ncand ? 2 : 4);
            if (!fixed) {
                trial.leaf_size = leaf;
                trial.batch_size = leaf;
            }
            trial.threads_per_target = tpt;
            bltc_plan* plan = nullptr;
            rc = bltc_plan_create(&plan, &trial, nt, tx, ty, tz, ns, sx, sy, sz,
                                  num_q > 1 ? 16 : 1, stream);
            if (rc != BLTC_OK)
                break;
            rc = bltc_plan_execute(plan, q, num_q, ns, phi, nt, stream);   // warm-up
            float ms = 0.0f;
            if (rc == BLTC_OK) {
                e = hipEventRecord(e0, s);
                if (e == hipSuccess)
                    rc = bltc_plan_execute(plan, q, num_q, ns, phi, nt, stream);
                if (e == hipSuccess && rc == BLTC_OK)
                    e = hipEventRecord(e1, s);
                if (e == hipSuccess && rc == BLTC_OK)
                    e = hipEventSynchronize(e1);
                if (e == hipSuccess && rc == BLTC_OK)
                    e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess)
                    rc = bltc_detail::hip_fail(e, "autotune timing");
            }
            bltc_plan_destroy(plan);
            if (rc == BLTC_OK && (best < 0 || ms < best_t)) {
                best = leaf;
                best_tpt = std::max(1, tpt);
                best_t = ms;
            }
        }
    } while (false);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (q)
        (void)hipFree(q);
    if (phi)
        (void)hipFree(phi);
    if (rc != BLTC_OK)
        return rc;
    if (!fixed) {
        out->leaf_size = best;
        out->batch_size = best;
    }
    if (tune_tpt)
        out->threads_per_target = best_tpt;
    if (best_ms)
        *best_ms = best_t;
    if (use_cache)
        cache_store(key, best, best_tpt, best_t);
    return BLTC_OK;
}

}  // namespace

extern "C" int bltc_autotune(const bltc_params* p, int64_t nt, const double* tx,
                             const double* ty, const double* tz, int64_t ns, const double* sx,
                             const double* sy, const double* sz, int32_t num_q,
                             const int32_t* candidates, int32_t ncand, int32_t use_cache,
                             bltc_params* out, double* best_ms, void* stream)
{
    if (!p || !out)
        return fail(BLTC_EINVAL, "NULL argument");
    if (!candidates || ncand < 1)
        return fail(BLTC_EINVAL, "at least one candidate size is needed");
    if (num_q < 1 || num_q > 16)
        return fail(BLTC_EINVAL, "num_q must be in 1..16");
    for (int32_t c = 0; c < ncand; ++c)
        if (candidates[c] < 1)
            return fail(BLTC_EINVAL, "candidate sizes must be >= 1");
    try {
        return autotune_impl(p, nt, tx, ty, tz, ns, sx, sy, sz, num_q, candidates, ncand,
                             use_cache, out, best_ms, stream);
    } catch (const std::bad_alloc&) {
        return fail(BLTC_ENOMEM, "host allocation failed while tuning");
    } catch (const std::exception& ex) {
        return fail(BLTC_EINTERNAL, "tuning failed: %s", ex.what());
    }
}

int bltc_internal_tune(const bltc_params* p, int64_t nt, const double* tx, const double* ty,
                       const double* tz, int64_t ns, const double* sx, const double* sy,
                       const double* sz, int32_t max_q, bltc_params* out, void* stream)
{
    static const int32_t kSizes[] = {1000, 2000, 3000, 4000};
    const int32_t num_q = max_q > 1 ? 16 : 1;
    const bool tpt_open = p->threads_per_target == 0 && max_q == 1 &&
                          (p->method == BLTC_PARTICLE_CLUSTER || p->method == BLTC_HERMITE);
    *out = *p;
    if (p->leaf_size == 0)
        return autotune_impl(p, nt, tx, ty, tz, ns, sx, sy, sz, num_q, kSizes, 4, 1, out,
                             nullptr, stream);
    if (tpt_open)
        return autotune_impl(p, nt, tx, ty, tz, ns, sx, sy, sz, num_q, nullptr, 0, 1, out,
                             nullptr, stream);
    return BLTC_OK;
}
