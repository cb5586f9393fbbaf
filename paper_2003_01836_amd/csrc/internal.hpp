// internal.hpp -- definitions shared by the C-ABI sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "bltc.h"
#include "kernels.hpp"
#include "planner.hpp"

namespace bltc_detail {

inline std::string& last_error()
{
    static thread_local std::string msg;
    return msg;
}

inline int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    last_error() = buf;
    return code;
}

// why the last allocation of the calling thread failed, when a plan's
// workspace limit refused it (empty otherwise)
inline std::string& limit_note()
{
    static thread_local std::string msg;
    return msg;
}

// A failed HIP call: BLTC_ENOMEM for allocations (the device's or a plan's
// workspace limit), BLTC_EHIP otherwise.
inline int hip_fail(hipError_t e, const char* what)
{
    if (e == hipErrorOutOfMemory) {
        std::string note;
        note.swap(limit_note());
        return fail(BLTC_ENOMEM, "%s: %s", what,
                    note.empty() ? "out of device memory" : note.c_str());
    }
    return fail(BLTC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

// device copy of a host vector (memory not owned by a plan)
template <class T>
hipError_t upload(T** dst, const std::vector<T>& v, hipStream_t s)
{
    const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), bytes);
    if (e != hipSuccess)
        return e;
    if (!v.empty())
        e = hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
    return e;
}

}  // namespace bltc_detail

// Device memory for the results of mutual leaf pairs when the whole result
// array does not fit: at most this many bytes per round (a plan's
// workspace_limit can lower it).  Pairs whose results alone exceed a quarter
// of it stay in the plain direct lists.
constexpr int64_t kPairWorkspaceBytes = int64_t(16) << 30;

#define HIP_TRY(call)                                              \
    do {                                                           \
        hipError_t e_ = (call);                                    \
        if (e_ != hipSuccess)                                      \
            return bltc_detail::hip_fail(e_, #call);               \
    } while (0)

struct bltc_plan {
    bltc_params prm{};
    int32_t max_q = 1;
    bltc::HostPlan hp;
    // true when the trees were built on the device: the per-particle arrays
    // (positions, orders, local coordinates) exist only in device memory
    bool device_particles = false;
    // true when the interaction lists were built on the device
    bool device_lists = false;
    int64_t n_items = 0;                 // interaction items (device lists)
    int32_t* item_batch = nullptr;       // device copies of the items (device lists)
    int32_t* item_cluster = nullptr;
    int32_t* item_kind = nullptr;
    // host copies for bltc_plan_view_get (device-built plans)
    mutable std::vector<int64_t> view_src_order, view_tgt_order;
    mutable std::vector<int32_t> view_item_batch, view_item_cluster, view_item_kind;
    mutable std::vector<double> view_batch_lo, view_batch_hi;
    // cluster-particle plans (method BLTC_CLUSTER_PARTICLE): host plan, the
    // proxy-potential and direct launches, interpolation lists, proxy potentials
    bool cp = false;
    bltc::CpPlan cpp;
    bltc::DevicePlan dprox, ddir;
    int32_t* cp_path_off = nullptr;
    int32_t* cp_path_slot = nullptr;
    double* cp_slot_nodes = nullptr;
    double* cp_phat = nullptr;
    // cluster-cluster plans (method BLTC_CLUSTER_CLUSTER): host plan; the
    // interaction launches, interpolation lists and proxy potentials use the
    // members above, the upward pass uses d
    bool cc = false;
    bltc::CcPlan ccp;
    bool uploaded = false;
    int device = -1;
    bltc::DevicePlan d;
    std::vector<void*> allocations;
    bool timing = false;
    int32_t last_q = 0;                  // charge vectors of the last execution
    int32_t timed_q = 0;                 // charge vectors covered by the recorded events
    int64_t sym_pair_evals = 0;          // kernel values of the mutual leaf pairs (each serving
                                         // two direct terms), once uploaded
    // threads per target > 1 (one charge vector, BLTC): each batch's lists cut
    // into tpt contiguous pieces, evaluated as separate batches over tpt
    // copies of the targets (view dt) into tpt_buf[piece][target], then summed
    // per target in piece order
    int32_t tpt = 1;
    bltc::DevicePlan dt;
    double* tpt_buf = nullptr;
    std::vector<int32_t> sym_near_off_h, sym_pc_off_h;   // host copies (mutual pairs)
    std::vector<hipEvent_t> events;      // 4 per charge vector
    hipEvent_t ev_pairs = nullptr;       // after the mutual-pair launch (timing)
    bool timed_pairs = false;            // ev_pairs belongs to the recorded execution
    // device memory the plan holds (requested bytes) and its limit (0: none)
    int64_t bytes = 0;
    int64_t limit = 0;
    // Mutual leaf pairs (d.sym): planned with the direct lists, their result
    // workspace and sub-units sized once the rest of the device side exists
    // (bltc_internal_finish_pairs), in one round when the whole result array
    // fits under the workspace cap, else in rounds folded into per-target sums.
    struct Pairs {
        bltc::DevicePlan* d = nullptr;   // the view whose direct lists hold the pairs
        bltc::SymPlan sp;                // every mutual pair taken
        std::vector<int64_t> batch_begin, batch_count;
        std::vector<int32_t> batch_node;
        bool pending = false;
        int64_t count = 0;               // mutual pairs evaluated once
        int32_t rounds = 0;
        int64_t workspace_bytes = 0;     // result workspace (and per-target sums)
        std::vector<int32_t> round_unit; // rounds + 1 sub-unit offsets
        int32_t* fold_off = nullptr;     // [rounds][batches + 1]
        int64_t* fold_base = nullptr;
        int64_t* batch_end = nullptr;    // device copy of begin + count per batch
    } pairs;

    ~bltc_plan()
    {
        for (hipEvent_t e : events)
            (void)hipEventDestroy(e);
        if (ev_pairs)
            (void)hipEventDestroy(ev_pairs);
        for (void* p : allocations)
            (void)hipFree(p);
    }

    // every device allocation of the plan: counted against its limit
    hipError_t alloc_bytes(void** dst, size_t bytes_wanted)
    {
        const size_t n = std::max<size_t>(1, bytes_wanted);
        if (limit > 0 && bytes + static_cast<int64_t>(n) > limit) {
            char buf[160];
            std::snprintf(buf, sizeof(buf),
                          "workspace_limit of %lld bytes reached (%lld held, %lld more needed)",
                          static_cast<long long>(limit), static_cast<long long>(bytes),
                          static_cast<long long>(n));
            bltc_detail::limit_note() = buf;
            return hipErrorOutOfMemory;
        }
        hipError_t e = hipMalloc(dst, n);
        if (e == hipSuccess) {
            allocations.push_back(*dst);
            bytes += static_cast<int64_t>(n);
        }
        return e;
    }

    template <class T>
    hipError_t put(T** dst, const std::vector<T>& v, hipStream_t s)
    {
        hipError_t e = alloc_bytes(reinterpret_cast<void**>(dst), v.size() * sizeof(T));
        if (e == hipSuccess && !v.empty())
            e = hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
        return e;
    }

    template <class T>
    hipError_t alloc(T** dst, size_t count)
    {
        return alloc_bytes(reinterpret_cast<void**>(dst), count * sizeof(T));
    }
};


// device side of a plan (uploads on first use); synchronises the stream
int bltc_internal_upload_plan(bltc_plan* plan, hipStream_t s);

// Mutual direct pairs of one-tree direct lists evaluated once (see
// plan_symmetric): plans them, uploads the reduced lists and the per-batch
// result offsets into d (d.sym = 1), lowers the lists' batch_cost in *cost to
// the work left to the batches, and leaves the result workspace and the
// sub-units to bltc_internal_finish_pairs.  Returns BLTC_OK and leaves d alone
// when no pair qualifies.  d must be a member of *plan (d or ddir).
int bltc_internal_upload_symmetric(bltc_plan* plan, bltc::DevicePlan& d,
                                   const bltc::DirectLists& dl, std::vector<int64_t>* cost,
                                   hipStream_t s);
// The result workspace of the planned mutual pairs, sized from what the
// plan's workspace limit leaves once every other device array exists: one
// round when all results fit (at most kPairWorkspaceBytes), else rounds.
// BLTC_ENOMEM when the limit leaves no room for the largest pair.
int bltc_internal_finish_pairs(bltc_plan* plan, hipStream_t s);
// Enqueues the mutual-pair launches of d (every round, each folded into the
// per-target sums when there are several).
int bltc_internal_pairs(bltc_plan* plan, const bltc::DevicePlan& d, const bltc::KernelParams& kp,
                        hipStream_t s);

// Parameters left to the tuner (leaf_size = batch_size = 0, or threads per
// target 0 for a one-vector BLTC or Hermite plan) filled in by timing plans
// on the device (autotune.cpp; results cached as bltc_autotune's).  *out = *p
// when nothing is open.
int bltc_internal_tune(const bltc_params* p, int64_t nt, const double* tx, const double* ty,
                       const double* tz, int64_t ns, const double* sx, const double* sy,
                       const double* sz, int32_t max_q, bltc_params* out, void* stream);

// BLTC_EUNSUPPORTED for an FP32-mixed plan whose points do not fit in a box of
// side kMixedMaxExtent (capi.cpp); BLTC_OK otherwise.
int bltc_internal_check_mixed_extent(const bltc_plan* plan);

// Argument checks of bltc_direct and bltc_direct_noalloc (capi.cpp).
int bltc_internal_check_direct(const bltc_params* p, int64_t nt, const double* tx,
                               const double* ty, const double* tz, int64_t ns, const double* sx,
                               const double* sy, const double* sz, const double* q, int32_t num_q,
                               const double* phi);

// cluster-particle plans (cp.cpp)
namespace bltc_cp {
int create_host(bltc_plan* plan, const bltc::PlanParams& pp, int64_t nt, const double* tx,
                const double* ty, const double* tz, int64_t ns, const double* sx, const double* sy,
                const double* sz);
int create_device(bltc_plan* plan, const bltc::PlanParams& pp, int64_t nt, const double* tx,
                  const double* ty, const double* tz, int64_t ns, const double* sx,
                  const double* sy, const double* sz, hipStream_t s);
int upload(bltc_plan* plan, hipStream_t s);
int execute(bltc_plan* plan, const double* q, int32_t num_q, double* phi, hipStream_t s);
int proxy_potentials(bltc_plan* plan, int64_t cluster, double* out, hipStream_t s);
void stats(const bltc_plan* plan, bltc_stats* out);
int view(const bltc_plan* plan, bltc_plan_view* out);
// Pieces of the proxy-potential lists off/count (one list per slot, entries
// = source ranges): runs of whole entries of one slot with at most
// max(8192, listed / 16384) sources, so that the heaviest clusters do not set
// the run time of launch_proxy_potentials.  A slot's only piece writes the
// slot's row, several pieces write partial rows past the slots (summed by
// launch_upward_reduce).  Uploads d.chunk_slot / chunk_begin (first entry) /
// chunk_count (entries) / chunk_dst (row) / slot_chunk_off, sets d.nchunks
// and d.nslots, and returns the number of rows in *rows.
int upload_pieces(bltc_plan* plan, bltc::DevicePlan& d, const std::vector<int32_t>& off,
                  const std::vector<int64_t>& count, int64_t* rows, hipStream_t s);
}  // namespace bltc_cp

// cluster-cluster plans (cc.cpp)
namespace bltc_cc {
int create_host(bltc_plan* plan, const bltc::PlanParams& pp, int64_t nt, const double* tx,
                const double* ty, const double* tz, int64_t ns, const double* sx, const double* sy,
                const double* sz);
int create_device(bltc_plan* plan, const bltc::PlanParams& pp, int64_t nt, const double* tx,
                  const double* ty, const double* tz, int64_t ns, const double* sx,
                  const double* sy, const double* sz, hipStream_t s);
int upload(bltc_plan* plan, hipStream_t s);
int execute(bltc_plan* plan, const double* q, int32_t num_q, double* phi, hipStream_t s);
int proxy_potentials(bltc_plan* plan, int64_t cluster, double* out, hipStream_t s);
void stats(const bltc_plan* plan, bltc_stats* out);
int view(const bltc_plan* plan, bltc_plan_view* out);
}  // namespace bltc_cc
