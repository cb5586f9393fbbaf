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

inline int hip_fail(hipError_t e, const char* what)
{
    return fail(BLTC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

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

    ~bltc_plan()
    {
        for (hipEvent_t e : events)
            (void)hipEventDestroy(e);
        if (ev_pairs)
            (void)hipEventDestroy(ev_pairs);
        for (void* p : allocations)
            (void)hipFree(p);
    }

    template <class T>
    hipError_t put(T** dst, const std::vector<T>& v, hipStream_t s)
    {
        hipError_t e = bltc_detail::upload(dst, v, s);
        if (e == hipSuccess)
            allocations.push_back(*dst);
        return e;
    }

    template <class T>
    hipError_t alloc(T** dst, size_t count)
    {
        hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), std::max<size_t>(1, count) * sizeof(T));
        if (e == hipSuccess)
            allocations.push_back(*dst);
        return e;
    }
};


// device side of a plan (uploads on first use); synchronises the stream
int bltc_internal_upload_plan(bltc_plan* plan, hipStream_t s);

// Mutual direct pairs of one-tree direct lists evaluated once (see
// plan_symmetric): plans the units, uploads them, the reduced lists and the
// per-batch result offsets into d (d.sym = 1), and lowers the lists' batch_cost
// in *cost to the work left to the batches.  Returns BLTC_OK and leaves d
// alone when no pair qualifies; `sub` = targets per sub-unit.
int bltc_internal_upload_symmetric(bltc_plan* plan, bltc::DevicePlan& d,
                                   const bltc::DirectLists& dl, std::vector<int64_t>* cost,
                                   hipStream_t s);

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
