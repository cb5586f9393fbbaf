// batch.cpp -- many independent systems in one evaluation: the C ABI
// bltc_batch_* of include/bltc.h.
//
// A batch is built from plans (one per system, each created with max_q >= 2 so
// that it holds the 16-vector tables).  One execution enqueues, per system,
// the gather of its charge vectors into tree order; one matrix-core upward
// launch over the chunks of all systems; per system the fixed-order chunk
// reduction; and ONE persistent work-queue launch that runs every
// (system, 256-target group) unit of every system, heaviest first.  The whole
// sequence is captured once into a hipGraph per set of caller buffers and
// replayed afterwards.
#include <cstring>
#include <exception>
#include <new>

#include "internal.hpp"

using bltc_detail::fail;

struct bltc_batch {
    std::vector<bltc_plan*> plans;
    bltc::KernelParams kp;
    int32_t mw = 16;
    // work-queue units (system, group), heaviest first, and upward units
    bltc::MrhsDesc* d_descs = nullptr;
    int2* d_units = nullptr;
    int32_t nunits = 0;
    bltc::UpwardDesc* d_updescs = nullptr;
    int2* d_upunits = nullptr;
    int32_t nupunits = 0;
    int32_t passes = 1;
    size_t lds = 0;
    // every system of one degree n <= 8: the 16-vector Lagrange upward kernel
    // (FP32 products for FP32-mixed batches) instead of the general one
    int32_t multi_np = 0;
    int32_t* d_counter = nullptr;
    int32_t workgroups = 0;
    // graph of the last set of caller buffers
    bool use_graph = true;
    std::vector<uintptr_t> key;
    hipGraphExec_t exec = nullptr;
    hipStream_t capture = nullptr;
    int64_t captures = 0, launches = 0;

    ~bltc_batch()
    {
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (capture)
            (void)hipStreamDestroy(capture);
        for (void* p : {static_cast<void*>(d_descs), static_cast<void*>(d_units),
                        static_cast<void*>(d_updescs), static_cast<void*>(d_upunits),
                        static_cast<void*>(d_counter)})
            if (p)
                (void)hipFree(p);
    }
};

namespace {

int enqueue(bltc_batch* b, const double* const* q, const int32_t* num_q, const int64_t* q_ld,
            const double* const* phi, hipStream_t s)
{
    (void)phi;
    const int32_t count = static_cast<int32_t>(b->plans.size());
    for (int32_t i = 0; i < count; ++i) {
        const bltc::DevicePlan& d = b->plans[i]->d;
        HIP_TRY(bltc::launch_gather_charges16(d, q[i], q_ld[i], num_q[i], s));
    }
    if (b->multi_np > 0)
        HIP_TRY(bltc::launch_upward_many_multi(b->d_updescs, b->d_upunits, b->nupunits,
                                               b->multi_np, b->kp.precision == 1, s));
    else
        HIP_TRY(bltc::launch_upward_many(b->d_updescs, b->d_upunits, b->nupunits, b->mw,
                                         b->passes, b->lds, s));
    for (int32_t i = 0; i < count; ++i) {
        const bltc::DevicePlan& d = b->plans[i]->d;
        HIP_TRY(bltc::launch_upward_reduce(d, b->mw, d.qhat16, d.qhat16f, s));
    }
    HIP_TRY(bltc::launch_reset_counter(b->d_counter, s));
    HIP_TRY(bltc::launch_interact_queue(b->d_descs, b->d_units, b->nunits, b->d_counter, b->kp,
                                        b->workgroups, s));
    return BLTC_OK;
}

int batch_create(bltc_batch** out, bltc_plan* const* plans, int32_t count, void* stream)
{
    if (!out)
        return fail(BLTC_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 1 || !plans)
        return fail(BLTC_EINVAL, "a batch needs at least one plan");
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int32_t i = 0; i < count; ++i) {
        if (!plans[i])
            return fail(BLTC_EINVAL, "plan %d is NULL", i);
        if (plans[i]->cp || plans[i]->cc || plans[i]->prm.method == BLTC_HERMITE)
            return fail(BLTC_EUNSUPPORTED, "plan %d is a cluster-particle, cluster-cluster or "
                                           "Hermite plan (not batchable)", i);
        if (plans[i]->max_q < 2)
            return fail(BLTC_EINVAL, "plan %d was created with max_q < 2 (batches use the "
                                     "16-vector tables)", i);
        if (plans[i]->prm.kernel != plans[0]->prm.kernel ||
            plans[i]->prm.precision != plans[0]->prm.precision)
            return fail(BLTC_EINVAL, "plans of a batch must share kernel and precision");
        int rc = bltc_internal_upload_plan(plans[i], s);
        if (rc != BLTC_OK)
            return rc;
    }
    bltc_batch* b = new (std::nothrow) bltc_batch();
    if (!b)
        return fail(BLTC_ENOMEM, "cannot allocate batch");
    b->plans.assign(plans, plans + count);
    b->kp.kernel = plans[0]->prm.kernel;
    b->kp.precision = plans[0]->prm.precision;
    b->kp.kappa = plans[0]->prm.kappa;
    b->kp.delta = plans[0]->prm.delta;

    // work-queue units: every non-empty group of every system, heaviest first
    struct Unit { int32_t sys, group; int64_t cost; };
    std::vector<Unit> units;
    std::vector<Unit> up;
    int32_t max_np = 1;
    bool one_np = true;
    for (int32_t i = 0; i < count; ++i) {
        const bltc::HostPlan& hp = plans[i]->hp;
        one_np = one_np && hp.np == plans[0]->hp.np && !plans[i]->d.hermite;
        for (size_t g = 0; g < hp.group_batch.size(); ++g) {
            const int32_t bt = hp.group_batch[g];
            if (bt >= 0)
                units.push_back({i, static_cast<int32_t>(g), hp.batch_cost[bt]});
        }
        for (size_t c = 0; c < hp.chunk_slot.size(); ++c)
            up.push_back({i, static_cast<int32_t>(c), hp.chunk_count[c]});
        max_np = std::max(max_np, hp.np);
    }
    std::stable_sort(units.begin(), units.end(),
                     [](const Unit& a, const Unit& c) { return a.cost > c.cost; });
    std::stable_sort(up.begin(), up.end(),
                     [](const Unit& a, const Unit& c) { return a.cost > c.cost; });
    std::vector<int2> hu(units.size()), hup(up.size());
    for (size_t k = 0; k < units.size(); ++k)
        hu[k] = make_int2(units[k].sys, units[k].group);
    for (size_t k = 0; k < up.size(); ++k)
        hup[k] = make_int2(up[k].sys, up[k].group);
    b->nunits = static_cast<int32_t>(hu.size());
    b->nupunits = static_cast<int32_t>(hup.size());
    b->passes = bltc::upward_passes(max_np, b->mw);
    b->lds = bltc::upward_lds_bytes(max_np, b->mw, max_np);
    if (one_np && bltc::upward_many_multi(max_np, b->mw))
        b->multi_np = max_np;

    std::vector<bltc::UpwardDesc> ud(count);
    for (int32_t i = 0; i < count; ++i) {
        const bltc::DevicePlan& d = plans[i]->d;
        ud[i] = bltc::UpwardDesc{d.src, d.qm, d.qm32, d.chunk_slot, d.chunk_begin, d.chunk_count,
                                 d.chunk_dst, d.slot_nodes, d.qhat16, d.degree + 1};
    }
    int rc = BLTC_OK;
    auto put = [&](auto** dst, const auto& v) -> hipError_t {
        return bltc_detail::upload(dst, v, s);
    };
    hipError_t e = put(&b->d_units, hu);
    if (e == hipSuccess)
        e = put(&b->d_upunits, hup);
    if (e == hipSuccess)
        e = put(&b->d_updescs, ud);
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void**>(&b->d_descs), sizeof(bltc::MrhsDesc) * count);
    if (e == hipSuccess)
        e = hipMalloc(reinterpret_cast<void**>(&b->d_counter), sizeof(int32_t));
    if (e == hipSuccess)
        e = bltc::upward_prepare(b->lds);
    if (e == hipSuccess) {
        int dev = 0, cus = 0, per_cu = 0;
        e = hipGetDevice(&dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, bltc::interact_queue_symbol(b->kp), bltc::kGroupSize, 0);
        b->workgroups = std::max(1, std::min(b->nunits, cus * std::max(1, per_cu)));
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        rc = bltc_detail::hip_fail(e, "batch setup");
    if (rc != BLTC_OK) {
        delete b;
        return rc;
    }
    *out = b;
    return BLTC_OK;
}

int batch_execute(bltc_batch* b, const double* const* q, const int32_t* num_q,
                  const int64_t* q_ld, double* const* phi, const int64_t* phi_ld, void* stream)
{
    if (!b || !q || !num_q || !q_ld || !phi || !phi_ld)
        return fail(BLTC_EINVAL, "NULL argument");
    const int32_t count = static_cast<int32_t>(b->plans.size());
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<uintptr_t> key;
    key.reserve(5 * count);
    for (int32_t i = 0; i < count; ++i) {
        const bltc_plan* p = b->plans[i];
        if (num_q[i] < 1 || num_q[i] > std::min<int32_t>(16, p->max_q))
            return fail(BLTC_EINVAL, "system %d: num_q must be in 1..min(16, max_q)", i);
        if (p->hp.src.n > 0 && !q[i])
            return fail(BLTC_EINVAL, "system %d: q is NULL", i);
        if (p->hp.tgt.n > 0 && !phi[i])
            return fail(BLTC_EINVAL, "system %d: phi is NULL", i);
        if (num_q[i] > 1 && (q_ld[i] < p->hp.src.n || phi_ld[i] < p->hp.tgt.n))
            return fail(BLTC_EINVAL, "system %d: leading dimensions too small", i);
        key.push_back(reinterpret_cast<uintptr_t>(q[i]));
        key.push_back(static_cast<uintptr_t>(num_q[i]));
        key.push_back(static_cast<uintptr_t>(q_ld[i]));
        key.push_back(reinterpret_cast<uintptr_t>(phi[i]));
        key.push_back(static_cast<uintptr_t>(phi_ld[i]));
    }
    if (key != b->key) {
        // new caller buffers: refresh the per-system descriptors, drop the graph
        std::vector<bltc::MrhsDesc> descs(count);
        for (int32_t i = 0; i < count; ++i) {
            // kernel constants per system (the kernel itself is shared)
            bltc::KernelParams kpi = b->kp;
            kpi.kappa = b->plans[i]->prm.kappa;
            kpi.delta = b->plans[i]->prm.delta;
            descs[i] = bltc::make_mrhs_desc(b->plans[i]->d, kpi, phi[i], phi_ld[i], num_q[i]);
        }
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(hipMemcpy(b->d_descs, descs.data(), sizeof(bltc::MrhsDesc) * count,
                          hipMemcpyHostToDevice));
        if (b->exec) {
            HIP_TRY(hipGraphExecDestroy(b->exec));
            b->exec = nullptr;
        }
        b->key = key;
        for (int32_t i = 0; i < count; ++i)
            b->plans[i]->last_q = num_q[i];
    }
    if (!b->use_graph) {
        ++b->launches;
        return enqueue(b, q, num_q, q_ld, phi, s);
    }
    if (!b->exec) {
        if (!b->capture)
            HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
        const int rc = enqueue(b, q, num_q, q_ld, phi, b->capture);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(b->capture, &graph);
        if (rc != BLTC_OK) {
            if (graph)
                (void)hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess)
            return bltc_detail::hip_fail(e, "hipStreamEndCapture");
        const hipError_t ei = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess)
            return bltc_detail::hip_fail(ei, "hipGraphInstantiate");
        ++b->captures;
    }
    HIP_TRY(hipGraphLaunch(b->exec, s));
    ++b->launches;
    return BLTC_OK;
}

}  // namespace

extern "C" {

// host allocations of the planner and the batch tables may throw: no
// exception leaves the C ABI
int bltc_batch_create(bltc_batch** out, bltc_plan* const* plans, int32_t count, void* stream)
{
    try {
        return batch_create(out, plans, count, stream);
    } catch (const std::bad_alloc&) {
        return fail(BLTC_ENOMEM, "host allocation failed while building the batch");
    } catch (const std::exception& ex) {
        return fail(BLTC_EINTERNAL, "batch creation failed: %s", ex.what());
    }
}

int bltc_batch_execute(bltc_batch* b, const double* const* q, const int32_t* num_q,
                       const int64_t* q_ld, double* const* phi, const int64_t* phi_ld,
                       void* stream)
{
    try {
        return batch_execute(b, q, num_q, q_ld, phi, phi_ld, stream);
    } catch (const std::bad_alloc&) {
        return fail(BLTC_ENOMEM, "host allocation failed");
    } catch (const std::exception& ex) {
        return fail(BLTC_EINTERNAL, "%s", ex.what());
    }
}

int bltc_batch_set_graph(bltc_batch* b, int32_t enable)
{
    if (!b)
        return fail(BLTC_EINVAL, "batch is NULL");
    b->use_graph = enable != 0;
    return BLTC_OK;
}

int bltc_batch_info_get(const bltc_batch* b, bltc_batch_info* out)
{
    if (!b || !out)
        return fail(BLTC_EINVAL, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    out->systems = static_cast<int32_t>(b->plans.size());
    out->units = b->nunits;
    out->upward_units = b->nupunits;
    out->workgroups = b->workgroups;
    out->graph_captures = b->captures;
    out->launches = b->launches;
    return BLTC_OK;
}

int bltc_batch_potential(bltc_plan* const* plans, int32_t count, const double* const* q,
                         const int32_t* num_q, const int64_t* q_ld, double* const* phi,
                         const int64_t* phi_ld, void* stream)
{
    bltc_batch* b = nullptr;
    int rc = bltc_batch_create(&b, plans, count, stream);
    if (rc != BLTC_OK)
        return rc;
    rc = bltc_batch_set_graph(b, 0);
    if (rc == BLTC_OK)
        rc = bltc_batch_execute(b, q, num_q, q_ld, phi, phi_ld, stream);
    if (rc == BLTC_OK) {
        hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (e != hipSuccess)
            rc = bltc_detail::hip_fail(e, "hipStreamSynchronize");
    }
    bltc_batch_destroy(b);
    return rc;
}

void bltc_batch_destroy(bltc_batch* b)
{
    delete b;
}

}  // extern "C"
