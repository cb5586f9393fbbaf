// capi.cpp -- the C ABI declared in include/bltc.h: argument checks, plans
// (host planning + device tables), execution on the caller's HIP stream.
#include "bltc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"
#include "parallel.hpp"
#include "kernels_split.hpp"
#include "setup_gpu.hpp"

using bltc_detail::fail;
using bltc_detail::hip_fail;

namespace {

int check_params(const bltc_params* p)
{
    if (!p)
        return fail(BLTC_EINVAL, "params is NULL");
    if (p->kernel != BLTC_COULOMB && p->kernel != BLTC_YUKAWA &&
        p->kernel != BLTC_REGULARIZED_COULOMB)
        return fail(BLTC_EINVAL,
                    "kernel must be BLTC_COULOMB, BLTC_YUKAWA or BLTC_REGULARIZED_COULOMB");
    if (p->precision != BLTC_FP64 && p->precision != BLTC_FP32_MIXED)
        return fail(BLTC_EINVAL, "precision must be BLTC_FP64 or BLTC_FP32_MIXED");
    if (!(p->kappa >= 0.0) || !std::isfinite(p->kappa))
        return fail(BLTC_EINVAL, "kappa must be finite and >= 0");
    if (!(p->delta >= 0.0) || !std::isfinite(p->delta))
        return fail(BLTC_EINVAL, "delta must be finite and >= 0");
    if (!(p->theta >= 0.0 && p->theta < 1.0))
        return fail(BLTC_EINVAL, "theta must satisfy 0 <= theta < 1");
    if (p->degree < 1 || p->degree > bltc::kMaxDegree)
        return fail(BLTC_EINVAL, "degree must be in 1..%d", bltc::kMaxDegree);
    if (p->leaf_size < 0 || p->batch_size < 0 || (p->leaf_size == 0) != (p->batch_size == 0))
        return fail(BLTC_EINVAL, "leaf_size and batch_size must both be >= 1, or both 0 "
                                 "(autotune)");
    if (p->workspace_limit < 0)
        return fail(BLTC_EINVAL, "workspace_limit must be >= 0 (0: no limit)");
    if (p->threads_per_target != 0 && p->threads_per_target != 1 && p->threads_per_target != 2 &&
        p->threads_per_target != 4)
        return fail(BLTC_EINVAL, "threads_per_target must be 0, 1, 2 or 4");
    if (p->no_symmetry != 0 && p->no_symmetry != 1)
        return fail(BLTC_EINVAL, "no_symmetry must be 0 or 1");
    if (p->method != BLTC_PARTICLE_CLUSTER && p->method != BLTC_CLUSTER_PARTICLE &&
        p->method != BLTC_CLUSTER_CLUSTER && p->method != BLTC_HERMITE)
        return fail(BLTC_EINVAL, "method must be BLTC_PARTICLE_CLUSTER, BLTC_CLUSTER_PARTICLE, "
                                 "BLTC_CLUSTER_CLUSTER or BLTC_HERMITE");
    if (p->method == BLTC_HERMITE && p->degree > bltc::kMaxHermiteDegree)
        return fail(BLTC_EUNSUPPORTED, "the Hermite treecode takes degree 1..%d",
                    bltc::kMaxHermiteDegree);
    return BLTC_OK;
}

int check_coords(int64_t n, const double* x, const double* y, const double* z, const char* what)
{
    if (n < 0)
        return fail(BLTC_EINVAL, "%s count is negative", what);
    if (n > 0 && (!x || !y || !z))
        return fail(BLTC_EINVAL, "%s coordinate pointer is NULL", what);
    return BLTC_OK;
}

int check_finite(int64_t n, const double* x, const double* y, const double* z, const char* what)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i]) || !std::isfinite(y[i]) || !std::isfinite(z[i]))
            return fail(BLTC_EINVAL, "%s coordinate %lld is not finite", what,
                        static_cast<long long>(i));
    return BLTC_OK;
}


}  // namespace

namespace {

bltc::PlanParams plan_params(const bltc_plan* plan, const bltc_params* p)
{
    bltc::PlanParams pp;
    pp.theta = p->theta;
    pp.degree = p->degree;
    pp.leaf_size = p->leaf_size;
    pp.batch_size = p->batch_size;
    pp.group_size = bltc::kGroupSize;
    pp.comps = p->method == BLTC_HERMITE ? 8 : 1;
    // upward-pass chunks: with one charge vector a chunk is a few MFMA tiles, so
    // smaller chunks give more workgroups; 16 vectors fill 9x more tiles per chunk
    pp.chunk_size = plan->max_q > 1 ? 8192 : 2048;
    return pp;
}

int make_host_plan(bltc_plan* plan, const bltc_params* p, int64_t nt, const double* tx,
                   const double* ty, const double* tz, int64_t ns, const double* sx,
                   const double* sy, const double* sz)
{
    std::string err = bltc::make_plan(plan->hp, plan_params(plan, p), nt, tx, ty, tz, ns, sx, sy, sz);
    if (!err.empty())
        return fail(BLTC_EINTERNAL, "%s", err.c_str());
    return BLTC_OK;
}

// Trees built on the device from device coordinates; the per-particle arrays
// of the plan are written there directly, the node arrays come back to the
// host for the interaction lists.
int make_device_plan(bltc_plan* plan, const bltc_params* p, int64_t nt, const double* tx,
                     const double* ty, const double* tz, int64_t ns, const double* sx,
                     const double* sy, const double* sz, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    bltc::HostPlan& hp = plan->hp;
    hp = bltc::HostPlan();
    hp.prm = plan_params(plan, p);
    bltc::DevicePlan& d = plan->d;
    const bool mixed = p->precision == BLTC_FP32_MIXED;
    HIP_TRY(hipGetDevice(&plan->device));
    int64_t* src_order = nullptr;
    HIP_TRY(plan->alloc(&d.src, static_cast<size_t>(ns)));
    HIP_TRY(plan->alloc(&src_order, static_cast<size_t>(ns)));
    d.src_order = src_order;
    if (mixed)
        HIP_TRY(plan->alloc(&d.src32, static_cast<size_t>(ns)));
    HIP_TRY(plan->alloc(&d.tgt, static_cast<size_t>(nt)));
    HIP_TRY(plan->alloc(&d.tgt_orig, static_cast<size_t>(nt)));
    int64_t bad = -1;
    std::string err = bltc::build_tree_device(hp.src, ns, sx, sy, sz, p->leaf_size, src_order,
                                              d.src, mixed ? d.src32 : nullptr, s, &bad);
    if (bad >= 0)
        return fail(BLTC_EINVAL, "source coordinate %lld is not finite", static_cast<long long>(bad));
    if (!err.empty())
        return fail(BLTC_EHIP, "device tree build: %s", err.c_str());
    if (nt == ns && tx == sx && ty == sy && tz == sz && p->batch_size == p->leaf_size) {
        // same particles, same capacity: identical partition
        hp.tgt = hp.src;
        hp.same_tree = true;
        if (nt > 0) {
            HIP_TRY(hipMemcpyAsync(d.tgt, d.src, nt * sizeof(double4), hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(d.tgt_orig, src_order, nt * sizeof(int64_t),
                                   hipMemcpyDeviceToDevice, s));
        }
    } else {
        err = bltc::build_tree_device(hp.tgt, nt, tx, ty, tz, p->batch_size, d.tgt_orig, d.tgt,
                                      nullptr, s, &bad);
        if (bad >= 0)
            return fail(BLTC_EINVAL, "target coordinate %lld is not finite",
                        static_cast<long long>(bad));
        if (!err.empty())
            return fail(BLTC_EHIP, "device tree build: %s", err.c_str());
    }
    bltc::plan_batches(hp);
    bltc::DeviceLists dl;
    auto alloc = [plan](void** ptr, size_t bytes) -> hipError_t {
        return plan->alloc_bytes(ptr, bytes);
    };
    err = bltc::build_lists_device(hp, dl, alloc, s);
    if (!err.empty())
        return fail(BLTC_EHIP, "device interaction lists: %s", err.c_str());
    bltc::plan_schedule(hp);
    d.far_slot = dl.far_slot;
    d.near_leaf = dl.near_leaf;
    d.near_begin = dl.near_begin;
    d.near_count = dl.near_count;
    plan->item_batch = dl.item_batch;
    plan->item_cluster = dl.item_cluster;
    plan->item_kind = dl.item_kind;
    plan->n_items = dl.n_items;
    plan->device_particles = true;
    plan->device_lists = true;
    hp.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return BLTC_OK;
}

// Mutual direct leaf pairs of a BLTC or Hermite plan evaluated once (targets
// are the sources, one charge vector).  Plans that do not qualify keep their
// lists (d.sym = 0).
int upload_symmetric(bltc_plan* plan, hipStream_t s)
{
    bltc::HostPlan& hp = plan->hp;
    bltc::DevicePlan& d = plan->d;
    if (plan->prm.no_symmetry || plan->max_q != 1 || !hp.same_tree ||
        (plan->prm.method != BLTC_PARTICLE_CLUSTER && plan->prm.method != BLTC_HERMITE))
        return BLTC_OK;
    const int64_t nb = static_cast<int64_t>(hp.batch_node.size());
    const int64_t nnear = nb > 0 ? hp.near_off[nb] : 0;
    std::vector<int32_t> near_leaf;
    if (plan->device_lists) {
        near_leaf.resize(nnear);
        if (nnear > 0)
            HIP_TRY(hipMemcpy(near_leaf.data(), d.near_leaf, nnear * sizeof(int32_t),
                              hipMemcpyDeviceToHost));
    } else {
        near_leaf = hp.near_leaf;
    }
    const bltc::DirectLists dl{&hp.src,      &hp.batch_node, &hp.batch_begin, &hp.batch_count,
                               &hp.near_off, &near_leaf,     &hp.batch_cost};
    return bltc_internal_upload_symmetric(plan, d, dl, &hp.batch_cost, s);
}

// Plans with one charge vector: interaction workgroups of kGroupSizeSym
// targets (one wave; a finer tail than kGroupSize), ordered by the work left
// to each batch.
void schedule_single_vector(bltc_plan* plan)
{
    bltc::HostPlan& hp = plan->hp;
    if (plan->max_q != 1)
        return;
    hp.prm.group_size = bltc::kGroupSizeSym;
    hp.group_batch.clear();
    hp.group_first.clear();
    // time per target: a direct term costs about 2.2 far-field terms (three
    // differences and squares against one add per kernel value)
    const int64_t nb = static_cast<int64_t>(hp.batch_begin.size());
    std::vector<int64_t> cost(nb);
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t far = static_cast<int64_t>(hp.far_off[b + 1] - hp.far_off[b]) * hp.P;
        const int64_t near = std::max<int64_t>(0, hp.batch_cost[b] - far);
        cost[b] = far + (near * 22) / 10;
    }
    bltc::group_schedule(hp.batch_begin, hp.batch_count, cost, hp.prm.group_size,
                         hp.prm.xcds, hp.group_batch, hp.group_first);
    plan->d.ngroups = static_cast<int64_t>(hp.group_batch.size());
    plan->d.group_threads = bltc::kGroupSizeSym;
}

// Threads per target T > 1: batch b becomes the batches b T + p, p < T, whose
// lists are contiguous pieces of b's far and (reduced) direct lists, over T
// copies of the targets; copy p writes its partial potentials to row p of
// plan->tpt_buf in caller order.  The mutual-pair results of b go with piece 0.
int upload_split(bltc_plan* plan, hipStream_t s)
{
    const bltc::HostPlan& hp = plan->hp;
    const bltc::DevicePlan& d = plan->d;
    const int32_t T = plan->prm.threads_per_target;
    const int64_t nb = d.nbatches, nt = d.nt;
    bltc::DevicePlan& t = plan->dt;
    t = d;
    auto split = [&](const std::vector<int32_t>& off) {
        std::vector<int32_t> out(static_cast<size_t>(nb * T + 1), 0);
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t n = off[b + 1] - off[b];
            for (int32_t p = 0; p < T; ++p)
                out[b * T + p] = static_cast<int32_t>(off[b] + n * p / T);
        }
        out[nb * T] = nb > 0 ? off[nb] : 0;
        return out;
    };
    HIP_TRY(plan->put(&t.far_off, split(hp.far_off), s));
    if (d.sym) {
        HIP_TRY(plan->put(&t.sym_near_off, split(plan->sym_near_off_h), s));
        std::vector<int32_t> pc_off(static_cast<size_t>(nb * T + 1), 0);
        std::vector<int64_t> bbeg(static_cast<size_t>(nb * T));
        for (int64_t b = 0; b < nb; ++b)
            for (int32_t p = 0; p < T; ++p) {
                pc_off[b * T + p] = p == 0 ? plan->sym_pc_off_h[b] : plan->sym_pc_off_h[b + 1];
                bbeg[b * T + p] = p * nt + hp.batch_begin[b];
            }
        pc_off[nb * T] = nb > 0 ? plan->sym_pc_off_h[nb] : 0;
        HIP_TRY(plan->put(&t.sym_pc_off, pc_off, s));
        HIP_TRY(plan->put(&t.batch_begin, bbeg, s));
    } else {
        HIP_TRY(plan->put(&t.near_off, split(hp.near_off), s));
    }
    // T copies of the targets, written on the device; copy p writes p nt +
    // caller index
    HIP_TRY(plan->alloc(&t.tgt, static_cast<size_t>(T * nt)));
    int64_t* orig_t = nullptr;
    HIP_TRY(plan->alloc(&orig_t, static_cast<size_t>(T * nt)));
    t.tgt_orig = orig_t;
    HIP_TRY(bltc::launch_replicate_targets(t.tgt, orig_t, d.tgt, d.tgt_orig, nt, T, s));
    std::vector<int64_t> end_t(static_cast<size_t>(nb * T));
    // batches, their boxes (FP32-mixed) and the workgroup schedule, each
    // piece with 1/T of its batch's work
    std::vector<int64_t> begin_t(static_cast<size_t>(nb * T)), count_t(begin_t.size()),
        cost_t(begin_t.size());
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t far = static_cast<int64_t>(hp.far_off[b + 1] - hp.far_off[b]) * hp.P;
        const int64_t near = std::max<int64_t>(0, hp.batch_cost[b] - far);
        const int64_t cost = far + (near * 22) / 10;
        for (int32_t p = 0; p < T; ++p) {
            begin_t[b * T + p] = p * nt + hp.batch_begin[b];
            count_t[b * T + p] = hp.batch_count[b];
            end_t[b * T + p] = begin_t[b * T + p] + hp.batch_count[b];
            cost_t[b * T + p] = cost / T;
        }
    }
    HIP_TRY(plan->put(&t.batch_end, end_t, s));
    if (plan->prm.precision == BLTC_FP32_MIXED) {
        std::vector<double4> bi(static_cast<size_t>(nb * T));
        for (int64_t b = 0; b < nb; ++b) {
            const int32_t bn = hp.batch_node[b];
            for (int32_t p = 0; p < T; ++p)
                bi[b * T + p] = make_double4(hp.tgt.center[3 * bn], hp.tgt.center[3 * bn + 1],
                                             hp.tgt.center[3 * bn + 2], hp.tgt.radius[bn]);
        }
        HIP_TRY(plan->put(&t.batch_info, bi, s));
    }
    std::vector<int32_t> gb;
    std::vector<int64_t> gf;
    bltc::group_schedule(begin_t, count_t, cost_t, bltc::kGroupSizeSym, hp.prm.xcds, gb, gf);
    HIP_TRY(plan->put(&t.group_batch, gb, s));
    HIP_TRY(plan->put(&t.group_first, gf, s));
    t.ngroups = static_cast<int64_t>(gb.size());
    t.group_threads = bltc::kGroupSizeSym;
    t.nbatches = nb * T;
    t.nt = T * nt;
    HIP_TRY(plan->alloc(&plan->tpt_buf, static_cast<size_t>(T * nt)));
    HIP_TRY(hipStreamSynchronize(s));
    plan->tpt = T;
    return BLTC_OK;
}

}  // namespace

namespace {

int upload_particle_cluster(bltc_plan* plan, hipStream_t s)
{
    const bltc::HostPlan& hp = plan->hp;
    bltc::DevicePlan& d = plan->d;
    HIP_TRY(hipGetDevice(&plan->device));
    d.degree = plan->prm.degree;
    d.hermite = plan->prm.method == BLTC_HERMITE;
    d.nt = hp.tgt.n;
    d.ns = hp.src.n;
    d.nslots = static_cast<int64_t>(hp.slot_cluster.size());
    d.nchunks = static_cast<int64_t>(hp.chunk_slot.size());
    d.ngroups = static_cast<int64_t>(hp.group_batch.size());
    d.nbatches = static_cast<int64_t>(hp.batch_begin.size());

    if (!plan->device_particles) {
        std::vector<double4> src(d.ns), tgt(d.nt);
        for (int64_t j = 0; j < d.ns; ++j)
            src[j] = make_double4(hp.src.x[j], hp.src.y[j], hp.src.z[j], 0.0);
        for (int64_t i = 0; i < d.nt; ++i)
            tgt[i] = make_double4(hp.tgt.x[i], hp.tgt.y[i], hp.tgt.z[i], 0.0);
        HIP_TRY(plan->put(&d.src, src, s));
        HIP_TRY(plan->put(&d.tgt, tgt, s));
        HIP_TRY(plan->put(&d.tgt_orig, hp.tgt.order, s));
        int64_t* src_order = nullptr;
        HIP_TRY(plan->put(&src_order, hp.src.order, s));
        d.src_order = src_order;
        HIP_TRY(hipStreamSynchronize(s));
    }
    int rc = upload_symmetric(plan, s);
    if (rc != BLTC_OK)
        return rc;
    schedule_single_vector(plan);
    std::vector<int64_t> batch_end(d.nbatches);
    for (int64_t b = 0; b < d.nbatches; ++b)
        batch_end[b] = hp.batch_begin[b] + hp.batch_count[b];
    HIP_TRY(plan->put(&d.group_batch, hp.group_batch, s));
    HIP_TRY(plan->put(&d.group_first, hp.group_first, s));
    HIP_TRY(plan->put(&d.batch_end, batch_end, s));
    HIP_TRY(plan->put(&d.far_off, hp.far_off, s));
    HIP_TRY(plan->put(&d.near_off, hp.near_off, s));
    if (!plan->device_lists) {
        HIP_TRY(plan->put(&d.far_slot, hp.far_slot, s));
        HIP_TRY(plan->put(&d.near_begin, hp.near_begin, s));
        HIP_TRY(plan->put(&d.near_count, hp.near_count, s));
        HIP_TRY(plan->put(&d.near_leaf, hp.near_leaf, s));
    }
    HIP_TRY(plan->put(&d.slot_nodes, hp.slot_nodes, s));
    HIP_TRY(plan->put(&d.chunk_slot, hp.chunk_slot, s));
    HIP_TRY(plan->put(&d.chunk_begin, hp.chunk_begin, s));
    HIP_TRY(plan->put(&d.chunk_count, hp.chunk_count, s));
    HIP_TRY(plan->put(&d.slot_chunk_off, hp.slot_chunk_off, s));
    HIP_TRY(plan->put(&d.chunk_dst, hp.chunk_dst, s));
    // modified charges (first nslots rows) and the partial rows of multi-chunk
    // clusters; [row][P] for one charge vector, [row][P][16] for several
    const size_t mw_max = plan->max_q > 1 ? 16 : 1;
    HIP_TRY(plan->alloc(&d.qhat, static_cast<size_t>(d.nslots + hp.npartial) * hp.P * mw_max));
    if (d.hermite)
        HIP_TRY(plan->alloc(&d.qhat_h, static_cast<size_t>(d.nslots) * hp.P));
    const bool mixed = plan->prm.precision == BLTC_FP32_MIXED;
    if (plan->max_q > 1) {
        // expanded proxy grids for the multi-vector kernels
        const int32_t np = hp.np;
        std::vector<double4> prox(static_cast<size_t>(d.nslots) * hp.P);
        std::vector<float4> prox32(mixed ? prox.size() : 0);
        for (int64_t sl = 0; sl < d.nslots; ++sl) {
            const double* nd = hp.slot_nodes.data() + sl * 3 * np;
            const int32_t c = hp.slot_cluster[sl];
            const double cx = hp.src.center[3 * c], cy = hp.src.center[3 * c + 1],
                         cz = hp.src.center[3 * c + 2];
            for (int32_t k1 = 0; k1 < np; ++k1)
                for (int32_t k2 = 0; k2 < np; ++k2)
                    for (int32_t k3 = 0; k3 < np; ++k3) {
                        const size_t k = static_cast<size_t>(sl) * hp.P + (k1 * np + k2) * np + k3;
                        prox[k] = make_double4(nd[k1], nd[np + k2], nd[2 * np + k3], 0.0);
                        if (mixed)
                            prox32[k] = make_float4(static_cast<float>(nd[k1] - cx),
                                                    static_cast<float>(nd[np + k2] - cy),
                                                    static_cast<float>(nd[2 * np + k3] - cz), 0.0f);
                    }
        }
        HIP_TRY(plan->put(&d.proxies, prox, s));
        if (mixed)
            HIP_TRY(plan->put(&d.proxies32, prox32, s));
        HIP_TRY(hipStreamSynchronize(s));
        HIP_TRY(plan->put(&d.slot_cluster, hp.slot_cluster, s));
        HIP_TRY(plan->alloc(&d.qm, static_cast<size_t>(d.ns) * 16));
        d.qhat16 = d.qhat;
        if (mixed) {
            HIP_TRY(plan->alloc(&d.qm32, static_cast<size_t>(d.ns) * 16));
            HIP_TRY(plan->alloc(&d.qhat16f, static_cast<size_t>(d.nslots) * hp.P * 16));
        }
    }
    if (mixed) {
        // sources relative to the center of their leaf, per-node and per-batch boxes
        const int64_t nn = hp.src.nodes();
        std::vector<double4> node_info(nn);
        for (int64_t c = 0; c < nn; ++c)
            node_info[c] = make_double4(hp.src.center[3 * c], hp.src.center[3 * c + 1],
                                        hp.src.center[3 * c + 2], hp.src.radius[c]);
        if (!plan->device_particles) {
            std::vector<float4> src32(d.ns);
            for (int64_t j = 0; j < d.ns; ++j) {
                const double4 c = node_info[hp.leaf_of_pos[j]];
                src32[j] = make_float4(static_cast<float>(hp.src.x[j] - c.x),
                                       static_cast<float>(hp.src.y[j] - c.y),
                                       static_cast<float>(hp.src.z[j] - c.z), 0.0f);
            }
            HIP_TRY(plan->put(&d.src32, src32, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        std::vector<double4> batch_info(d.nbatches);
        for (int64_t b = 0; b < d.nbatches; ++b) {
            const int32_t bn = hp.batch_node[b];
            batch_info[b] = make_double4(hp.tgt.center[3 * bn], hp.tgt.center[3 * bn + 1],
                                         hp.tgt.center[3 * bn + 2], hp.tgt.radius[bn]);
        }
        HIP_TRY(plan->put(&d.node_info, node_info, s));
        HIP_TRY(plan->put(&d.batch_info, batch_info, s));
        HIP_TRY(plan->alloc(&d.qhat32, static_cast<size_t>(d.nslots) * hp.P));
        HIP_TRY(hipStreamSynchronize(s));
    }
    if (plan->prm.threads_per_target > 1) {
        rc = upload_split(plan, s);
        if (rc != BLTC_OK)
            return rc;
    }
    // host staging vectors die at return: finish the copies first
    HIP_TRY(hipStreamSynchronize(s));
    plan->uploaded = true;
    return BLTC_OK;
}

}  // namespace

namespace {

// Side of the smallest cube-aligned box around every point of the plan's trees.
double plan_extent(const bltc_plan* plan)
{
    double lo[3], hi[3];
    for (int l = 0; l < 3; ++l) {
        lo[l] = std::numeric_limits<double>::infinity();
        hi[l] = -std::numeric_limits<double>::infinity();
    }
    auto take = [&](const bltc::Tree& t) {
        if (t.nodes() == 0)
            return;
        for (int l = 0; l < 3; ++l) {   // node 0 is the root
            lo[l] = std::min(lo[l], t.lo[l]);
            hi[l] = std::max(hi[l], t.hi[l]);
        }
    };
    if (plan->cp) {
        take(plan->cpp.tgt);
        take(plan->cpp.src);
    } else if (plan->cc) {
        take(plan->ccp.tgt);
        take(plan->ccp.src);
    } else {
        take(plan->hp.src);
        take(plan->hp.tgt);
        const size_t nb = plan->hp.batch_lo.size() / 3;
        for (size_t b = 0; b < nb; ++b)
            for (int l = 0; l < 3; ++l) {
                lo[l] = std::min(lo[l], plan->hp.batch_lo[3 * b + l]);
                hi[l] = std::max(hi[l], plan->hp.batch_hi[3 * b + l]);
            }
    }
    double ext = 0.0;
    for (int l = 0; l < 3; ++l)
        if (hi[l] >= lo[l])
            ext = std::max(ext, hi[l] - lo[l]);
    return ext;
}

}  // namespace

// FP32-mixed kernels square coordinate differences in FP32: every distance
// between two points of the plan must keep its square finite there.
int bltc_internal_check_mixed_extent(const bltc_plan* plan)
{
    if (plan->prm.precision != BLTC_FP32_MIXED)
        return BLTC_OK;
    const double ext = plan_extent(plan);
    if (ext <= bltc::kMixedMaxExtent)
        return BLTC_OK;
    return fail(BLTC_EUNSUPPORTED,
                "FP32-mixed plans take points within a box of side at most 2^60 (%.3e here): "
                "FP32 squared distances would overflow; use BLTC_FP64",
                ext);
}

int bltc_internal_upload_plan(bltc_plan* plan, hipStream_t s)
{
    int rc = plan->uploaded ? BLTC_OK : bltc_internal_check_mixed_extent(plan);
    if (rc != BLTC_OK)
        return rc;
    if (!plan->uploaded)
        rc = plan->cp ? bltc_cp::upload(plan, s)
           : plan->cc ? bltc_cc::upload(plan, s)
                      : upload_particle_cluster(plan, s);
    // the mutual-pair workspace last: it takes what the workspace limit leaves
    if (rc == BLTC_OK)
        rc = bltc_internal_finish_pairs(plan, s);
    return rc;
}

namespace {

int zero_phi(int64_t nt, int32_t num_q, double* phi, int64_t phi_ld, hipStream_t s)
{
    for (int32_t m = 0; m < num_q; ++m)
        HIP_TRY(hipMemsetAsync(phi + static_cast<int64_t>(m) * phi_ld, 0, nt * sizeof(double), s));
    return BLTC_OK;
}

int execute(bltc_plan* plan, const double* q, int32_t num_q, int64_t q_ld, double* phi,
            int64_t phi_ld, hipStream_t s)
{
    const bltc::HostPlan& hp = plan->hp;
    const int64_t nt = plan->cp ? plan->cpp.tgt.n : plan->cc ? plan->ccp.tgt.n : hp.tgt.n;
    const int64_t ns = plan->cp ? plan->cpp.src.n : plan->cc ? plan->ccp.src.n : hp.src.n;
    if (num_q < 1 || num_q > plan->max_q)
        return fail(BLTC_EINVAL, "num_q must be in 1..max_q (%d)", plan->max_q);
    if (nt == 0)
        return BLTC_OK;
    if (!phi)
        return fail(BLTC_EINVAL, "phi is NULL");
    if (phi_ld < nt && num_q > 1)
        return fail(BLTC_EINVAL, "phi_ld must be >= nt");
    if (ns == 0)
        return zero_phi(nt, num_q, phi, phi_ld, s);
    if (!q)
        return fail(BLTC_EINVAL, "q is NULL");
    if (q_ld < ns && num_q > 1)
        return fail(BLTC_EINVAL, "q_ld must be >= ns");
    int rc = bltc_internal_upload_plan(plan, s);
    if (rc != BLTC_OK)
        return rc;
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != plan->device)
        return fail(BLTC_EINVAL, "plan was uploaded on device %d, current device is %d",
                    plan->device, dev);
    if (plan->cp)
        return bltc_cp::execute(plan, q, num_q, phi, s);
    if (plan->cc)
        return bltc_cc::execute(plan, q, num_q, phi, s);
    bltc::KernelParams kp;
    kp.kernel = plan->prm.kernel;
    kp.precision = plan->prm.precision;
    kp.kappa = plan->prm.kappa;
    kp.delta = plan->prm.delta;
    bltc::DevicePlan d = plan->d;
    // one charge vector: the scalar-charge kernels; several: passes of up to 16
    // vectors whose kernel values are shared (matrix-core contraction)
    const int32_t units = num_q == 1 ? 1 : (num_q + 15) / 16;
    if (plan->timing) {
        while (static_cast<int32_t>(plan->events.size()) < 4 * units) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            plan->events.push_back(e);
        }
    }
    plan->timed_q = 0;
    auto mark = [&](int32_t u, int k) -> hipError_t {
        return plan->timing ? hipEventRecord(plan->events[4 * u + k], s) : hipSuccess;
    };
    if (num_q == 1) {
        HIP_TRY(mark(0, 0));
        HIP_TRY(bltc::launch_gather_charges(d, q, s));
        HIP_TRY(mark(0, 1));
        HIP_TRY(bltc::launch_upward_mfma(d, 1, d.qhat, d.qhat32, s));
        HIP_TRY(mark(0, 2));
        if (d.sym) {
            rc = bltc_internal_pairs(plan, d, kp, s);
            if (rc != BLTC_OK)
                return rc;
            if (plan->timing) {
                if (!plan->ev_pairs)
                    HIP_TRY(hipEventCreate(&plan->ev_pairs));
                HIP_TRY(hipEventRecord(plan->ev_pairs, s));
            }
        }
        if (plan->tpt > 1) {
            // several lanes per target: partial potentials, then their sum
            if (d.hermite)
                HIP_TRY(bltc::launch_interact_hermite(plan->dt, kp, plan->tpt_buf, s));
            else if (kp.precision == BLTC_FP32_MIXED)
                HIP_TRY(bltc::launch_interact_mixed(plan->dt, kp, plan->tpt_buf, s));
            else
                HIP_TRY(bltc::launch_interact(plan->dt, kp, plan->tpt_buf, s));
            HIP_TRY(bltc::launch_sum_parts(plan->tpt_buf, d.nt, plan->tpt, phi, s));
        } else if (d.hermite) {
            HIP_TRY(bltc::launch_interact_hermite(d, kp, phi, s));
        } else if (kp.precision == BLTC_FP32_MIXED) {
            HIP_TRY(bltc::launch_interact_mixed(d, kp, phi, s));
        } else {
            HIP_TRY(bltc::launch_interact(d, kp, phi, s));
        }
        HIP_TRY(mark(0, 3));
    } else {
        for (int32_t u = 0; u < units; ++u) {
            const int32_t m0 = 16 * u;
            const int32_t mc = std::min<int32_t>(16, num_q - m0);
            HIP_TRY(mark(u, 0));
            HIP_TRY(bltc::launch_gather_charges16(d, q + static_cast<int64_t>(m0) * q_ld, q_ld, mc, s));
            HIP_TRY(mark(u, 1));
            HIP_TRY(bltc::launch_upward_mfma(d, 16, d.qhat16, d.qhat16f, s));
            HIP_TRY(mark(u, 2));
            HIP_TRY(bltc::launch_interact_mrhs(d, kp, phi + static_cast<int64_t>(m0) * phi_ld, phi_ld,
                                               mc, s));
            HIP_TRY(mark(u, 3));
        }
    }
    plan->timed_q = plan->timing ? units : 0;
    plan->timed_pairs = plan->timing && num_q == 1 && d.sym;
    plan->last_q = num_q;
    return BLTC_OK;
}

int create_common(bltc_plan** out, const bltc_params* p, int64_t nt, const double* tx,
                  const double* ty, const double* tz, int64_t ns, const double* sx,
                  const double* sy, const double* sz, int32_t max_q)
{
    if (!out)
        return fail(BLTC_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_params(p);
    if (rc != BLTC_OK)
        return rc;
    if ((rc = check_coords(nt, tx, ty, tz, "target")) != BLTC_OK)
        return rc;
    if ((rc = check_coords(ns, sx, sy, sz, "source")) != BLTC_OK)
        return rc;
    if (max_q < 1)
        return fail(BLTC_EINVAL, "max_q must be >= 1");
    if (p->method != BLTC_PARTICLE_CLUSTER && max_q != 1)
        return fail(BLTC_EUNSUPPORTED, "cluster-particle, cluster-cluster and Hermite plans take "
                                       "one charge vector (max_q = 1)");
    if (p->threads_per_target > 1 &&
        ((p->method != BLTC_PARTICLE_CLUSTER && p->method != BLTC_HERMITE) || max_q != 1))
        return fail(BLTC_EUNSUPPORTED, "threads_per_target > 1 needs a BLTC_PARTICLE_CLUSTER or "
                                       "BLTC_HERMITE plan with max_q = 1");
    return BLTC_OK;
}

int create_from_host(bltc_plan** out, const bltc_params* p, int64_t nt, const double* tx,
                     const double* ty, const double* tz, int64_t ns, const double* sx,
                     const double* sy, const double* sz, int32_t max_q)
{
    int rc;
    if (p->leaf_size == 0)
        return fail(BLTC_EUNSUPPORTED, "leaf_size = batch_size = 0 (autotune) needs a plan "
                                       "created from device coordinates");
    if ((rc = check_finite(nt, tx, ty, tz, "target")) != BLTC_OK)
        return rc;
    if ((rc = check_finite(ns, sx, sy, sz, "source")) != BLTC_OK)
        return rc;
    bltc_plan* plan = new (std::nothrow) bltc_plan();
    if (!plan)
        return fail(BLTC_ENOMEM, "cannot allocate plan");
    plan->prm = *p;
    plan->max_q = max_q;
    plan->limit = p->workspace_limit;
    try {
        if (p->method == BLTC_CLUSTER_PARTICLE)
            rc = bltc_cp::create_host(plan, plan_params(plan, p), nt, tx, ty, tz, ns, sx, sy, sz);
        else if (p->method == BLTC_CLUSTER_CLUSTER)
            rc = bltc_cc::create_host(plan, plan_params(plan, p), nt, tx, ty, tz, ns, sx, sy, sz);
        else
            rc = make_host_plan(plan, p, nt, tx, ty, tz, ns, sx, sy, sz);
        if (rc == BLTC_OK)
            rc = bltc_internal_check_mixed_extent(plan);
    } catch (const std::bad_alloc&) {
        rc = fail(BLTC_ENOMEM, "host allocation failed while planning");
    } catch (const std::exception& ex) {
        rc = fail(BLTC_EINTERNAL, "planning failed: %s", ex.what());
    }
    if (rc != BLTC_OK) {
        delete plan;
        return rc;
    }
    *out = plan;
    return BLTC_OK;
}

}  // namespace

int bltc_internal_upload_symmetric(bltc_plan* plan, bltc::DevicePlan& d,
                                   const bltc::DirectLists& dl, std::vector<int64_t>* cost,
                                   hipStream_t s)
{
    const int64_t sub = plan->prm.precision == BLTC_FP32_MIXED ? bltc::kSymTargetsMixed
                                                               : bltc::kSymTargetsF64;
    // every mutual pair whose results fit in a quarter of the round workspace
    bltc::SymPlan sp;
    if (!bltc::plan_symmetric(dl, sub, INT64_MAX, kPairWorkspaceBytes / 4 / sizeof(double), sp))
        return BLTC_OK;
    if (&d == &plan->d) {
        plan->sym_near_off_h = sp.near_off;
        plan->sym_pc_off_h = sp.pc_off;
    }
    HIP_TRY(plan->put(&d.sym_near_off, sp.near_off, s));
    HIP_TRY(plan->put(&d.sym_near_begin, sp.near_begin, s));
    HIP_TRY(plan->put(&d.sym_near_count, sp.near_count, s));
    HIP_TRY(plan->put(&d.sym_near_leaf, sp.near_leaf, s));
    HIP_TRY(plan->put(&d.sym_pc_off, sp.pc_off, s));
    HIP_TRY(plan->put(&d.sym_pc_base, sp.pc_base, s));
    HIP_TRY(plan->put(&d.batch_begin, *dl.batch_begin, s));
    HIP_TRY(hipStreamSynchronize(s));
    d.sym = 1;
    d.sym_rounds = 1;
    plan->sym_pair_evals = sp.pair_evals;
    *cost = sp.batch_cost;
    bltc_plan::Pairs& pr = plan->pairs;
    pr.d = &d;
    pr.batch_begin = *dl.batch_begin;
    pr.batch_count = *dl.batch_count;
    pr.batch_node = *dl.batch_node;
    pr.count = static_cast<int64_t>(sp.ub.size());
    pr.sp = std::move(sp);
    pr.pending = true;
    return BLTC_OK;
}

int bltc_internal_finish_pairs(bltc_plan* plan, hipStream_t s)
{
    bltc_plan::Pairs& pr = plan->pairs;
    if (!pr.pending)
        return BLTC_OK;
    bltc::DevicePlan& d = *pr.d;
    const bltc::SymPlan& sp = pr.sp;
    const int64_t nb = static_cast<int64_t>(pr.batch_begin.size());
    const int64_t nu = static_cast<int64_t>(sp.ub.size());
    const int64_t sub = sp.sub;
    int64_t nsubunits = 0;
    for (int64_t k = 0; k < nu; ++k)
        nsubunits += sp.nsub[k];
    const int64_t units_bytes = nsubunits * static_cast<int64_t>(sizeof(bltc::SymUnit));
    const int64_t full_bytes = sp.out_size * static_cast<int64_t>(sizeof(double));
    const int64_t left = plan->limit > 0 ? plan->limit - plan->bytes : INT64_MAX;
    // one round: the whole result array; rounds: a workspace, the per-target
    // sums, the per-round fold tables and the batch ranges
    std::vector<int32_t> round_unit;
    std::vector<int64_t> base;
    int64_t ws_values = sp.out_size;
    if (full_bytes + units_bytes <= std::min<int64_t>(kPairWorkspaceBytes, left)) {
        round_unit = {0, static_cast<int32_t>(nu)};
        base = {0, sp.out_size};
    } else {
        int64_t ntgt = 0;
        for (int64_t b = 0; b < nb; ++b)
            ntgt = std::max(ntgt, pr.batch_begin[b] + pr.batch_count[b]);
        const int64_t npc = nb > 0 ? sp.pc_off[nb] : 0;
        // pieces of several lanes per target read the sums through their own table
        const int64_t piece_bytes = (&d == &plan->d && plan->tpt > 1) ? (nb * plan->tpt + 1) * 4 : 0;
        const int64_t fixed = units_bytes + ntgt * 8 + nb * 8 + npc * 8 + (nb + 1) * 4 + piece_bytes;
        int64_t rounds = 1;
        for (int it = 0;; ++it) {
            const int64_t room = std::min<int64_t>(kPairWorkspaceBytes,
                                                   left - fixed - rounds * (nb + 1) * 4);
            const int64_t cap = room / static_cast<int64_t>(sizeof(double));
            if (cap < 1 || !bltc::plan_pair_rounds(sp, cap, round_unit, base))
                return bltc_detail::fail(
                    BLTC_ENOMEM,
                    "workspace_limit of %lld bytes leaves no room for the results of the "
                    "largest mutual leaf pair (%lld bytes held); raise the limit or set "
                    "no_symmetry",
                    static_cast<long long>(plan->limit), static_cast<long long>(plan->bytes));
            const int64_t r = static_cast<int64_t>(round_unit.size()) - 1;
            if (r <= rounds || it > 8) {
                ws_values = 0;
                for (int64_t k = 0; k < r; ++k)
                    ws_values = std::max(ws_values, base[k + 1] - base[k]);
                break;
            }
            rounds = r;
        }
    }
    const int32_t R = static_cast<int32_t>(round_unit.size()) - 1;
    // sub-units round by round, each round heaviest first, offsets relative
    // to the round's base; the rounds are built and sorted on host threads
    std::vector<int32_t> round_sub(static_cast<size_t>(R) + 1, 0);
    for (int32_t r = 0; r < R; ++r) {
        int64_t n = 0;
        for (int32_t k = round_unit[r]; k < round_unit[r + 1]; ++k)
            n += sp.nsub[k];
        round_sub[r + 1] = static_cast<int32_t>(round_sub[r] + n);
    }
    std::vector<bltc::SymUnit> units(static_cast<size_t>(nsubunits));
    bltc::parallel_each(R, [&](int64_t r) {
        size_t pos = static_cast<size_t>(round_sub[r]);
        for (int32_t k = round_unit[r]; k < round_unit[r + 1]; ++k) {
            const int32_t b = sp.ub[k], c = sp.uc[k];
            for (int32_t q = 0; q < sp.nsub[k]; ++q) {
                bltc::SymUnit& su = units[pos++];
                su.tb = pr.batch_begin[b] + q * sub;
                su.sb = pr.batch_begin[c];
                su.roff = sp.roff[k] - base[r] + q * sub;
                su.coff = sp.coff[k] - base[r] + q * pr.batch_count[c];
                su.nb = static_cast<int32_t>(std::min<int64_t>(sub, pr.batch_count[b] - q * sub));
                su.nc = static_cast<int32_t>(pr.batch_count[c]);
                su.batch = b;
                su.leaf = pr.batch_node[c];
                su.apart = sp.apart[k];
                su.pad = 0;
            }
        }
        // heaviest sub-unit first (one wave each)
        std::stable_sort(units.begin() + round_sub[r], units.begin() + round_sub[r + 1],
                         [](const bltc::SymUnit& a, const bltc::SymUnit& c) {
                             return static_cast<int64_t>(a.nb) * a.nc >
                                    static_cast<int64_t>(c.nb) * c.nc;
                         });
    });
    const int64_t held = plan->bytes;
    HIP_TRY(plan->put(&d.sym_unit, units, s));
    HIP_TRY(plan->alloc(&d.sym_out, static_cast<size_t>(ws_values)));
    d.sym_units = static_cast<int64_t>(units.size());
    if (R > 1) {
        // fold tables: per round and batch, the batch's result entries of that
        // round, rounds in order, batches in order, entries in list order
        // (counted and filled per batch on host threads)
        std::vector<int32_t> off(static_cast<size_t>(R) * (nb + 1), 0);
        auto round_of = [&](int64_t v) {
            return static_cast<int32_t>(std::upper_bound(base.begin(), base.end(), v) -
                                        base.begin()) - 1;
        };
        bltc::parallel_for(nb, [&](int64_t b) {
            for (int32_t e = sp.pc_off[b]; e < sp.pc_off[b + 1]; ++e)
                ++off[round_of(sp.pc_base[e]) * (nb + 1) + b];
        });
        int32_t total = 0;
        for (int32_t r = 0; r < R; ++r) {
            for (int64_t b = 0; b < nb; ++b) {
                const int32_t c = off[r * (nb + 1) + b];
                off[r * (nb + 1) + b] = total;
                total += c;
            }
            off[r * (nb + 1) + nb] = total;
        }
        std::vector<int64_t> fbase(static_cast<size_t>(total));
        bltc::parallel_for(nb, [&](int64_t b) {
            std::vector<int32_t> next(static_cast<size_t>(R));
            for (int32_t r = 0; r < R; ++r)
                next[r] = off[r * (nb + 1) + b];
            for (int32_t e = sp.pc_off[b]; e < sp.pc_off[b + 1]; ++e) {
                const int32_t r = round_of(sp.pc_base[e]);
                fbase[next[r]++] = sp.pc_base[e] - base[r];
            }
        });
        std::vector<int64_t> bend(static_cast<size_t>(nb));
        int64_t ntgt = 0;
        for (int64_t b = 0; b < nb; ++b) {
            bend[b] = pr.batch_begin[b] + pr.batch_count[b];
            ntgt = std::max(ntgt, bend[b]);
        }
        std::vector<int32_t> ident(static_cast<size_t>(nb) + 1);
        for (int64_t b = 0; b <= nb; ++b)
            ident[b] = static_cast<int32_t>(b);
        HIP_TRY(plan->put(&pr.fold_off, off, s));
        HIP_TRY(plan->put(&pr.fold_base, fbase, s));
        HIP_TRY(plan->put(&pr.batch_end, bend, s));
        HIP_TRY(plan->alloc(&d.sym_acc, static_cast<size_t>(ntgt)));
        // the interaction kernels read the per-target sums: one entry per batch
        int32_t* pc_off = nullptr;
        HIP_TRY(plan->put(&pc_off, ident, s));
        d.sym_pc_off = pc_off;
        d.sym_pc_base = d.batch_begin;
        if (&d == &plan->d)
            plan->sym_pc_off_h = ident;
        if (&d == &plan->d && plan->tpt > 1) {
            // pieces of several lanes per target: the sums go with piece 0
            const int32_t T = plan->tpt;
            std::vector<int32_t> pc_t(static_cast<size_t>(nb * T + 1), 0);
            for (int64_t b = 0; b < nb; ++b)
                for (int32_t p = 0; p < T; ++p)
                    pc_t[b * T + p] = p == 0 ? static_cast<int32_t>(b) : static_cast<int32_t>(b + 1);
            pc_t[nb * T] = static_cast<int32_t>(nb);
            HIP_TRY(plan->put(&plan->dt.sym_pc_off, pc_t, s));
            plan->dt.sym_pc_base = d.batch_begin;
        }
    }
    d.sym_rounds = R;
    if (&d == &plan->d && plan->tpt > 1) {
        plan->dt.sym_unit = d.sym_unit;
        plan->dt.sym_units = d.sym_units;
        plan->dt.sym_out = d.sym_out;
        plan->dt.sym_acc = d.sym_acc;
        plan->dt.sym_rounds = R;
    }
    HIP_TRY(hipStreamSynchronize(s));
    pr.round_unit = round_sub;
    pr.rounds = R;
    pr.workspace_bytes = plan->bytes - held;
    pr.pending = false;
    pr.sp = bltc::SymPlan();
    return BLTC_OK;
}

int bltc_internal_pairs(bltc_plan* plan, const bltc::DevicePlan& d, const bltc::KernelParams& kp,
                        hipStream_t s)
{
    if (!d.sym)
        return BLTC_OK;
    const bltc_plan::Pairs& pr = plan->pairs;
    if (pr.rounds <= 1) {
        HIP_TRY(bltc::launch_near_pairs(d, 0, d.sym_units, kp, s));
        return BLTC_OK;
    }
    const int64_t nb = static_cast<int64_t>(pr.batch_begin.size());
    for (int32_t r = 0; r < pr.rounds; ++r) {
        HIP_TRY(bltc::launch_near_pairs(d, pr.round_unit[r], pr.round_unit[r + 1] - pr.round_unit[r],
                                        kp, s));
        HIP_TRY(bltc::launch_fold_pairs(nb, d.batch_begin, pr.batch_end, pr.fold_off + r * (nb + 1),
                                        pr.fold_base, d.sym_out, d.sym_acc, r == 0, s));
    }
    return BLTC_OK;
}

int bltc_internal_check_direct(const bltc_params* p, int64_t nt, const double* tx,
                               const double* ty, const double* tz, int64_t ns, const double* sx,
                               const double* sy, const double* sz, const double* q, int32_t num_q,
                               const double* phi)
{
    int rc = check_params(p);
    if (rc != BLTC_OK)
        return rc;
    if ((rc = check_coords(nt, tx, ty, tz, "target")) != BLTC_OK)
        return rc;
    if ((rc = check_coords(ns, sx, sy, sz, "source")) != BLTC_OK)
        return rc;
    if (num_q < 1)
        return fail(BLTC_EINVAL, "num_q must be >= 1");
    if (nt > 0 && !phi)
        return fail(BLTC_EINVAL, "phi is NULL");
    if (nt > 0 && ns > 0 && !q)
        return fail(BLTC_EINVAL, "q is NULL");
    return BLTC_OK;
}

extern "C" {

void bltc_params_default(bltc_params* p)
{
    if (!p)
        return;
    std::memset(p, 0, sizeof(*p));
    p->kernel = BLTC_COULOMB;
    p->precision = BLTC_FP64;
    p->kappa = 0.0;
    p->theta = 0.7;
    p->degree = 8;
    p->leaf_size = 2000;
    p->batch_size = 2000;
    p->threads_per_target = 1;
    p->method = BLTC_PARTICLE_CLUSTER;
    p->delta = 0.0;
    p->workspace_limit = 0;
}

int bltc_plan_create_host(bltc_plan** out, const bltc_params* p, int64_t nt, const double* tx,
                          const double* ty, const double* tz, int64_t ns, const double* sx,
                          const double* sy, const double* sz, int32_t max_q)
{
    int rc = create_common(out, p, nt, tx, ty, tz, ns, sx, sy, sz, max_q);
    if (rc != BLTC_OK)
        return rc;
    return create_from_host(out, p, nt, tx, ty, tz, ns, sx, sy, sz, max_q);
}

int bltc_plan_create(bltc_plan** out, const bltc_params* p_in, int64_t nt, const double* tx,
                     const double* ty, const double* tz, int64_t ns, const double* sx,
                     const double* sy, const double* sz, int32_t max_q, void* stream)
{
    int rc = create_common(out, p_in, nt, tx, ty, tz, ns, sx, sy, sz, max_q);
    if (rc != BLTC_OK)
        return rc;
    // sizes or threads per target left open: the tuner times plans first
    bltc_params tuned;
    try {
        rc = bltc_internal_tune(p_in, nt, tx, ty, tz, ns, sx, sy, sz, max_q, &tuned, stream);
    } catch (const std::bad_alloc&) {
        rc = fail(BLTC_ENOMEM, "host allocation failed while tuning");
    } catch (const std::exception& ex) {
        rc = fail(BLTC_EINTERNAL, "tuning failed: %s", ex.what());
    }
    if (rc != BLTC_OK)
        return rc;
    if (tuned.leaf_size == 0) {
        // nothing to time on (no targets or no sources): the default size
        tuned.leaf_size = tuned.batch_size = 2000;
    }
    const bltc_params* p = &tuned;
    hipStream_t s = static_cast<hipStream_t>(stream);
    bltc_plan* plan = new (std::nothrow) bltc_plan();
    if (!plan)
        return fail(BLTC_ENOMEM, "cannot allocate plan");
    plan->prm = *p;
    plan->max_q = max_q;
    plan->limit = p->workspace_limit;
    try {
        if (p->method == BLTC_CLUSTER_PARTICLE)
            rc = bltc_cp::create_device(plan, plan_params(plan, p), nt, tx, ty, tz, ns, sx, sy, sz, s);
        else if (p->method == BLTC_CLUSTER_CLUSTER)
            rc = bltc_cc::create_device(plan, plan_params(plan, p), nt, tx, ty, tz, ns, sx, sy, sz, s);
        else
            rc = make_device_plan(plan, p, nt, tx, ty, tz, ns, sx, sy, sz, s);
        if (rc == BLTC_OK)
            rc = bltc_internal_upload_plan(plan, s);
    } catch (const std::bad_alloc&) {
        rc = fail(BLTC_ENOMEM, "host allocation failed while planning");
    } catch (const std::exception& ex) {
        rc = fail(BLTC_EINTERNAL, "planning failed: %s", ex.what());
    }
    if (rc != BLTC_OK) {
        delete plan;
        return rc;
    }
    *out = plan;
    return BLTC_OK;
}

int bltc_plan_execute(bltc_plan* plan, const double* q, int32_t num_q, int64_t q_ld, double* phi,
                      int64_t phi_ld, void* stream)
{
    if (!plan)
        return fail(BLTC_EINVAL, "plan is NULL");
    try {
        return execute(plan, q, num_q, q_ld, phi, phi_ld, static_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc&) {
        return fail(BLTC_ENOMEM, "host allocation failed");
    } catch (const std::exception& ex) {
        return fail(BLTC_EINTERNAL, "%s", ex.what());
    }
}

int bltc_potential(const bltc_params* p, int64_t nt, const double* tx, const double* ty,
                   const double* tz, int64_t ns, const double* sx, const double* sy,
                   const double* sz, const double* q, int32_t num_q, int64_t q_ld, double* phi,
                   int64_t phi_ld, void* stream)
{
    if (nt == 0) {
        int rc = check_params(p);
        return rc != BLTC_OK ? rc : BLTC_OK;
    }
    if (num_q < 1)
        return fail(BLTC_EINVAL, "num_q must be >= 1");
    bltc_plan* plan = nullptr;
    int rc = bltc_plan_create(&plan, p, nt, tx, ty, tz, ns, sx, sy, sz, num_q, stream);
    if (rc != BLTC_OK)
        return rc;
    rc = bltc_plan_execute(plan, q, num_q, q_ld, phi, phi_ld, stream);
    if (rc == BLTC_OK) {
        hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
        if (e != hipSuccess)
            rc = hip_fail(e, "hipStreamSynchronize");
    }
    bltc_plan_destroy(plan);
    return rc;
}

int bltc_plan_modified_charges(bltc_plan* plan, int64_t cluster, int32_t qi, double* out,
                               void* stream)
{
    if (!plan || !out)
        return fail(BLTC_EINVAL, "NULL argument");
    if (plan->cp || plan->cc) {
        if (qi != 0)
            return fail(BLTC_EINVAL, "cluster-particle and cluster-cluster plans have one charge vector");
        return plan->cp ? bltc_cp::proxy_potentials(plan, cluster, out, static_cast<hipStream_t>(stream))
                        : bltc_cc::proxy_potentials(plan, cluster, out, static_cast<hipStream_t>(stream));
    }
    const bltc::HostPlan& hp = plan->hp;
    if (cluster < 0 || cluster >= hp.src.nodes())
        return fail(BLTC_EINVAL, "cluster index out of range");
    if (qi < 0 || qi >= plan->max_q)
        return fail(BLTC_EINVAL, "charge-vector index out of range");
    const int32_t slot = hp.cluster_slot[cluster];
    if (slot < 0)
        return fail(BLTC_EINVAL, "cluster %lld has no modified charges",
                    static_cast<long long>(cluster));
    if (!plan->uploaded || plan->last_q == 0)
        return fail(BLTC_EINVAL, "plan has not been executed");
    // one vector: qhat[slot][k]; several: the last pass of 16, qhat16[slot][k][m]
    const int32_t m0 = plan->last_q == 1 ? 0 : 16 * ((plan->last_q - 1) / 16);
    if (qi < m0 || qi >= plan->last_q)
        return fail(BLTC_EINVAL, "charge vector %d is not in the last execution's last pass", qi);
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::vector<double> buf(plan->last_q == 1 ? hp.P : hp.P * 16);
    // Hermite: the charges regrouped per grid point, [slot][k][a]
    const double* src = (plan->d.hermite ? plan->d.qhat_h : plan->d.qhat) +
                        static_cast<int64_t>(slot) * static_cast<int64_t>(buf.size());
    HIP_TRY(hipMemcpyAsync(buf.data(), src, buf.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int64_t k = 0; k < hp.P; ++k)
        out[k] = plan->last_q == 1 ? buf[k] : buf[k * 16 + (qi - m0)];
    return BLTC_OK;
}

namespace {

void pair_stats(const bltc_plan* plan, bltc_stats* out)
{
    out->workspace_bytes = plan->bytes;
    out->mutual_pairs = plan->pairs.count;
    out->pair_workspace_bytes = plan->pairs.workspace_bytes;
    out->pair_rounds = plan->pairs.rounds;
}

}  // namespace

int bltc_plan_stats(const bltc_plan* plan, bltc_stats* out)
{
    if (!plan || !out)
        return fail(BLTC_EINVAL, "NULL argument");
    const bltc::HostPlan& hp = plan->hp;
    std::memset(out, 0, sizeof(*out));
    if (plan->cp || plan->cc) {
        if (plan->cp)
            bltc_cp::stats(plan, out);
        else
            bltc_cc::stats(plan, out);
        out->degree = plan->prm.degree;
        out->leaf_size = plan->prm.leaf_size;
        out->batch_size = plan->prm.batch_size;
        out->mutual_pair_evals = plan->sym_pair_evals;
        out->threads_per_target = 1;
        pair_stats(plan, out);
        return BLTC_OK;
    }
    out->clusters = hp.src.nodes();
    out->leaves = hp.leaves;
    out->batches = static_cast<int64_t>(hp.batch_begin.size());
    out->approx_pairs = hp.approx_pairs;
    out->direct_pairs = hp.direct_pairs;
    out->approx_clusters = static_cast<int64_t>(hp.slot_cluster.size());
    out->far_evals = hp.far_evals;
    out->near_evals = hp.near_evals;
    out->upward_terms = hp.upward_terms;
    out->depth = hp.src.depth;
    out->degree = plan->prm.degree;
    out->leaf_size = plan->prm.leaf_size;
    out->batch_size = plan->prm.batch_size;
    out->setup_seconds = hp.setup_seconds;
    out->mutual_pair_evals = plan->sym_pair_evals;
    out->threads_per_target = std::max(1, plan->prm.threads_per_target);
    pair_stats(plan, out);
    return BLTC_OK;
}

int bltc_plan_view_get(const bltc_plan* plan, bltc_plan_view* out)
{
    if (!plan || !out)
        return fail(BLTC_EINVAL, "NULL argument");
    const bltc::HostPlan& hp = plan->hp;
    std::memset(out, 0, sizeof(*out));
    if (plan->cp)
        return bltc_cp::view(plan, out);
    if (plan->cc)
        return bltc_cc::view(plan, out);
    out->nt = hp.tgt.n;
    out->ns = hp.src.n;
    out->n_clusters = hp.src.nodes();
    out->n_batches = static_cast<int64_t>(hp.batch_begin.size());
    out->n_items = plan->device_lists ? plan->n_items : static_cast<int64_t>(hp.item_batch.size());
    out->source_order = hp.src.order.data();
    out->target_order = hp.tgt.order.data();
    if (plan->device_particles) {
        // tree orders live on the device: copy them once
        if (plan->view_src_order.size() != static_cast<size_t>(hp.src.n)) {
            plan->view_src_order.resize(hp.src.n);
            plan->view_tgt_order.resize(hp.tgt.n);
            if (hp.src.n > 0)
                HIP_TRY(hipMemcpy(plan->view_src_order.data(), plan->d.src_order,
                                  hp.src.n * sizeof(int64_t), hipMemcpyDeviceToHost));
            if (hp.tgt.n > 0)
                HIP_TRY(hipMemcpy(plan->view_tgt_order.data(), plan->d.tgt_orig,
                                  hp.tgt.n * sizeof(int64_t), hipMemcpyDeviceToHost));
        }
        out->source_order = plan->view_src_order.data();
        out->target_order = plan->view_tgt_order.data();
    }
    out->cluster_begin = hp.src.begin.data();
    out->cluster_count = hp.src.count.data();
    out->cluster_lo = hp.src.lo.data();
    out->cluster_hi = hp.src.hi.data();
    out->cluster_first_child = hp.src.first_child.data();
    out->cluster_nchild = hp.src.nchild.data();
    out->cluster_level = hp.src.level.data();
    out->batch_begin = hp.batch_begin.data();
    out->batch_count = hp.batch_count.data();
    out->batch_lo = hp.batch_lo.data();
    out->batch_hi = hp.batch_hi.data();
    out->item_batch = hp.item_batch.data();
    out->item_cluster = hp.item_cluster.data();
    out->item_kind = hp.item_kind.data();
    if (plan->device_lists) {
        if (plan->view_item_batch.size() != static_cast<size_t>(plan->n_items)) {
            const size_t ni = static_cast<size_t>(plan->n_items);
            plan->view_item_batch.resize(ni);
            plan->view_item_cluster.resize(ni);
            plan->view_item_kind.resize(ni);
            if (ni > 0) {
                HIP_TRY(hipMemcpy(plan->view_item_batch.data(), plan->item_batch,
                                  ni * sizeof(int32_t), hipMemcpyDeviceToHost));
                HIP_TRY(hipMemcpy(plan->view_item_cluster.data(), plan->item_cluster,
                                  ni * sizeof(int32_t), hipMemcpyDeviceToHost));
                HIP_TRY(hipMemcpy(plan->view_item_kind.data(), plan->item_kind,
                                  ni * sizeof(int32_t), hipMemcpyDeviceToHost));
            }
        }
        out->item_batch = plan->view_item_batch.data();
        out->item_cluster = plan->view_item_cluster.data();
        out->item_kind = plan->view_item_kind.data();
    }
    return BLTC_OK;
}

int bltc_plan_set_timing(bltc_plan* plan, int32_t enable)
{
    if (!plan)
        return fail(BLTC_EINVAL, "plan is NULL");
    plan->timing = enable != 0;
    plan->timed_q = 0;
    return BLTC_OK;
}

int bltc_plan_phase_times(bltc_plan* plan, double* ms)
{
    if (!plan || !ms)
        return fail(BLTC_EINVAL, "NULL argument");
    if (!plan->timing || plan->timed_q == 0)
        return fail(BLTC_EINVAL, "no timed execution (enable timing, then execute)");
    double acc[3] = {0.0, 0.0, 0.0};
    for (int32_t m = 0; m < plan->timed_q; ++m) {
        HIP_TRY(hipEventSynchronize(plan->events[4 * m + 3]));
        for (int k = 0; k < 3; ++k) {
            float t = 0.0f;
            HIP_TRY(hipEventElapsedTime(&t, plan->events[4 * m + k], plan->events[4 * m + k + 1]));
            acc[k] += t;
        }
    }
    for (int k = 0; k < 3; ++k)
        ms[k] = acc[k];
    ms[3] = acc[0] + acc[1] + acc[2];
    ms[4] = 0.0;
    if (plan->timed_pairs) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, plan->events[2], plan->ev_pairs));
        ms[4] = t;
    }
    return BLTC_OK;
}

void bltc_plan_destroy(bltc_plan* plan)
{
    delete plan;
}

int bltc_direct(const bltc_params* p, int64_t nt, const double* tx, const double* ty,
                const double* tz, int64_t ns, const double* sx, const double* sy, const double* sz,
                const double* q, int32_t num_q, int64_t q_ld, double* phi, int64_t phi_ld,
                void* stream)
{
    int rc = bltc_internal_check_direct(p, nt, tx, ty, tz, ns, sx, sy, sz, q, num_q, phi);
    if (rc != BLTC_OK)
        return rc;
    if (nt == 0)
        return BLTC_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ns == 0)
        return zero_phi(nt, num_q, phi, phi_ld, s);
    double4* packed = nullptr;
    HIP_TRY(hipMallocAsync(reinterpret_cast<void**>(&packed), ns * sizeof(double4), s));
    bltc::KernelParams kp;
    kp.kernel = p->kernel;
    kp.kappa = p->kappa;
    kp.delta = p->delta;
    hipError_t e = hipSuccess;
    for (int32_t m = 0; m < num_q && e == hipSuccess; ++m) {
        e = bltc::launch_pack_sources(ns, sx, sy, sz, q + static_cast<int64_t>(m) * q_ld, packed, s);
        if (e == hipSuccess)
            e = bltc::launch_direct(nt, tx, ty, tz, ns, packed, kp,
                                    phi + static_cast<int64_t>(m) * phi_ld, s);
    }
    hipError_t f = hipFreeAsync(packed, s);
    if (e != hipSuccess)
        return hip_fail(e, "direct-sum launch");
    if (f != hipSuccess)
        return hip_fail(f, "hipFreeAsync");
    return BLTC_OK;
}

const char* bltc_status_string(int code)
{
    switch (code) {
    case BLTC_OK: return "ok";
    case BLTC_EINVAL: return "invalid argument";
    case BLTC_ENOMEM: return "out of memory";
    case BLTC_EHIP: return "HIP runtime error";
    case BLTC_EUNSUPPORTED: return "unsupported";
    case BLTC_EINTERNAL: return "internal error";
    default: return "unknown status";
    }
}

const char* bltc_last_error(void)
{
    return bltc_detail::last_error().c_str();
}

const char* bltc_version(void)
{
    return "bltc-mi355x 0.1 (gfx950)";
}

}  // extern "C"
