// cp.cpp -- plans of the cluster-particle treecode (method
// BLTC_CLUSTER_PARTICLE): the barycentric interpolation of Sec. II applied to
// the target variable.
//
// Device layout:
//  * proxy potentials (their own kernel, kernels_cp.hip): one "batch" per
//    target cluster that some source batch approximates, its list holding
//    those source batches; the result is phat[slot][k] at the cluster's
//    (n+1)^3 Chebyshev points;
//  * direct sums (the interaction kernels): the targets in target-tree
//    order, one batch per target leaf, lists holding the source batches of
//    the direct pairs of every cluster on the leaf's root-to-leaf path; phi
//    is written once;
// and then interpolate_targets adds, for every target, the interpolant of the
// proxy potentials of each cluster on its path (kernels_cp.hip).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "internal.hpp"
#include "kernels_cp.hpp"
#include "setup_gpu.hpp"

using bltc_detail::fail;

namespace bltc_cp {

// pieces of the proxy-potential lists (one wave per piece and part of the
// grid): at least this many sources each, and about kProxyPieces in all
constexpr int64_t kProxyPieceSources = 8192;
constexpr int64_t kProxyPieces = 16384;

int upload_pieces(bltc_plan* plan, bltc::DevicePlan& d, const std::vector<int32_t>& off,
                  const std::vector<int64_t>& count, int64_t* rows, hipStream_t s)
{
    const int64_t nslots = static_cast<int64_t>(off.size()) - 1;
    int64_t listed = 0;
    for (const int64_t c : count)
        listed += c;
    const int64_t piece = std::max(kProxyPieceSources, (listed + kProxyPieces - 1) / kProxyPieces);
    std::vector<int32_t> piece_slot, slot_piece_off(nslots + 1, 0);
    std::vector<int64_t> piece_entry, piece_entries, piece_row;
    int64_t nrows = nslots;
    for (int64_t sl = 0; sl < nslots; ++sl) {
        const size_t first = piece_slot.size();
        int32_t e0 = off[sl];
        int64_t run = 0;
        for (int32_t e = off[sl]; e < off[sl + 1]; ++e) {
            if (run > 0 && run + count[e] > piece) {
                piece_slot.push_back(static_cast<int32_t>(sl));
                piece_entry.push_back(e0);
                piece_entries.push_back(e - e0);
                e0 = e;
                run = 0;
            }
            run += count[e];
        }
        piece_slot.push_back(static_cast<int32_t>(sl));
        piece_entry.push_back(e0);
        piece_entries.push_back(off[sl + 1] - e0);
        const size_t np_sl = piece_slot.size() - first;
        for (size_t k = 0; k < np_sl; ++k)
            piece_row.push_back(np_sl == 1 ? sl : nrows++);
        slot_piece_off[sl + 1] = static_cast<int32_t>(piece_slot.size());
    }
    d.nslots = nslots;
    d.nchunks = static_cast<int64_t>(piece_slot.size());
    HIP_TRY(plan->put(&d.chunk_slot, piece_slot, s));
    HIP_TRY(plan->put(&d.chunk_begin, piece_entry, s));
    HIP_TRY(plan->put(&d.chunk_count, piece_entries, s));
    HIP_TRY(plan->put(&d.chunk_dst, piece_row, s));
    HIP_TRY(plan->put(&d.slot_chunk_off, slot_piece_off, s));
    *rows = nrows;
    return BLTC_OK;
}

int create_host(bltc_plan* plan, const bltc::PlanParams& pp, int64_t nt, const double* tx,
                const double* ty, const double* tz, int64_t ns, const double* sx, const double* sy,
                const double* sz)
{
    plan->cp = true;
    bltc::make_cp_plan(plan->cpp, pp, nt, tx, ty, tz, ns, sx, sy, sz);
    return BLTC_OK;
}

int create_device(bltc_plan* plan, const bltc::PlanParams& pp, int64_t nt, const double* tx,
                  const double* ty, const double* tz, int64_t ns, const double* sx,
                  const double* sy, const double* sz, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    plan->cp = true;
    bltc::CpPlan& cp = plan->cpp;
    cp = bltc::CpPlan();
    cp.prm = pp;
    const bool mixed = plan->prm.precision == BLTC_FP32_MIXED;
    HIP_TRY(hipGetDevice(&plan->device));
    bltc::DevicePlan& px = plan->dprox;
    bltc::DevicePlan& dd = plan->ddir;
    int64_t* src_order = nullptr;
    HIP_TRY(plan->alloc(&px.src, static_cast<size_t>(ns)));
    HIP_TRY(plan->alloc(&src_order, static_cast<size_t>(ns)));
    px.src_order = src_order;
    if (mixed)
        HIP_TRY(plan->alloc(&px.src32, static_cast<size_t>(ns)));
    HIP_TRY(plan->alloc(&dd.tgt, static_cast<size_t>(nt)));
    HIP_TRY(plan->alloc(&dd.tgt_orig, static_cast<size_t>(nt)));
    int64_t bad = -1;
    std::string err = bltc::build_tree_device(cp.tgt, nt, tx, ty, tz, pp.leaf_size, dd.tgt_orig,
                                              dd.tgt, nullptr, s, &bad);
    if (bad >= 0)
        return fail(BLTC_EINVAL, "target coordinate %lld is not finite", static_cast<long long>(bad));
    if (!err.empty())
        return fail(BLTC_EHIP, "device tree build: %s", err.c_str());
    err = bltc::build_tree_device(cp.src, ns, sx, sy, sz, pp.batch_size, src_order, px.src,
                                  mixed ? px.src32 : nullptr, s, &bad);
    if (bad >= 0)
        return fail(BLTC_EINVAL, "source coordinate %lld is not finite", static_cast<long long>(bad));
    if (!err.empty())
        return fail(BLTC_EHIP, "device tree build: %s", err.c_str());
    cp.same_arrays = nt == ns && tx == sx && ty == sy && tz == sz && pp.batch_size == pp.leaf_size;
    bltc::cp_plan_from_trees(cp);
    plan->device_particles = true;
    cp.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return BLTC_OK;
}

namespace {

bool same_nodes(const bltc::Tree& a, const bltc::Tree& b)
{
    return a.n == b.n && a.begin == b.begin && a.count == b.count && a.nchild == b.nchild &&
           a.first_child == b.first_child && a.lo == b.lo && a.hi == b.hi;
}

// Both trees of a device-built plan come from the same arrays with the same
// capacity: the build is deterministic, and this confirms it (node arrays and
// particle orders equal) before the one-tree evaluation relies on it.
int confirm_same_tree(bltc_plan* plan)
{
    bltc::CpPlan& cp = plan->cpp;
    if (!cp.same_arrays || cp.same_tree || !same_nodes(cp.src, cp.tgt))
        return BLTC_OK;
    const int64_t n = cp.src.n;
    std::vector<int64_t> a(n), b(n);
    if (n > 0) {
        HIP_TRY(hipMemcpy(a.data(), plan->dprox.src_order, n * sizeof(int64_t),
                          hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(b.data(), plan->ddir.tgt_orig, n * sizeof(int64_t),
                          hipMemcpyDeviceToHost));
    }
    cp.same_tree = a == b;
    return BLTC_OK;
}

}  // namespace

int upload(bltc_plan* plan, hipStream_t s)
{
    if (plan->uploaded)
        return BLTC_OK;
    bltc::CpPlan& cp = plan->cpp;
    const bool mixed = plan->prm.precision == BLTC_FP32_MIXED;
    bltc::DevicePlan& px = plan->dprox;
    bltc::DevicePlan& dd = plan->ddir;
    HIP_TRY(hipGetDevice(&plan->device));
    const int64_t nt = cp.tgt.n, ns = cp.src.n;
    const int64_t nslots = static_cast<int64_t>(cp.slot_cluster.size());
    const int64_t ntl = static_cast<int64_t>(cp.tl_node.size());
    const int32_t np = cp.np;
    const int64_t P = cp.P;

    // particles in tree order (host-built plans)
    if (!plan->device_particles) {
        std::vector<double4> src(ns), tgt(nt);
        for (int64_t j = 0; j < ns; ++j)
            src[j] = make_double4(cp.src.x[j], cp.src.y[j], cp.src.z[j], 0.0);
        for (int64_t i = 0; i < nt; ++i)
            tgt[i] = make_double4(cp.tgt.x[i], cp.tgt.y[i], cp.tgt.z[i], 0.0);
        HIP_TRY(plan->put(&px.src, src, s));
        HIP_TRY(plan->put(&dd.tgt, tgt, s));
        HIP_TRY(plan->put(&dd.tgt_orig, cp.tgt.order, s));
        int64_t* src_order = nullptr;
        HIP_TRY(plan->put(&src_order, cp.src.order, s));
        px.src_order = src_order;
        if (mixed) {
            // sources relative to the center of their source batch
            std::vector<float4> src32(ns);
            for (size_t b = 0; b < cp.sb_node.size(); ++b) {
                const int32_t u = cp.sb_node[b];
                const double cx = cp.src.center[3 * u], cy = cp.src.center[3 * u + 1],
                             cz = cp.src.center[3 * u + 2];
                for (int64_t j = cp.sb_begin[b]; j < cp.sb_begin[b] + cp.sb_count[b]; ++j)
                    src32[j] = make_float4(static_cast<float>(cp.src.x[j] - cx),
                                           static_cast<float>(cp.src.y[j] - cy),
                                           static_cast<float>(cp.src.z[j] - cz), 0.0f);
            }
            HIP_TRY(plan->put(&px.src32, src32, s));
        }
        HIP_TRY(hipStreamSynchronize(s));
    }
    dd.src = px.src;
    dd.src_order = px.src_order;
    dd.src32 = px.src32;
    px.degree = dd.degree = plan->prm.degree;
    px.ns = dd.ns = ns;

    // proxy potentials: one "batch" per slot, its list the source batches
    // approximated with the slot's cluster; the proxy points are formed from
    // the slot's grid inside the kernel
    std::vector<int64_t> leaf_end(ntl);
    for (int64_t t = 0; t < ntl; ++t)
        leaf_end[t] = cp.tl_begin[t] + cp.tl_count[t];
    const std::vector<int32_t> far_off_d(ntl + 1, 0), one_i(1, 0);
    const std::vector<double> one_d(1, 0.0);

    px.nt = nslots * P;
    px.nbatches = nslots;
    px.ngroups = 0;
    HIP_TRY(plan->put(&px.near_begin, cp.pf_begin, s));
    HIP_TRY(plan->put(&px.near_count, cp.pf_count, s));
    HIP_TRY(plan->put(&px.near_leaf, cp.pf_leaf, s));
    int64_t rows = 0;
    int rc = upload_pieces(plan, px, cp.pf_off, cp.pf_count, &rows, s);
    if (rc != BLTC_OK)
        return rc;
    HIP_TRY(plan->put(&px.slot_nodes, one_d, s));
    HIP_TRY(plan->put(&px.qhat, one_d, s));

    dd.nt = nt;
    dd.nslots = 0;
    dd.nbatches = ntl;
    dd.ngroups = static_cast<int64_t>(cp.dg_batch.size());
    HIP_TRY(plan->put(&dd.group_batch, cp.dg_batch, s));
    HIP_TRY(plan->put(&dd.group_first, cp.dg_first, s));
    HIP_TRY(plan->put(&dd.batch_end, leaf_end, s));
    HIP_TRY(plan->put(&dd.far_off, far_off_d, s));
    HIP_TRY(plan->put(&dd.far_slot, one_i, s));
    HIP_TRY(plan->put(&dd.near_off, cp.dn_off, s));
    HIP_TRY(plan->put(&dd.near_begin, cp.dn_begin, s));
    HIP_TRY(plan->put(&dd.near_count, cp.dn_count, s));
    HIP_TRY(plan->put(&dd.near_leaf, cp.dn_leaf, s));
    dd.slot_nodes = px.slot_nodes;
    dd.qhat = px.qhat;

    HIP_TRY(plan->put(&plan->cp_path_off, cp.dw_off, s));
    HIP_TRY(plan->put(&plan->cp_path_slot, cp.dw_slot, s));
    HIP_TRY(plan->put(&plan->cp_slot_nodes, cp.slot_nodes, s));
    HIP_TRY(plan->alloc(&plan->cp_phat, static_cast<size_t>(rows * P)));

    if (mixed) {
        // per source node (the lists name source leaves): center and radius;
        // per batch of each launch: the target cluster's center and radius
        const int64_t nn = cp.src.nodes();
        std::vector<double4> node_info(nn);
        for (int64_t c = 0; c < nn; ++c)
            node_info[c] = make_double4(cp.src.center[3 * c], cp.src.center[3 * c + 1],
                                        cp.src.center[3 * c + 2], cp.src.radius[c]);
        std::vector<double4> bi_p(nslots), bi_d(ntl);
        for (int64_t sl = 0; sl < nslots; ++sl) {
            const int32_t c = cp.slot_cluster[sl];
            bi_p[sl] = make_double4(cp.tgt.center[3 * c], cp.tgt.center[3 * c + 1],
                                    cp.tgt.center[3 * c + 2], cp.tgt.radius[c]);
        }
        for (int64_t t = 0; t < ntl; ++t) {
            const int32_t c = cp.tl_node[t];
            bi_d[t] = make_double4(cp.tgt.center[3 * c], cp.tgt.center[3 * c + 1],
                                   cp.tgt.center[3 * c + 2], cp.tgt.radius[c]);
        }
        HIP_TRY(plan->put(&px.node_info, node_info, s));
        dd.node_info = px.node_info;
        HIP_TRY(plan->put(&px.batch_info, bi_p, s));
        HIP_TRY(plan->put(&dd.batch_info, bi_d, s));
        HIP_TRY(plan->alloc(&px.qhat32, 1));
        dd.qhat32 = px.qhat32;
    }
    // targets are the sources: mutual direct leaf pairs once for both directions,
    // and the target-leaf workgroups (one wave each) re-ordered by the work left
    if (cp.same_arrays && !plan->prm.no_symmetry) {
        int rc = plan->device_particles ? confirm_same_tree(plan) : BLTC_OK;
        if (rc != BLTC_OK)
            return rc;
    }
    if (cp.same_tree && !plan->prm.no_symmetry) {
        const bltc::DirectLists dl{&cp.src,    &cp.tl_node, &cp.tl_begin, &cp.tl_count,
                                   &cp.dn_off, &cp.dn_leaf, &cp.dn_cost};
        int rc = bltc_internal_upload_symmetric(plan, dd, dl, &cp.dn_cost, s);
        if (rc != BLTC_OK)
            return rc;
        if (dd.sym) {
            cp.dg_batch.clear();
            cp.dg_first.clear();
            bltc::group_schedule(cp.tl_begin, cp.tl_count, cp.dn_cost, bltc::kGroupSizeSym,
                                 cp.prm.xcds, cp.dg_batch, cp.dg_first);
            HIP_TRY(plan->put(&dd.group_batch, cp.dg_batch, s));
            HIP_TRY(plan->put(&dd.group_first, cp.dg_first, s));
            dd.ngroups = static_cast<int64_t>(cp.dg_batch.size());
            dd.group_threads = bltc::kGroupSizeSym;
        }
    }
    // host staging vectors die at return: finish the copies first
    HIP_TRY(hipStreamSynchronize(s));
    plan->uploaded = true;
    return BLTC_OK;
}

int execute(bltc_plan* plan, const double* q, int32_t num_q, double* phi, hipStream_t s)
{
    if (num_q != 1)
        return fail(BLTC_EUNSUPPORTED, "cluster-particle plans take one charge vector");
    int rc = bltc_internal_upload_plan(plan, s);
    if (rc != BLTC_OK)
        return rc;
    bltc::KernelParams kp;
    kp.kernel = plan->prm.kernel;
    kp.precision = plan->prm.precision;
    kp.kappa = plan->prm.kappa;
    kp.delta = plan->prm.delta;
    const bool mixed = kp.precision == BLTC_FP32_MIXED;
    if (plan->timing) {
        while (plan->events.size() < 4) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            plan->events.push_back(e);
        }
    }
    auto mark = [&](int k) -> hipError_t {
        return plan->timing ? hipEventRecord(plan->events[k], s) : hipSuccess;
    };
    plan->timed_q = 0;
    HIP_TRY(mark(0));
    HIP_TRY(bltc::launch_gather_charges(plan->dprox, q, s));
    HIP_TRY(mark(1));
    HIP_TRY(bltc::launch_proxy_potentials(plan->dprox, plan->cp_slot_nodes, kp, plan->cp_phat, s));
    if (plan->dprox.nchunks != plan->dprox.nslots) {
        // clusters of several pieces: partial rows summed in piece order
        HIP_TRY(bltc::launch_upward_reduce(plan->dprox, 1, plan->cp_phat, nullptr, s));
    }
    HIP_TRY(mark(2));
    rc = bltc_internal_pairs(plan, plan->ddir, kp, s);
    if (rc != BLTC_OK)
        return rc;
    if (mixed)
        HIP_TRY(bltc::launch_interact_mixed(plan->ddir, kp, phi, s));
    else
        HIP_TRY(bltc::launch_interact(plan->ddir, kp, phi, s));
    HIP_TRY(bltc::launch_interpolate_targets(plan->ddir, plan->cp_path_off, plan->cp_path_slot,
                                             plan->cp_slot_nodes, plan->cp_phat, phi, s));
    HIP_TRY(mark(3));
    plan->timed_q = plan->timing ? 1 : 0;
    plan->last_q = 1;
    return BLTC_OK;
}

int proxy_potentials(bltc_plan* plan, int64_t cluster, double* out, hipStream_t s)
{
    const bltc::CpPlan& cp = plan->cpp;
    if (cluster < 0 || cluster >= cp.tgt.nodes())
        return fail(BLTC_EINVAL, "cluster index out of range");
    const int32_t slot = cp.cluster_slot[cluster];
    if (slot < 0)
        return fail(BLTC_EINVAL, "target cluster %lld has no proxy potentials",
                    static_cast<long long>(cluster));
    if (!plan->uploaded || plan->last_q == 0)
        return fail(BLTC_EINVAL, "plan has not been executed");
    HIP_TRY(hipMemcpyAsync(out, plan->cp_phat + static_cast<int64_t>(slot) * cp.P,
                           cp.P * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return BLTC_OK;
}

void stats(const bltc_plan* plan, bltc_stats* out)
{
    const bltc::CpPlan& cp = plan->cpp;
    out->clusters = cp.tgt.nodes();
    out->leaves = cp.leaves;
    out->batches = static_cast<int64_t>(cp.sb_node.size());
    out->approx_pairs = cp.approx_pairs;
    out->direct_pairs = cp.direct_pairs;
    out->approx_clusters = static_cast<int64_t>(cp.slot_cluster.size());
    out->far_evals = cp.proxy_evals;
    out->near_evals = cp.near_evals;
    out->upward_terms = cp.interp_terms;
    out->depth = cp.tgt.depth;
    out->setup_seconds = cp.setup_seconds;
}

int view(const bltc_plan* plan, bltc_plan_view* out)
{
    const bltc::CpPlan& cp = plan->cpp;
    out->nt = cp.tgt.n;
    out->ns = cp.src.n;
    out->n_clusters = cp.tgt.nodes();
    out->n_batches = static_cast<int64_t>(cp.sb_node.size());
    out->n_items = static_cast<int64_t>(cp.item_batch.size());
    out->source_order = cp.src.order.data();
    out->target_order = cp.tgt.order.data();
    if (plan->device_particles) {
        if (plan->view_src_order.size() != static_cast<size_t>(cp.src.n)) {
            plan->view_src_order.resize(cp.src.n);
            plan->view_tgt_order.resize(cp.tgt.n);
            if (cp.src.n > 0)
                HIP_TRY(hipMemcpy(plan->view_src_order.data(), plan->dprox.src_order,
                                  cp.src.n * sizeof(int64_t), hipMemcpyDeviceToHost));
            if (cp.tgt.n > 0)
                HIP_TRY(hipMemcpy(plan->view_tgt_order.data(), plan->ddir.tgt_orig,
                                  cp.tgt.n * sizeof(int64_t), hipMemcpyDeviceToHost));
        }
        out->source_order = plan->view_src_order.data();
        out->target_order = plan->view_tgt_order.data();
    }
    out->cluster_begin = cp.tgt.begin.data();
    out->cluster_count = cp.tgt.count.data();
    out->cluster_lo = cp.tgt.lo.data();
    out->cluster_hi = cp.tgt.hi.data();
    out->cluster_first_child = cp.tgt.first_child.data();
    out->cluster_nchild = cp.tgt.nchild.data();
    out->cluster_level = cp.tgt.level.data();
    if (plan->view_batch_lo.size() != 3 * cp.sb_node.size()) {
        plan->view_batch_lo.clear();
        plan->view_batch_hi.clear();
        for (int32_t u : cp.sb_node)
            for (int l = 0; l < 3; ++l) {
                plan->view_batch_lo.push_back(cp.src.lo[3 * u + l]);
                plan->view_batch_hi.push_back(cp.src.hi[3 * u + l]);
            }
    }
    out->batch_begin = cp.sb_begin.data();
    out->batch_count = cp.sb_count.data();
    out->batch_lo = plan->view_batch_lo.data();
    out->batch_hi = plan->view_batch_hi.data();
    out->item_batch = cp.item_batch.data();
    out->item_cluster = cp.item_cluster.data();
    out->item_kind = cp.item_kind.data();
    return BLTC_OK;
}

}  // namespace bltc_cp
