// cc.cpp -- plans of the cluster-cluster treecode (method
// BLTC_CLUSTER_CLUSTER): both sides interpolated, pairs from a dual walk.
//
// One evaluation:
//  1. charges into source-tree order, modified charges of the source slots
//     (the BLTC upward pass on the matrix cores, eqs. 14-15);
//  2. proxy potentials of the target slots: the interaction kernel over the
//     target grids as targets; a grid-grid pair is a far-field entry (eq. 11
//     at the grid points, separable in the source grid), a sources-grid pair
//     a particle range;
//  3. targets by target leaf: far lists (grid-targets pairs, eq. 11) and
//     direct lists, phi written once;
//  4. interpolation of the proxy potentials of every target slot on each
//     target's path (kernels_cp.hip), phi +=.
#include <chrono>
#include <cstring>
#include <numeric>

#include "internal.hpp"
#include "kernels_cp.hpp"
#include "setup_gpu.hpp"

using bltc_detail::fail;

namespace bltc_cc {

int create_host(bltc_plan* plan, const bltc::PlanParams& pp, int64_t nt, const double* tx,
                const double* ty, const double* tz, int64_t ns, const double* sx, const double* sy,
                const double* sz)
{
    plan->cc = true;
    bltc::make_cc_plan(plan->ccp, pp, nt, tx, ty, tz, ns, sx, sy, sz);
    return BLTC_OK;
}

int create_device(bltc_plan* plan, const bltc::PlanParams& pp, int64_t nt, const double* tx,
                  const double* ty, const double* tz, int64_t ns, const double* sx,
                  const double* sy, const double* sz, hipStream_t s)
{
    const auto t0 = std::chrono::steady_clock::now();
    plan->cc = true;
    bltc::CcPlan& cc = plan->ccp;
    cc = bltc::CcPlan();
    cc.prm = pp;
    const bool mixed = plan->prm.precision == BLTC_FP32_MIXED;
    HIP_TRY(hipGetDevice(&plan->device));
    bltc::DevicePlan& du = plan->d;
    bltc::DevicePlan& dd = plan->ddir;
    int64_t* src_order = nullptr;
    HIP_TRY(plan->alloc(&du.src, static_cast<size_t>(ns)));
    HIP_TRY(plan->alloc(&src_order, static_cast<size_t>(ns)));
    du.src_order = src_order;
    if (mixed)
        HIP_TRY(plan->alloc(&du.src32, static_cast<size_t>(ns)));
    HIP_TRY(plan->alloc(&dd.tgt, static_cast<size_t>(nt)));
    HIP_TRY(plan->alloc(&dd.tgt_orig, static_cast<size_t>(nt)));
    int64_t bad = -1;
    std::string err = bltc::build_tree_device(cc.src, ns, sx, sy, sz, pp.leaf_size, src_order,
                                              du.src, mixed ? du.src32 : nullptr, s, &bad);
    if (bad >= 0)
        return fail(BLTC_EINVAL, "source coordinate %lld is not finite", static_cast<long long>(bad));
    if (!err.empty())
        return fail(BLTC_EHIP, "device tree build: %s", err.c_str());
    if (nt == ns && tx == sx && ty == sy && tz == sz && pp.batch_size == pp.leaf_size) {
        cc.tgt = cc.src;
        cc.same_tree = true;
        if (nt > 0) {
            HIP_TRY(hipMemcpyAsync(dd.tgt, du.src, nt * sizeof(double4), hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(dd.tgt_orig, src_order, nt * sizeof(int64_t),
                                   hipMemcpyDeviceToDevice, s));
        }
    } else {
        err = bltc::build_tree_device(cc.tgt, nt, tx, ty, tz, pp.batch_size, dd.tgt_orig, dd.tgt,
                                      nullptr, s, &bad);
        if (bad >= 0)
            return fail(BLTC_EINVAL, "target coordinate %lld is not finite",
                        static_cast<long long>(bad));
        if (!err.empty())
            return fail(BLTC_EHIP, "device tree build: %s", err.c_str());
    }
    bltc::cc_plan_from_trees(cc);
    plan->device_particles = true;
    cc.setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return BLTC_OK;
}

int upload(bltc_plan* plan, hipStream_t s)
{
    if (plan->uploaded)
        return BLTC_OK;
    bltc::CcPlan& cc = plan->ccp;
    const bool mixed = plan->prm.precision == BLTC_FP32_MIXED;
    bltc::DevicePlan& du = plan->d;
    bltc::DevicePlan& px = plan->dprox;
    bltc::DevicePlan& dd = plan->ddir;
    HIP_TRY(hipGetDevice(&plan->device));
    const int64_t nt = cc.tgt.n, ns = cc.src.n;
    const int64_t nns = cc.src.nodes();
    const int64_t nss = static_cast<int64_t>(cc.sslot_cluster.size());
    const int64_t nts = static_cast<int64_t>(cc.tslot_cluster.size());
    const int64_t ntl = static_cast<int64_t>(cc.tl_node.size());
    const int32_t np = cc.np;
    const int64_t P = cc.P;

    auto expand = [&](const std::vector<double>& nodes, int64_t nslots) {
        std::vector<double4> g(static_cast<size_t>(nslots * P));
        for (int64_t sl = 0; sl < nslots; ++sl) {
            const double* nd = nodes.data() + sl * 3 * np;
            for (int32_t k1 = 0; k1 < np; ++k1)
                for (int32_t k2 = 0; k2 < np; ++k2)
                    for (int32_t k3 = 0; k3 < np; ++k3)
                        g[static_cast<size_t>(sl * P + (k1 * np + k2) * np + k3)] =
                            make_double4(nd[k1], nd[np + k2], nd[2 * np + k3], 0.0);
        }
        return g;
    };

    // ---- particles in tree order (host-built plans)
    if (!plan->device_particles) {
        std::vector<double4> src(ns), tgt(nt);
        for (int64_t j = 0; j < ns; ++j)
            src[j] = make_double4(cc.src.x[j], cc.src.y[j], cc.src.z[j], 0.0);
        for (int64_t i = 0; i < nt; ++i)
            tgt[i] = make_double4(cc.tgt.x[i], cc.tgt.y[i], cc.tgt.z[i], 0.0);
        HIP_TRY(plan->put(&du.src, src, s));
        HIP_TRY(plan->put(&dd.tgt, tgt, s));
        HIP_TRY(plan->put(&dd.tgt_orig, cc.tgt.order, s));
        int64_t* src_order = nullptr;
        HIP_TRY(plan->put(&src_order, cc.src.order, s));
        du.src_order = src_order;
        if (mixed) {
            // particles relative to the center of their source leaf
            std::vector<float4> src32(ns);
            for (int64_t u = 0; u < nns; ++u) {
                if (cc.src.nchild[u] != 0)
                    continue;
                const double cx = cc.src.center[3 * u], cy = cc.src.center[3 * u + 1],
                             cz = cc.src.center[3 * u + 2];
                for (int64_t j = cc.src.begin[u]; j < cc.src.begin[u] + cc.src.count[u]; ++j)
                    src32[j] = make_float4(static_cast<float>(cc.src.x[j] - cx),
                                           static_cast<float>(cc.src.y[j] - cy),
                                           static_cast<float>(cc.src.z[j] - cz), 0.0f);
            }
            HIP_TRY(plan->put(&du.src32, src32, s));
        }
        HIP_TRY(hipStreamSynchronize(s));
    }

    // ---- upward pass over the source slots
    du.degree = px.degree = dd.degree = plan->prm.degree;
    du.ns = ns;
    du.nslots = nss;
    du.nchunks = static_cast<int64_t>(cc.chunk_slot.size());
    HIP_TRY(plan->put(&du.slot_nodes, cc.sslot_nodes, s));
    HIP_TRY(plan->put(&du.chunk_slot, cc.chunk_slot, s));
    HIP_TRY(plan->put(&du.chunk_begin, cc.chunk_begin, s));
    HIP_TRY(plan->put(&du.chunk_count, cc.chunk_count, s));
    HIP_TRY(plan->put(&du.slot_chunk_off, cc.slot_chunk_off, s));
    HIP_TRY(plan->put(&du.chunk_dst, cc.chunk_dst, s));
    HIP_TRY(plan->alloc(&du.qhat, static_cast<size_t>((nss + cc.npartial) * P)));
    if (mixed)
        HIP_TRY(plan->alloc(&du.qhat32, static_cast<size_t>(nss * P)));

    // ---- proxy potentials of the target slots
    const std::vector<double4> tgrid = expand(cc.tslot_nodes, nts);
    std::vector<int64_t> tgrid_orig(tgrid.size()), tgrid_end(nts), leaf_end(ntl);
    std::iota(tgrid_orig.begin(), tgrid_orig.end(), int64_t(0));
    for (int64_t u = 0; u < nts; ++u)
        tgrid_end[u] = (u + 1) * P;
    for (int64_t r = 0; r < ntl; ++r)
        leaf_end[r] = cc.tl_begin[r] + cc.tl_count[r];
    px.src = dd.src = du.src;
    px.src32 = dd.src32 = du.src32;
    px.ns = dd.ns = ns;
    px.nt = nts * P;
    px.nbatches = nts;
    px.ngroups = static_cast<int64_t>(cc.pg_batch.size());
    HIP_TRY(plan->put(&px.tgt, tgrid, s));
    HIP_TRY(plan->put(&px.tgt_orig, tgrid_orig, s));
    HIP_TRY(plan->put(&px.group_batch, cc.pg_batch, s));
    HIP_TRY(plan->put(&px.group_first, cc.pg_first, s));
    HIP_TRY(plan->put(&px.batch_end, tgrid_end, s));
    HIP_TRY(plan->put(&px.far_off, cc.gg_off, s));
    HIP_TRY(plan->put(&px.far_slot, cc.gg_slot, s));
    HIP_TRY(plan->put(&px.near_off, cc.pf_off, s));
    HIP_TRY(plan->put(&px.near_begin, cc.pf_begin, s));
    HIP_TRY(plan->put(&px.near_count, cc.pf_count, s));
    HIP_TRY(plan->put(&px.near_leaf, cc.pf_leaf, s));
    px.slot_nodes = du.slot_nodes;
    px.qhat = du.qhat;
    px.qhat32 = du.qhat32;

    // ---- targets by target leaf
    dd.nt = nt;
    dd.nbatches = ntl;
    dd.ngroups = static_cast<int64_t>(cc.dg_batch.size());
    HIP_TRY(plan->put(&dd.group_batch, cc.dg_batch, s));
    HIP_TRY(plan->put(&dd.group_first, cc.dg_first, s));
    HIP_TRY(plan->put(&dd.batch_end, leaf_end, s));
    HIP_TRY(plan->put(&dd.far_off, cc.far_off, s));
    HIP_TRY(plan->put(&dd.far_slot, cc.far_slot, s));
    HIP_TRY(plan->put(&dd.near_off, cc.dn_off, s));
    HIP_TRY(plan->put(&dd.near_begin, cc.dn_begin, s));
    HIP_TRY(plan->put(&dd.near_count, cc.dn_count, s));
    HIP_TRY(plan->put(&dd.near_leaf, cc.dn_leaf, s));
    dd.slot_nodes = du.slot_nodes;
    dd.qhat = du.qhat;
    dd.qhat32 = du.qhat32;

    HIP_TRY(plan->put(&plan->cp_path_off, cc.dw_off, s));
    HIP_TRY(plan->put(&plan->cp_path_slot, cc.dw_slot, s));
    HIP_TRY(plan->put(&plan->cp_slot_nodes, cc.tslot_nodes, s));
    HIP_TRY(plan->alloc(&plan->cp_phat, static_cast<size_t>(nts * P)));

    if (mixed) {
        // per source node (the lists name source leaves): center and radius
        std::vector<double4> node_info(nns);
        for (int64_t c = 0; c < nns; ++c)
            node_info[c] = make_double4(cc.src.center[3 * c], cc.src.center[3 * c + 1],
                                        cc.src.center[3 * c + 2], cc.src.radius[c]);
        std::vector<double4> bi_p(nts), bi_d(ntl);
        for (int64_t u = 0; u < nts; ++u) {
            const int32_t c = cc.tslot_cluster[u];
            bi_p[u] = make_double4(cc.tgt.center[3 * c], cc.tgt.center[3 * c + 1],
                                   cc.tgt.center[3 * c + 2], cc.tgt.radius[c]);
        }
        for (int64_t r = 0; r < ntl; ++r) {
            const int32_t c = cc.tl_node[r];
            bi_d[r] = make_double4(cc.tgt.center[3 * c], cc.tgt.center[3 * c + 1],
                                   cc.tgt.center[3 * c + 2], cc.tgt.radius[c]);
        }
        HIP_TRY(plan->put(&px.node_info, node_info, s));
        dd.node_info = px.node_info;
        HIP_TRY(plan->put(&px.batch_info, bi_p, s));
        HIP_TRY(plan->put(&dd.batch_info, bi_d, s));
        if (!du.qhat32) {
            HIP_TRY(plan->alloc(&du.qhat32, 1));
            px.qhat32 = dd.qhat32 = du.qhat32;
        }
    }
    // targets are the sources: mutual direct leaf pairs once for both directions,
    // and the target-leaf workgroups (one wave each) re-ordered by the work left
    if (cc.same_tree && !plan->prm.no_symmetry) {
        const bltc::DirectLists dl{&cc.src,    &cc.tl_node, &cc.tl_begin, &cc.tl_count,
                                   &cc.dn_off, &cc.dn_leaf, &cc.dn_cost};
        int rc = bltc_internal_upload_symmetric(plan, dd, dl, &cc.dn_cost, s);
        if (rc != BLTC_OK)
            return rc;
        if (dd.sym) {
            cc.dg_batch.clear();
            cc.dg_first.clear();
            bltc::group_schedule(cc.tl_begin, cc.tl_count, cc.dn_cost, bltc::kGroupSizeSym,
                                 cc.prm.xcds, cc.dg_batch, cc.dg_first);
            HIP_TRY(plan->put(&dd.group_batch, cc.dg_batch, s));
            HIP_TRY(plan->put(&dd.group_first, cc.dg_first, s));
            dd.ngroups = static_cast<int64_t>(cc.dg_batch.size());
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
        return fail(BLTC_EUNSUPPORTED, "cluster-cluster plans take one charge vector");
    int rc = bltc_internal_upload_plan(plan, s);
    if (rc != BLTC_OK)
        return rc;
    const bltc::CcPlan& cc = plan->ccp;
    bltc::KernelParams kp;
    kp.kernel = plan->prm.kernel;
    kp.precision = plan->prm.precision;
    kp.kappa = plan->prm.kappa;
    kp.delta = plan->prm.delta;
    const bool mixed = kp.precision == BLTC_FP32_MIXED;
    bltc::DevicePlan& du = plan->d;
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
    HIP_TRY(bltc::launch_gather_charges(du, q, s));
    HIP_TRY(mark(1));
    HIP_TRY(bltc::launch_upward_mfma(du, 1, du.qhat, mixed ? du.qhat32 : nullptr, s));
    if (mixed)
        HIP_TRY(bltc::launch_interact_mixed(plan->dprox, kp, plan->cp_phat, s));
    else
        HIP_TRY(bltc::launch_interact(plan->dprox, kp, plan->cp_phat, s));
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
    const bltc::CcPlan& cc = plan->ccp;
    if (cluster < 0 || cluster >= cc.tgt.nodes())
        return fail(BLTC_EINVAL, "target node index out of range");
    const int32_t slot = cc.cluster_tslot[cluster];
    if (slot < 0)
        return fail(BLTC_EINVAL, "target node %lld has no proxy potentials",
                    static_cast<long long>(cluster));
    if (!plan->uploaded || plan->last_q == 0)
        return fail(BLTC_EINVAL, "plan has not been executed");
    HIP_TRY(hipMemcpyAsync(out, plan->cp_phat + static_cast<int64_t>(slot) * cc.P,
                           cc.P * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return BLTC_OK;
}

void stats(const bltc_plan* plan, bltc_stats* out)
{
    const bltc::CcPlan& cc = plan->ccp;
    out->clusters = cc.src.nodes();
    int64_t leaves = 0;
    for (int64_t u = 0; u < cc.src.nodes(); ++u)
        leaves += cc.src.nchild[u] == 0;
    out->leaves = leaves;
    out->batches = static_cast<int64_t>(cc.tl_node.size());
    out->approx_pairs = cc.kind_pairs[0] + cc.kind_pairs[1] + cc.kind_pairs[2];
    out->direct_pairs = cc.kind_pairs[3];
    out->approx_clusters = static_cast<int64_t>(cc.sslot_cluster.size());
    out->far_evals = cc.cc_evals + cc.pc_evals + cc.cp_evals;
    out->near_evals = cc.near_evals;
    out->upward_terms = cc.upward_terms + cc.interp_terms;
    out->depth = std::max(cc.src.depth, cc.tgt.depth);
    out->setup_seconds = cc.setup_seconds;
}

int view(const bltc_plan* plan, bltc_plan_view* out)
{
    const bltc::CcPlan& cc = plan->ccp;
    out->nt = cc.tgt.n;
    out->ns = cc.src.n;
    out->n_clusters = cc.src.nodes();
    out->n_batches = cc.tgt.nodes();
    out->n_items = static_cast<int64_t>(cc.pair_t.size());
    out->source_order = cc.src.order.data();
    out->target_order = cc.tgt.order.data();
    if (plan->device_particles) {
        if (plan->view_src_order.size() != static_cast<size_t>(cc.src.n)) {
            plan->view_src_order.resize(cc.src.n);
            plan->view_tgt_order.resize(cc.tgt.n);
            if (cc.src.n > 0)
                HIP_TRY(hipMemcpy(plan->view_src_order.data(), plan->d.src_order,
                                  cc.src.n * sizeof(int64_t), hipMemcpyDeviceToHost));
            if (cc.tgt.n > 0)
                HIP_TRY(hipMemcpy(plan->view_tgt_order.data(), plan->ddir.tgt_orig,
                                  cc.tgt.n * sizeof(int64_t), hipMemcpyDeviceToHost));
        }
        out->source_order = plan->view_src_order.data();
        out->target_order = plan->view_tgt_order.data();
    }
    out->cluster_begin = cc.src.begin.data();
    out->cluster_count = cc.src.count.data();
    out->cluster_lo = cc.src.lo.data();
    out->cluster_hi = cc.src.hi.data();
    out->cluster_first_child = cc.src.first_child.data();
    out->cluster_nchild = cc.src.nchild.data();
    out->cluster_level = cc.src.level.data();
    out->batch_begin = cc.tgt.begin.data();
    out->batch_count = cc.tgt.count.data();
    out->batch_lo = cc.tgt.lo.data();
    out->batch_hi = cc.tgt.hi.data();
    out->item_batch = cc.pair_t.data();
    out->item_cluster = cc.pair_s.data();
    out->item_kind = cc.pair_kind.data();
    return BLTC_OK;
}

}  // namespace bltc_cc
