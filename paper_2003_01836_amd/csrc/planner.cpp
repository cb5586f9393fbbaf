// planner.cpp -- host planning of the treecode (Sec. II-D, Alg. 1, eq. 13).
//
// Tree rules (Sec. II-D, Sec. III-A).  Where the paper is silent the same
// readings as the library's documentation apply:
//  * every node keeps the minimal bounding box of its own particles; its
//    center is the box midpoint (lo + hi)/2 and its radius half the diagonal;
//  * a node is a leaf when it holds <= cap particles or its box is a point;
//  * otherwise dimension l is split at the midpoint iff 2 L_l^2 >= L_max^2
//    (aspect-ratio rule: 8, 4 or 2 children); a coordinate equal to the
//    midpoint goes to the upper child; empty children are dropped; a split
//    that leaves every particle in one child makes the node a leaf.
// MAC (eq. 13): geometric part r_B + r_C < theta * R with
// R = sqrt(dx*dx + dy*dy + dz*dz), size part (n+1)^3 < N_C, both strict.
// Alg. 1 branch order: geometric failure recurses into the children of a
// non-leaf cluster (direct sum at a leaf); a size-only failure is a direct sum
// over the whole cluster.
#include "planner.hpp"
#include "parallel.hpp"

#include <algorithm>
#include <limits>
#include <map>
#include <atomic>
#include <chrono>
#include <climits>
#include <cmath>
#include <numeric>
#include <stdexcept>
#include <thread>

namespace bltc {

int32_t Tree::add_node(int64_t b, int64_t c, int32_t lev, int32_t par)
{
    begin.push_back(b);
    count.push_back(c);
    for (int l = 0; l < 3; ++l) {
        lo.push_back(0.0);
        hi.push_back(0.0);
        center.push_back(0.0);
    }
    radius.push_back(0.0);
    first_child.push_back(-1);
    nchild.push_back(0);
    level.push_back(lev);
    parent.push_back(par);
    depth = std::max(depth, lev);
    return static_cast<int32_t>(begin.size() - 1);
}

void Tree::set_box(int64_t id, const double a[3], const double b[3])
{
    double L[3];
    for (int l = 0; l < 3; ++l) {
        lo[3 * id + l] = a[l];
        hi[3 * id + l] = b[l];
        center[3 * id + l] = (a[l] + b[l]) / 2.0;
        L[l] = b[l] - a[l];
    }
    radius[id] = 0.5 * std::sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
}

bool node_split(const Tree& t, int64_t id, int64_t cap, bool split[3])
{
    double L[3];
    for (int l = 0; l < 3; ++l)
        L[l] = t.hi[3 * id + l] - t.lo[3 * id + l];
    const double Lmax = std::max(L[0], std::max(L[1], L[2]));
    if (t.count[id] <= cap || Lmax == 0.0)
        return false;
    for (int l = 0; l < 3; ++l)
        split[l] = (2.0 * L[l] * L[l] >= Lmax * Lmax);
    return true;
}

void build_tree(Tree& t, int64_t n, const double* x, const double* y, const double* z,
                int64_t cap)
{
    t = Tree();
    t.n = n;
    t.order.resize(n);
    std::iota(t.order.begin(), t.order.end(), int64_t(0));
    t.x.assign(x, x + n);
    t.y.assign(y, y + n);
    t.z.assign(z, z + n);
    if (n == 0)
        return;
    t.add_node(0, n, 0, -1);

    std::vector<uint8_t> code;
    std::vector<int64_t> tmp_o;
    std::vector<double> tmp_x, tmp_y, tmp_z;
    // breadth-first: node ids grow as children are appended
    for (int64_t id = 0; id < t.nodes(); ++id) {
        const int64_t b = t.begin[id], c = t.count[id];
        double lo[3] = {t.x[b], t.y[b], t.z[b]};
        double hi[3] = {t.x[b], t.y[b], t.z[b]};
        for (int64_t p = b + 1; p < b + c; ++p) {
            const double v[3] = {t.x[p], t.y[p], t.z[p]};
            for (int l = 0; l < 3; ++l) {
                lo[l] = std::min(lo[l], v[l]);
                hi[l] = std::max(hi[l], v[l]);
            }
        }
        t.set_box(id, lo, hi);
        bool split[3];
        if (!node_split(t, id, cap, split))
            continue;
        const double ctr[3] = {t.center[3 * id], t.center[3 * id + 1], t.center[3 * id + 2]};

        code.resize(c);
        int64_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t p = 0; p < c; ++p) {
            uint8_t k = 0;
            if (split[0] && t.x[b + p] >= ctr[0]) k |= 1;
            if (split[1] && t.y[b + p] >= ctr[1]) k |= 2;
            if (split[2] && t.z[b + p] >= ctr[2]) k |= 4;
            code[p] = k;
            ++cnt[k];
        }
        int nonempty = 0;
        for (int k = 0; k < 8; ++k)
            nonempty += cnt[k] > 0;
        if (nonempty < 2)
            continue;
        // stable counting sort of the node's range by child code
        int64_t off[8];
        int64_t run = 0;
        for (int k = 0; k < 8; ++k) {
            off[k] = run;
            run += cnt[k];
        }
        tmp_o.resize(c);
        tmp_x.resize(c);
        tmp_y.resize(c);
        tmp_z.resize(c);
        for (int64_t p = 0; p < c; ++p) {
            const int64_t d = off[code[p]]++;
            tmp_o[d] = t.order[b + p];
            tmp_x[d] = t.x[b + p];
            tmp_y[d] = t.y[b + p];
            tmp_z[d] = t.z[b + p];
        }
        std::copy(tmp_o.begin(), tmp_o.begin() + c, t.order.begin() + b);
        std::copy(tmp_x.begin(), tmp_x.begin() + c, t.x.begin() + b);
        std::copy(tmp_y.begin(), tmp_y.begin() + c, t.y.begin() + b);
        std::copy(tmp_z.begin(), tmp_z.begin() + c, t.z.begin() + b);

        const int32_t first = static_cast<int32_t>(t.nodes());
        int64_t start = b;
        int32_t nk = 0;
        for (int k = 0; k < 8; ++k) {
            if (cnt[k] == 0)
                continue;
            t.add_node(start, cnt[k], t.level[id] + 1, static_cast<int32_t>(id));
            start += cnt[k];
            ++nk;
        }
        t.first_child[id] = first;
        t.nchild[id] = nk;
    }
}

std::string make_plan(HostPlan& hp, const PlanParams& prm,
                      int64_t nt, const double* tx, const double* ty, const double* tz,
                      int64_t ns, const double* sx, const double* sy, const double* sz)
{
    auto t0 = std::chrono::steady_clock::now();
    hp = HostPlan();
    hp.prm = prm;

    build_tree(hp.src, ns, sx, sy, sz, prm.leaf_size);
    if (nt == ns && tx == sx && ty == sy && tz == sz && prm.batch_size == prm.leaf_size) {
        hp.tgt = hp.src;    // same particles, same capacity: identical partition
        hp.same_tree = true;
    } else
        build_tree(hp.tgt, nt, tx, ty, tz, prm.batch_size);
    plan_from_trees(hp);

    const Tree& S = hp.src;
    hp.leaf_of_pos.assign(ns, -1);
    for (int64_t id = 0; id < S.nodes(); ++id)
        if (S.nchild[id] == 0)
            for (int64_t p = S.begin[id]; p < S.begin[id] + S.count[id]; ++p)
                hp.leaf_of_pos[p] = static_cast<int32_t>(id);

    hp.setup_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return std::string();
}

void plan_batches(HostPlan& hp)
{
    const PlanParams& prm = hp.prm;
    hp.np = prm.degree + 1;
    hp.P = static_cast<int64_t>(prm.comps) * hp.np * hp.np * hp.np;
    const Tree& S = hp.src;
    const Tree& T = hp.tgt;
    // batches: leaves of the target tree, ordered by their first position
    for (int64_t id = 0; id < T.nodes(); ++id)
        if (T.nchild[id] == 0)
            hp.batch_node.push_back(static_cast<int32_t>(id));
    std::sort(hp.batch_node.begin(), hp.batch_node.end(),
              [&](int32_t a, int32_t b) { return T.begin[a] < T.begin[b]; });
    const int64_t nb = static_cast<int64_t>(hp.batch_node.size());
    hp.batch_begin.resize(nb);
    hp.batch_count.resize(nb);
    for (int64_t b = 0; b < nb; ++b) {
        hp.batch_begin[b] = T.begin[hp.batch_node[b]];
        hp.batch_count[b] = T.count[hp.batch_node[b]];
        for (int l = 0; l < 3; ++l) {
            hp.batch_lo.push_back(T.lo[3 * hp.batch_node[b] + l]);
            hp.batch_hi.push_back(T.hi[3 * hp.batch_node[b] + l]);
        }
    }
    for (int64_t id = 0; id < S.nodes(); ++id)
        hp.leaves += S.nchild[id] == 0;
}

void leaf_runs(const Tree& S, std::vector<int32_t>& leaf_list, std::vector<int64_t>& run_lo,
               std::vector<int64_t>& run_hi)
{
    leaf_list.clear();
    for (int64_t id = 0; id < S.nodes(); ++id)
        if (S.nchild[id] == 0)
            leaf_list.push_back(static_cast<int32_t>(id));
    std::sort(leaf_list.begin(), leaf_list.end(),
              [&](int32_t a, int32_t b) { return S.begin[a] < S.begin[b]; });
    std::vector<int64_t> leaf_first(leaf_list.size());
    for (size_t i = 0; i < leaf_list.size(); ++i)
        leaf_first[i] = S.begin[leaf_list[i]];
    run_lo.resize(S.nodes());
    run_hi.resize(S.nodes());
    for (int64_t c = 0; c < S.nodes(); ++c) {
        run_lo[c] = std::lower_bound(leaf_first.begin(), leaf_first.end(), S.begin[c]) -
                    leaf_first.begin();
        run_hi[c] = std::lower_bound(leaf_first.begin(), leaf_first.end(),
                                     S.begin[c] + S.count[c]) - leaf_first.begin();
    }
}

void grid_nodes(const Tree& t, const std::vector<int32_t>& clusters, int32_t degree,
                std::vector<double>& out)
{
    const int32_t np = degree + 1;
    const int64_t nc = static_cast<int64_t>(clusters.size());
    out.resize(nc * 3 * np);
    for (int64_t s = 0; s < nc; ++s) {
        const int32_t c = clusters[s];
        for (int l = 0; l < 3; ++l) {
            const double a = t.lo[3 * c + l], bb = t.hi[3 * c + l];
            const double mid = (a + bb) / 2.0;
            const double h = (bb - a) / 2.0;
            for (int32_t k = 0; k < np; ++k)
                out[(s * 3 + l) * np + k] =
                    mid + h * std::cos(M_PI * static_cast<double>(k) / static_cast<double>(degree));
        }
    }
}

void upward_chunks(const Tree& S, const std::vector<int32_t>& slot_cluster, int64_t chunk_size,
                   std::vector<int32_t>& chunk_slot, std::vector<int64_t>& chunk_begin,
                   std::vector<int64_t>& chunk_count, std::vector<int32_t>& slot_chunk_off,
                   std::vector<int64_t>& chunk_dst, int64_t& npartial)
{
    const int64_t nslots = static_cast<int64_t>(slot_cluster.size());
    slot_chunk_off.assign(nslots + 1, 0);
    for (int64_t s = 0; s < nslots; ++s) {
        const int32_t c = slot_cluster[s];
        for (int64_t off = 0; off < S.count[c]; off += chunk_size) {
            chunk_slot.push_back(static_cast<int32_t>(s));
            chunk_begin.push_back(S.begin[c] + off);
            chunk_count.push_back(std::min<int64_t>(chunk_size, S.count[c] - off));
        }
        slot_chunk_off[s + 1] = static_cast<int32_t>(chunk_slot.size());
        const int32_t c0 = slot_chunk_off[s], c1 = slot_chunk_off[s + 1];
        for (int32_t c = c0; c < c1; ++c)
            chunk_dst.push_back(c1 - c0 == 1 ? s : nslots + npartial++);
    }
}

void plan_slots(HostPlan& hp, const std::vector<uint8_t>& used)
{
    const Tree& S = hp.src;
    hp.cluster_slot.assign(S.nodes(), -1);
    hp.slot_cluster.clear();
    for (int64_t c = 0; c < S.nodes(); ++c)
        if (used[c]) {
            hp.cluster_slot[c] = static_cast<int32_t>(hp.slot_cluster.size());
            hp.slot_cluster.push_back(static_cast<int32_t>(c));
        }
    grid_nodes(S, hp.slot_cluster, hp.prm.degree, hp.slot_nodes);
}

void plan_from_trees(HostPlan& hp)
{
    plan_batches(hp);
    const PlanParams& prm = hp.prm;
    const int64_t ns = hp.src.n;
    const Tree& S = hp.src;
    const Tree& T = hp.tgt;
    const int64_t nb = static_cast<int64_t>(hp.batch_node.size());

    // ---- interaction lists (Alg. 1), one traversal per batch --------------
    std::vector<std::vector<int32_t>> approx(nb), direct(nb);
    if (ns > 0) {
        parallel_for(nb, [&](int64_t b) {
            const int32_t bn = hp.batch_node[b];
            const double cb[3] = {T.center[3 * bn], T.center[3 * bn + 1], T.center[3 * bn + 2]};
            const double rb = T.radius[bn];
            std::vector<int32_t> stack;
            stack.push_back(0);
            while (!stack.empty()) {
                const int32_t c = stack.back();
                stack.pop_back();
                const double dx = cb[0] - S.center[3 * c];
                const double dy = cb[1] - S.center[3 * c + 1];
                const double dz = cb[2] - S.center[3 * c + 2];
                const double R = std::sqrt(dx * dx + dy * dy + dz * dz);
                const bool geometric = rb + S.radius[c] < prm.theta * R;
                const bool size = hp.P < S.count[c];
                if (geometric && size) {
                    approx[b].push_back(c);
                } else if (!geometric) {
                    if (S.nchild[c] == 0) {
                        direct[b].push_back(c);
                    } else {
                        for (int32_t k = S.nchild[c] - 1; k >= 0; --k)
                            stack.push_back(S.first_child[c] + k);
                    }
                } else {
                    direct[b].push_back(c);
                }
            }
        });
    }

    // ---- slots: clusters that need modified charges ------------------------
    {
        std::vector<uint8_t> used(S.nodes(), 0);
        for (int64_t b = 0; b < nb; ++b)
            for (int32_t c : approx[b])
                used[c] = 1;
        plan_slots(hp, used);
    }

    // ---- flattened lists ----------------------------------------------------
    // The leaves below a node, in depth-first order, are the leaves inside its
    // position range ordered by their first position: a contiguous run of the
    // leaf list sorted by begin.
    std::vector<int32_t> leaf_list;
    std::vector<int64_t> run_lo, run_hi;
    leaf_runs(S, leaf_list, run_lo, run_hi);
    // sizes per batch, offsets, then every batch fills its own range
    std::vector<int64_t> item_off(nb + 1, 0), far_o(nb + 1, 0), near_o(nb + 1, 0);
    for (int64_t b = 0; b < nb; ++b) {
        int64_t nn = 0;
        for (int32_t c : direct[b])
            nn += run_hi[c] - run_lo[c];
        item_off[b + 1] = item_off[b] + static_cast<int64_t>(approx[b].size() + direct[b].size());
        far_o[b + 1] = far_o[b] + static_cast<int64_t>(approx[b].size());
        near_o[b + 1] = near_o[b] + nn;
    }
    if (far_o[nb] > INT32_MAX || near_o[nb] > INT32_MAX)
        throw std::length_error("interaction lists exceed 2^31 entries");
    hp.far_off.assign(nb + 1, 0);
    hp.near_off.assign(nb + 1, 0);
    for (int64_t b = 0; b <= nb; ++b) {
        hp.far_off[b] = static_cast<int32_t>(far_o[b]);
        hp.near_off[b] = static_cast<int32_t>(near_o[b]);
    }
    hp.batch_cost.assign(nb, 0);
    hp.item_batch.resize(item_off[nb]);
    hp.item_cluster.resize(item_off[nb]);
    hp.item_kind.resize(item_off[nb]);
    hp.far_slot.resize(far_o[nb]);
    hp.near_leaf.resize(near_o[nb]);
    hp.near_begin.resize(near_o[nb]);
    hp.near_count.resize(near_o[nb]);
    std::vector<int64_t> far_ev(nb), near_ev(nb);
    parallel_for(nb, [&](int64_t b) {
        const int64_t nbt = hp.batch_count[b];
        int64_t it = item_off[b], f = far_o[b], q = near_o[b];
        int64_t cost = 0, fe = 0, ne = 0;
        for (int32_t c : approx[b]) {
            hp.item_batch[it] = static_cast<int32_t>(b);
            hp.item_cluster[it] = c;
            hp.item_kind[it++] = 0;
            hp.far_slot[f++] = hp.cluster_slot[c];
            fe += nbt * hp.P;
            cost += hp.P;
        }
        for (int32_t c : direct[b]) {
            hp.item_batch[it] = static_cast<int32_t>(b);
            hp.item_cluster[it] = c;
            hp.item_kind[it++] = 1;
            ne += nbt * S.count[c];
            cost += S.count[c];
            // the leaves below c (c itself when it is a leaf)
            for (int64_t r = run_lo[c]; r < run_hi[c]; ++r) {
                const int32_t u = leaf_list[r];
                hp.near_leaf[q] = u;
                hp.near_begin[q] = S.begin[u];
                hp.near_count[q++] = S.count[u];
            }
        }
        hp.batch_cost[b] = cost;
        far_ev[b] = fe;
        near_ev[b] = ne;
    });
    for (int64_t b = 0; b < nb; ++b) {
        hp.far_evals += far_ev[b];
        hp.near_evals += near_ev[b];
        hp.approx_pairs += static_cast<int64_t>(approx[b].size());
        hp.direct_pairs += static_cast<int64_t>(direct[b].size());
    }

    plan_schedule(hp);
}

// Workgroups are dispatched round-robin over the dies (workgroup k on die
// k % X), and each die has its own L2.  Batches in tree order are split into
// X contiguous segments of equal work (neighbouring batches share most of
// their near-field sources), each segment is ordered heaviest batch first,
// and the segments are interleaved so that segment x lands on die x.
void group_schedule(const std::vector<int64_t>& begin, const std::vector<int64_t>& count,
                    const std::vector<int64_t>& cost, int32_t group_size, int32_t xcds,
                    std::vector<int32_t>& group_batch, std::vector<int64_t>& group_first)
{
    const int64_t nb = static_cast<int64_t>(begin.size());
    const int32_t X = std::max(1, xcds);
    std::vector<double> work(nb);
    double total = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t ng = (count[b] + group_size - 1) / group_size;
        work[b] = static_cast<double>(cost[b] + 1) * static_cast<double>(ng);
        total += work[b];
    }
    std::vector<std::vector<int32_t>> seg(X);
    double run_w = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
        int32_t x = static_cast<int32_t>(run_w * X / (total > 0.0 ? total : 1.0));
        x = std::min(x, X - 1);
        seg[x].push_back(static_cast<int32_t>(b));
        run_w += work[b];
    }
    std::vector<std::vector<std::pair<int32_t, int64_t>>> queue(X);
    size_t longest = 0;
    for (int32_t x = 0; x < X; ++x) {
        std::stable_sort(seg[x].begin(), seg[x].end(),
                         [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
        for (int32_t b : seg[x])
            for (int64_t f = 0; f < count[b]; f += group_size)
                queue[x].emplace_back(b, begin[b] + f);
        longest = std::max(longest, queue[x].size());
    }
    group_batch.assign(longest * X, -1);
    group_first.assign(longest * X, 0);
    for (int32_t x = 0; x < X; ++x)
        for (size_t i = 0; i < queue[x].size(); ++i) {
            group_batch[i * X + x] = queue[x][i].first;
            group_first[i * X + x] = queue[x][i].second;
        }
}

void plan_schedule(HostPlan& hp)
{
    const PlanParams& prm = hp.prm;
    const Tree& S = hp.src;
    const int64_t nslots = static_cast<int64_t>(hp.slot_cluster.size());
    // ---- upward-pass chunks ----------------------------------------------------
    for (int64_t s = 0; s < nslots; ++s)
        hp.upward_terms += S.count[hp.slot_cluster[s]] * hp.P;
    upward_chunks(S, hp.slot_cluster, prm.chunk_size, hp.chunk_slot, hp.chunk_begin, hp.chunk_count,
                  hp.slot_chunk_off, hp.chunk_dst, hp.npartial);

    group_schedule(hp.batch_begin, hp.batch_count, hp.batch_cost, prm.group_size, prm.xcds,
                   hp.group_batch, hp.group_first);
}

bool plan_symmetric(const DirectLists& dl, int64_t sub, int64_t max_out, int64_t max_unit,
                    SymPlan& sp)
{
    if (sub < 1)
        return false;
    const Tree& S = *dl.tree;
    const std::vector<int32_t>& batch_node = *dl.batch_node;
    const std::vector<int64_t>& batch_count = *dl.batch_count;
    const std::vector<int32_t>& near_off = *dl.near_off;
    const std::vector<int32_t>& near_leaf = *dl.near_leaf;
    const int64_t nb = static_cast<int64_t>(batch_node.size());
    if (static_cast<int64_t>(near_off.size()) != nb + 1 ||
        static_cast<int64_t>(near_leaf.size()) != (nb > 0 ? near_off[nb] : 0))
        return false;
    std::vector<int32_t> batch_of_node(S.nodes(), -1);
    for (int64_t b = 0; b < nb; ++b)
        batch_of_node[batch_node[b]] = static_cast<int32_t>(b);
    // direct partners (as batches) of every batch, sorted within the batch's
    // segment [near_off[b], near_off[b + 1]), for membership tests
    const int64_t ne = nb > 0 ? near_off[nb] : 0;
    std::vector<int32_t> part(static_cast<size_t>(ne));
    std::atomic<bool> not_leaf{false};
    parallel_for(nb, [&](int64_t b) {
        for (int32_t e = near_off[b]; e < near_off[b + 1]; ++e) {
            const int32_t c = batch_of_node[near_leaf[e]];
            if (c < 0)
                not_leaf = true;
            part[e] = c;
        }
        std::sort(part.begin() + near_off[b], part.begin() + near_off[b + 1]);
    });
    if (not_leaf)
        return false;   // a direct entry that is not a leaf
    // position of c in b's sorted partners, or -1
    auto find = [&](int64_t b, int32_t c) -> int64_t {
        const auto first = part.begin() + near_off[b], last = part.begin() + near_off[b + 1];
        const auto it = std::lower_bound(first, last, c);
        return it != last && *it == c ? it - part.begin() : -1;
    };
    // units: every mutual pair once, from its lower batch, in batch order and
    // partner order (per batch on host threads: count, then fill)
    std::vector<int64_t> uoff(static_cast<size_t>(nb) + 1, 0);
    parallel_for(nb, [&](int64_t b) {
        int64_t m = 0;
        for (int32_t e = near_off[b]; e < near_off[b + 1]; ++e)
            m += part[e] > b && find(part[e], static_cast<int32_t>(b)) >= 0;
        uoff[b + 1] = m;
    });
    for (int64_t b = 0; b < nb; ++b)
        uoff[b + 1] += uoff[b];
    // (pair evaluations, lower batch, upper batch)
    struct Cand {
        int64_t evals;
        int32_t b, c;
    };
    std::vector<Cand> units(static_cast<size_t>(uoff[nb]));
    if (units.empty())
        return false;
    parallel_for(nb, [&](int64_t b) {
        int64_t k = uoff[b];
        for (int32_t e = near_off[b]; e < near_off[b + 1]; ++e) {
            const int32_t c = part[e];
            if (c > b && find(c, static_cast<int32_t>(b)) >= 0)
                units[k++] = Cand{batch_count[b] * batch_count[c], static_cast<int32_t>(b), c};
        }
    });
    // heaviest first (equal weights keep the batch and partner order) when the
    // caps below leave some unit out; when every unit fits, the batch order
    // serves as well (it only places the units' results)
    int64_t total = 0, largest = 0;
    for (const Cand& u : units) {
        const int64_t nbk = batch_count[u.b], nck = batch_count[u.c];
        const int64_t size = nbk + ((nbk + sub - 1) / sub) * nck;
        total += size;
        largest = std::max(largest, size);
    }
    if (total > max_out || largest > max_unit)
        parallel_sort(units.begin(), units.end(), [](const Cand& a, const Cand& c) {
            if (a.evals != c.evals)
                return a.evals > c.evals;
            return a.b != c.b ? a.b < c.b : a.c < c.c;
        });
    // heaviest first while the results fit in max_out values; the mutual pairs
    // left over stay in the lists
    SymPlan out;
    out.sub = sub;
    std::vector<int64_t> taken;
    int64_t off = 0;
    for (int64_t k = 0; k < static_cast<int64_t>(units.size()); ++k) {
        const int64_t nbk = batch_count[units[k].b], nck = batch_count[units[k].c];
        const int64_t ns = (nbk + sub - 1) / sub;
        const int64_t size = nbk + ns * nck;
        if (size > max_unit || off + size > max_out)
            continue;
        taken.push_back(k);
        out.roff.push_back(off);
        out.coff.push_back(off + nbk);
        off += size;
        out.pair_evals += units[k].evals;
    }
    out.out_size = off;
    if (taken.empty())
        return false;
    // the taken units' fields; unit_at[e]: the unit of sorted partner entry e
    // (in both batches' segments), or -1
    const int64_t nu = static_cast<int64_t>(taken.size());
    out.ub.resize(nu);
    out.uc.resize(nu);
    out.nsub.resize(nu);
    out.apart.resize(nu);
    std::vector<int32_t> unit_at(static_cast<size_t>(ne), -1);
    parallel_for(nu, [&](int64_t id) {
        const Cand& u = units[taken[id]];
        out.ub[id] = u.b;
        out.uc[id] = u.c;
        out.nsub[id] = static_cast<int32_t>((batch_count[u.b] + sub - 1) / sub);
        unit_at[find(u.b, u.c)] = static_cast<int32_t>(id);
        unit_at[find(u.c, u.b)] = static_cast<int32_t>(id);
        // separation of the two leaves' boxes (points with equal coordinates
        // always share a leaf, so distinct leaves have a positive gap; the
        // test guards against squares that would underflow)
        const int64_t bn = batch_node[u.b], cn = batch_node[u.c];
        double gap = -std::numeric_limits<double>::infinity();
        for (int l = 0; l < 3; ++l)
            gap = std::max(gap, std::max(S.lo[3 * cn + l] - S.hi[3 * bn + l],
                                         S.lo[3 * bn + l] - S.hi[3 * cn + l]));
        out.apart[id] = gap >= 0x1p-500 ? 1 : 0;
    });
    // reduced lists in the original list order, and the costs left to the
    // batches (per batch on host threads: count, then fill)
    out.near_off.assign(nb + 1, 0);
    out.pc_off.assign(nb + 1, 0);
    out.batch_cost = (*dl.batch_cost);
    auto unit_of_entry = [&](int64_t b, int32_t e) -> int64_t {
        const int32_t c = batch_of_node[near_leaf[e]];
        return c != b ? unit_at[find(b, c)] : -1;
    };
    parallel_for(nb, [&](int64_t b) {
        int32_t nl = 0, npc = 0;
        for (int32_t e = near_off[b]; e < near_off[b + 1]; ++e) {
            const int64_t u = unit_of_entry(b, e);
            if (u < 0)
                ++nl;
            else
                npc += b < out.uc[u] ? 1 : out.nsub[u];
        }
        out.near_off[b + 1] = nl;
        out.pc_off[b + 1] = npc;
    });
    for (int64_t b = 0; b < nb; ++b) {
        out.near_off[b + 1] += out.near_off[b];
        out.pc_off[b + 1] += out.pc_off[b];
    }
    out.near_leaf.resize(out.near_off[nb]);
    out.near_begin.resize(out.near_off[nb]);
    out.near_count.resize(out.near_off[nb]);
    out.pc_base.resize(out.pc_off[nb]);
    parallel_for(nb, [&](int64_t b) {
        int32_t kl = out.near_off[b], kp = out.pc_off[b];
        for (int32_t e = near_off[b]; e < near_off[b + 1]; ++e) {
            const int32_t leaf = near_leaf[e];
            const int64_t u = unit_of_entry(b, e);
            if (u < 0) {
                out.near_leaf[kl] = leaf;
                out.near_begin[kl] = S.begin[leaf];
                out.near_count[kl] = S.count[leaf];
                ++kl;
            } else if (b < out.uc[u]) {
                out.pc_base[kp++] = out.roff[u];
                out.batch_cost[b] -= S.count[leaf] - 1;   // one read instead of |C| evaluations
            } else {
                for (int32_t q = 0; q < out.nsub[u]; ++q)
                    out.pc_base[kp++] = out.coff[u] + q * batch_count[b];
                out.batch_cost[b] -= S.count[leaf] - out.nsub[u];
            }
        }
    });
    sp = std::move(out);
    return true;
}

bool plan_pair_rounds(const SymPlan& sp, int64_t cap, std::vector<int32_t>& unit_begin,
                      std::vector<int64_t>& base)
{
    unit_begin.assign(1, 0);
    base.assign(1, 0);
    const int64_t nu = static_cast<int64_t>(sp.ub.size());
    for (int64_t u = 0; u < nu; ++u) {
        const int64_t end = u + 1 < nu ? sp.roff[u + 1] : sp.out_size;   // offsets are ascending
        if (end - sp.roff[u] > cap)
            return false;
        if (end - base.back() > cap) {
            unit_begin.push_back(static_cast<int32_t>(u));
            base.push_back(sp.roff[u]);
        }
    }
    unit_begin.push_back(static_cast<int32_t>(nu));
    base.push_back(sp.out_size);
    return true;
}

// ---------------------------------------------------------------------------
// Cluster-particle treecode (interpolation on the target side)
// ---------------------------------------------------------------------------
namespace {

// leaves of a tree ordered by first position
void leaves_by_begin(const Tree& t, std::vector<int32_t>& node, std::vector<int64_t>& begin,
                     std::vector<int64_t>& count)
{
    node.clear();
    for (int64_t id = 0; id < t.nodes(); ++id)
        if (t.nchild[id] == 0)
            node.push_back(static_cast<int32_t>(id));
    std::sort(node.begin(), node.end(), [&](int32_t a, int32_t b) { return t.begin[a] < t.begin[b]; });
    begin.resize(node.size());
    count.resize(node.size());
    for (size_t i = 0; i < node.size(); ++i) {
        begin[i] = t.begin[node[i]];
        count[i] = t.count[node[i]];
    }
}

}  // namespace

void cp_plan_from_trees(CpPlan& cp)
{
    const PlanParams& prm = cp.prm;
    cp.np = prm.degree + 1;
    cp.P = static_cast<int64_t>(cp.np) * cp.np * cp.np;
    const Tree& T = cp.tgt;
    const Tree& S = cp.src;
    leaves_by_begin(S, cp.sb_node, cp.sb_begin, cp.sb_count);
    leaves_by_begin(T, cp.tl_node, cp.tl_begin, cp.tl_count);
    const int64_t nsb = static_cast<int64_t>(cp.sb_node.size());
    const int64_t ntl = static_cast<int64_t>(cp.tl_node.size());
    const int64_t nn = T.nodes();
    cp.leaves = ntl;

    // ---- walks: every source batch over the target tree (Alg. 1, roles exchanged)
    std::vector<std::vector<int32_t>> approx(nsb), direct(nsb);
    if (nn > 0) {
        parallel_for(nsb, [&](int64_t b) {
            const int32_t sn = cp.sb_node[b];
            const double cs[3] = {S.center[3 * sn], S.center[3 * sn + 1], S.center[3 * sn + 2]};
            const double rs = S.radius[sn];
            std::vector<int32_t> stack{0};
            while (!stack.empty()) {
                const int32_t c = stack.back();
                stack.pop_back();
                const double dx = cs[0] - T.center[3 * c];
                const double dy = cs[1] - T.center[3 * c + 1];
                const double dz = cs[2] - T.center[3 * c + 2];
                const double R = std::sqrt(dx * dx + dy * dy + dz * dz);
                const bool geometric = rs + T.radius[c] < prm.theta * R;
                const bool size = cp.P < T.count[c];
                if (geometric && size) {
                    approx[b].push_back(c);
                } else if (!geometric && T.nchild[c] > 0) {
                    for (int32_t k = T.nchild[c] - 1; k >= 0; --k)
                        stack.push_back(T.first_child[c] + k);
                } else {
                    direct[b].push_back(c);
                }
            }
        });
    }
    for (int64_t b = 0; b < nsb; ++b) {
        for (int32_t c : approx[b]) {
            cp.item_batch.push_back(static_cast<int32_t>(b));
            cp.item_cluster.push_back(c);
            cp.item_kind.push_back(0);
        }
        for (int32_t c : direct[b]) {
            cp.item_batch.push_back(static_cast<int32_t>(b));
            cp.item_cluster.push_back(c);
            cp.item_kind.push_back(1);
        }
        cp.approx_pairs += static_cast<int64_t>(approx[b].size());
        cp.direct_pairs += static_cast<int64_t>(direct[b].size());
    }

    // ---- slots and their Chebyshev grids
    cp.cluster_slot.assign(nn, -1);
    std::vector<int64_t> nfar(nn, 0);
    for (int64_t b = 0; b < nsb; ++b)
        for (int32_t c : approx[b])
            ++nfar[c];
    for (int64_t c = 0; c < nn; ++c)
        if (nfar[c] > 0) {
            cp.cluster_slot[c] = static_cast<int32_t>(cp.slot_cluster.size());
            cp.slot_cluster.push_back(static_cast<int32_t>(c));
        }
    const int64_t nslots = static_cast<int64_t>(cp.slot_cluster.size());
    grid_nodes(T, cp.slot_cluster, prm.degree, cp.slot_nodes);
    for (int64_t sl = 0; sl < nslots; ++sl)
        cp.interp_terms += T.count[cp.slot_cluster[sl]] * cp.P;

    // ---- proxy lists: per slot, its source batches in batch order
    cp.pf_off.assign(nslots + 1, 0);
    for (int64_t sl = 0; sl < nslots; ++sl)
        cp.pf_off[sl + 1] = cp.pf_off[sl] + static_cast<int32_t>(nfar[cp.slot_cluster[sl]]);
    const int64_t npf = cp.pf_off[nslots];
    cp.pf_leaf.resize(npf);
    cp.pf_begin.resize(npf);
    cp.pf_count.resize(npf);
    cp.pf_cost.assign(nslots, 0);
    {
        std::vector<int32_t> fill(cp.pf_off.begin(), cp.pf_off.end() - 1);
        for (int64_t b = 0; b < nsb; ++b)
            for (int32_t c : approx[b]) {
                const int32_t sl = cp.cluster_slot[c];
                const int32_t e = fill[sl]++;
                cp.pf_leaf[e] = cp.sb_node[b];
                cp.pf_begin[e] = cp.sb_begin[b];
                cp.pf_count[e] = cp.sb_count[b];
                cp.pf_cost[sl] += cp.sb_count[b];
                cp.proxy_evals += cp.P * cp.sb_count[b];
            }
    }

    // ---- direct lists: per target leaf, the source batches of the direct
    // pairs of every cluster containing it, in batch order
    std::vector<int32_t> leaf_list;
    std::vector<int64_t> run_lo, run_hi;
    leaf_runs(T, leaf_list, run_lo, run_hi);     // leaf_list equals tl_node
    std::vector<int64_t> ndir(ntl, 0);
    for (int64_t b = 0; b < nsb; ++b)
        for (int32_t c : direct[b]) {
            for (int64_t r = run_lo[c]; r < run_hi[c]; ++r)
                ++ndir[r];
            cp.near_evals += T.count[c] * cp.sb_count[b];
        }
    cp.dn_off.assign(ntl + 1, 0);
    for (int64_t t = 0; t < ntl; ++t) {
        const int64_t v = cp.dn_off[t] + ndir[t];
        if (v > INT32_MAX)
            throw std::length_error("direct lists exceed 2^31 entries");
        cp.dn_off[t + 1] = static_cast<int32_t>(v);
    }
    const int64_t ndn = cp.dn_off[ntl];
    cp.dn_leaf.resize(ndn);
    cp.dn_begin.resize(ndn);
    cp.dn_count.resize(ndn);
    cp.dn_cost.assign(ntl, 0);
    {
        std::vector<int64_t> fill(cp.dn_off.begin(), cp.dn_off.end() - 1);
        for (int64_t b = 0; b < nsb; ++b)
            for (int32_t c : direct[b])
                for (int64_t r = run_lo[c]; r < run_hi[c]; ++r) {
                    const int64_t e = fill[r]++;
                    cp.dn_leaf[e] = cp.sb_node[b];
                    cp.dn_begin[e] = cp.sb_begin[b];
                    cp.dn_count[e] = cp.sb_count[b];
                    cp.dn_cost[r] += cp.sb_count[b];
                }
    }

    // ---- interpolation lists: slots on each target leaf's root-to-leaf path
    cp.dw_off.assign(ntl + 1, 0);
    for (int64_t t = 0; t < ntl; ++t) {
        std::vector<int32_t> path;
        for (int32_t u = cp.tl_node[t]; u >= 0; u = T.parent[u])
            if (cp.cluster_slot[u] >= 0)
                path.push_back(cp.cluster_slot[u]);
        std::reverse(path.begin(), path.end());
        cp.dw_slot.insert(cp.dw_slot.end(), path.begin(), path.end());
        cp.dw_off[t + 1] = static_cast<int32_t>(cp.dw_slot.size());
        cp.dn_cost[t] += static_cast<int64_t>(path.size()) * cp.P;
    }

    // ---- workgroups
    std::vector<int64_t> pbegin(nslots), pcount(nslots, cp.P);
    for (int64_t sl = 0; sl < nslots; ++sl)
        pbegin[sl] = sl * cp.P;
    group_schedule(pbegin, pcount, cp.pf_cost, prm.group_size, prm.xcds, cp.pg_batch, cp.pg_first);
    group_schedule(cp.tl_begin, cp.tl_count, cp.dn_cost, prm.group_size, prm.xcds, cp.dg_batch,
                   cp.dg_first);
}

void make_cp_plan(CpPlan& cp, const PlanParams& prm,
                  int64_t nt, const double* tx, const double* ty, const double* tz,
                  int64_t ns, const double* sx, const double* sy, const double* sz)
{
    auto t0 = std::chrono::steady_clock::now();
    cp = CpPlan();
    cp.prm = prm;
    build_tree(cp.tgt, nt, tx, ty, tz, prm.leaf_size);
    if (nt == ns && tx == sx && ty == sy && tz == sz && prm.batch_size == prm.leaf_size) {
        cp.src = cp.tgt;
        cp.same_arrays = cp.same_tree = true;
    } else
        build_tree(cp.src, ns, sx, sy, sz, prm.batch_size);
    cp_plan_from_trees(cp);
    cp.setup_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------------------
// Cluster-cluster treecode (both sides interpolated)
// ---------------------------------------------------------------------------
void cc_plan_from_trees(CcPlan& cc)
{
    const PlanParams& prm = cc.prm;
    cc.np = prm.degree + 1;
    cc.P = static_cast<int64_t>(cc.np) * cc.np * cc.np;
    const Tree& T = cc.tgt;
    const Tree& S = cc.src;
    const int64_t P = cc.P;
    const int64_t nnt = T.nodes(), nns = S.nodes();

    // ---- dual walk (explicit stack, children pushed in reverse: the visiting
    // order of the recursive walk)
    if (nnt > 0 && nns > 0) {
        std::vector<std::pair<int32_t, int32_t>> stack{{0, 0}};
        while (!stack.empty()) {
            const int32_t t = stack.back().first, s = stack.back().second;
            stack.pop_back();
            const double dx = T.center[3 * t] - S.center[3 * s];
            const double dy = T.center[3 * t + 1] - S.center[3 * s + 1];
            const double dz = T.center[3 * t + 2] - S.center[3 * s + 2];
            const double R = std::sqrt(dx * dx + dy * dy + dz * dz);
            int32_t kind = -1;
            if (T.radius[t] + S.radius[s] < prm.theta * R) {
                const bool bt = P < T.count[t], bs = P < S.count[s];
                kind = bt && bs ? 0 : (bs ? 1 : (bt ? 2 : 3));
            } else if (T.nchild[t] == 0 && S.nchild[s] == 0) {
                kind = 3;
            }
            if (kind >= 0) {
                cc.pair_t.push_back(t);
                cc.pair_s.push_back(s);
                cc.pair_kind.push_back(kind);
                ++cc.kind_pairs[kind];
                continue;
            }
            bool split_t, split_s;
            if (S.nchild[s] == 0) {
                split_t = true;
                split_s = false;
            } else if (T.nchild[t] == 0) {
                split_t = false;
                split_s = true;
            } else if (T.radius[t] > S.radius[s]) {
                split_t = true;
                split_s = false;
            } else if (S.radius[s] > T.radius[t]) {
                split_t = false;
                split_s = true;
            } else {
                split_t = split_s = true;
            }
            const int32_t nkt = split_t ? T.nchild[t] : 1, nks = split_s ? S.nchild[s] : 1;
            for (int32_t a = nkt - 1; a >= 0; --a)
                for (int32_t b = nks - 1; b >= 0; --b)
                    stack.emplace_back(split_t ? T.first_child[t] + a : t,
                                       split_s ? S.first_child[s] + b : s);
        }
    }
    const int64_t npairs = static_cast<int64_t>(cc.pair_t.size());

    // ---- slots on both sides
    cc.cluster_sslot.assign(nns, -1);
    cc.cluster_tslot.assign(nnt, -1);
    {
        std::vector<uint8_t> us(nns, 0), ut(nnt, 0);
        for (int64_t k = 0; k < npairs; ++k) {
            if (cc.pair_kind[k] <= 1)
                us[cc.pair_s[k]] = 1;
            if (cc.pair_kind[k] == 0 || cc.pair_kind[k] == 2)
                ut[cc.pair_t[k]] = 1;
        }
        for (int64_t c = 0; c < nns; ++c)
            if (us[c]) {
                cc.cluster_sslot[c] = static_cast<int32_t>(cc.sslot_cluster.size());
                cc.sslot_cluster.push_back(static_cast<int32_t>(c));
            }
        for (int64_t c = 0; c < nnt; ++c)
            if (ut[c]) {
                cc.cluster_tslot[c] = static_cast<int32_t>(cc.tslot_cluster.size());
                cc.tslot_cluster.push_back(static_cast<int32_t>(c));
            }
    }
    const int64_t nts = static_cast<int64_t>(cc.tslot_cluster.size());
    grid_nodes(S, cc.sslot_cluster, prm.degree, cc.sslot_nodes);
    grid_nodes(T, cc.tslot_cluster, prm.degree, cc.tslot_nodes);
    for (int32_t c : cc.sslot_cluster)
        cc.upward_terms += S.count[c] * P;
    for (int32_t c : cc.tslot_cluster)
        cc.interp_terms += T.count[c] * P;
    upward_chunks(S, cc.sslot_cluster, prm.chunk_size, cc.chunk_slot, cc.chunk_begin, cc.chunk_count,
                  cc.slot_chunk_off, cc.chunk_dst, cc.npartial);

    // leaf runs: the leaves below a node, in depth-first order
    std::vector<int32_t> s_leaves, t_leaves;
    std::vector<int64_t> s_lo, s_hi, t_lo, t_hi;
    leaf_runs(S, s_leaves, s_lo, s_hi);
    leaf_runs(T, t_leaves, t_lo, t_hi);
    leaves_by_begin(T, cc.tl_node, cc.tl_begin, cc.tl_count);     // equals t_leaves
    const int64_t ntl = static_cast<int64_t>(cc.tl_node.size());

    // ---- proxy lists per target slot (pairs in walk order): grid-grid pairs
    // as far-field entries (the target grid points are the "targets" of eq.
    // 11), sources-grid pairs as particle ranges
    std::vector<int64_t> npf(nts, 0), ngg(nts, 0);
    for (int64_t k = 0; k < npairs; ++k) {
        const int32_t kind = cc.pair_kind[k];
        if (kind == 0)
            ngg[cc.cluster_tslot[cc.pair_t[k]]] += 1;
        else if (kind == 2)
            npf[cc.cluster_tslot[cc.pair_t[k]]] += s_hi[cc.pair_s[k]] - s_lo[cc.pair_s[k]];
    }
    cc.pf_off.assign(nts + 1, 0);
    cc.gg_off.assign(nts + 1, 0);
    for (int64_t u = 0; u < nts; ++u) {
        const int64_t v = cc.pf_off[u] + npf[u], w = cc.gg_off[u] + ngg[u];
        if (v > INT32_MAX || w > INT32_MAX)
            throw std::length_error("proxy lists exceed 2^31 entries");
        cc.pf_off[u + 1] = static_cast<int32_t>(v);
        cc.gg_off[u + 1] = static_cast<int32_t>(w);
    }
    cc.pf_leaf.resize(cc.pf_off[nts]);
    cc.pf_begin.resize(cc.pf_off[nts]);
    cc.pf_count.resize(cc.pf_off[nts]);
    cc.gg_slot.resize(cc.gg_off[nts]);
    cc.pf_cost.assign(nts, 0);
    {
        std::vector<int64_t> fill(cc.pf_off.begin(), cc.pf_off.end() - 1);
        std::vector<int64_t> gfill(cc.gg_off.begin(), cc.gg_off.end() - 1);
        for (int64_t k = 0; k < npairs; ++k) {
            const int32_t kind = cc.pair_kind[k], t = cc.pair_t[k], s = cc.pair_s[k];
            if (kind == 0) {
                const int32_t u = cc.cluster_tslot[t];
                cc.gg_slot[gfill[u]++] = cc.cluster_sslot[s];
                cc.pf_cost[u] += P;
                cc.cc_evals += P * P;
            } else if (kind == 2) {
                const int32_t u = cc.cluster_tslot[t];
                for (int64_t r = s_lo[s]; r < s_hi[s]; ++r) {
                    const int32_t lf = s_leaves[r];
                    const int64_t e = fill[u]++;
                    cc.pf_leaf[e] = lf;
                    cc.pf_begin[e] = S.begin[lf];
                    cc.pf_count[e] = S.count[lf];
                }
                cc.pf_cost[u] += S.count[s];
                cc.cp_evals += P * S.count[s];
            }
        }
    }

    // ---- per target leaf: particle-cluster slots and direct ranges of the
    // pairs of every cluster on its path (pairs in walk order)
    std::vector<int64_t> nfar(ntl, 0), nnear(ntl, 0);
    for (int64_t k = 0; k < npairs; ++k) {
        const int32_t kind = cc.pair_kind[k], t = cc.pair_t[k], s = cc.pair_s[k];
        if (kind != 1 && kind != 3)
            continue;
        for (int64_t r = t_lo[t]; r < t_hi[t]; ++r) {
            if (kind == 1)
                ++nfar[r];
            else
                nnear[r] += s_hi[s] - s_lo[s];
        }
        if (kind == 1)
            cc.pc_evals += T.count[t] * P;
        else
            cc.near_evals += T.count[t] * S.count[s];
    }
    cc.far_off.assign(ntl + 1, 0);
    cc.dn_off.assign(ntl + 1, 0);
    for (int64_t r = 0; r < ntl; ++r) {
        const int64_t f = cc.far_off[r] + nfar[r], d = cc.dn_off[r] + nnear[r];
        if (f > INT32_MAX || d > INT32_MAX)
            throw std::length_error("interaction lists exceed 2^31 entries");
        cc.far_off[r + 1] = static_cast<int32_t>(f);
        cc.dn_off[r + 1] = static_cast<int32_t>(d);
    }
    cc.far_slot.resize(cc.far_off[ntl]);
    cc.dn_leaf.resize(cc.dn_off[ntl]);
    cc.dn_begin.resize(cc.dn_off[ntl]);
    cc.dn_count.resize(cc.dn_off[ntl]);
    cc.dn_cost.assign(ntl, 0);
    {
        std::vector<int64_t> ff(cc.far_off.begin(), cc.far_off.end() - 1);
        std::vector<int64_t> fd(cc.dn_off.begin(), cc.dn_off.end() - 1);
        for (int64_t k = 0; k < npairs; ++k) {
            const int32_t kind = cc.pair_kind[k], t = cc.pair_t[k], s = cc.pair_s[k];
            if (kind != 1 && kind != 3)
                continue;
            for (int64_t r = t_lo[t]; r < t_hi[t]; ++r) {
                if (kind == 1) {
                    cc.far_slot[ff[r]++] = cc.cluster_sslot[s];
                    cc.dn_cost[r] += P;
                } else {
                    for (int64_t q = s_lo[s]; q < s_hi[s]; ++q) {
                        const int32_t lf = s_leaves[q];
                        const int64_t e = fd[r]++;
                        cc.dn_leaf[e] = lf;
                        cc.dn_begin[e] = S.begin[lf];
                        cc.dn_count[e] = S.count[lf];
                    }
                    cc.dn_cost[r] += S.count[s];
                }
            }
        }
    }

    // ---- interpolation lists
    cc.dw_off.assign(ntl + 1, 0);
    for (int64_t r = 0; r < ntl; ++r) {
        std::vector<int32_t> path;
        for (int32_t u = cc.tl_node[r]; u >= 0; u = T.parent[u])
            if (cc.cluster_tslot[u] >= 0)
                path.push_back(cc.cluster_tslot[u]);
        std::reverse(path.begin(), path.end());
        cc.dw_slot.insert(cc.dw_slot.end(), path.begin(), path.end());
        cc.dw_off[r + 1] = static_cast<int32_t>(cc.dw_slot.size());
        cc.dn_cost[r] += static_cast<int64_t>(path.size()) * P;
    }

    // ---- workgroups
    std::vector<int64_t> pbegin(nts), pcount(nts, P);
    for (int64_t u = 0; u < nts; ++u)
        pbegin[u] = u * P;
    group_schedule(pbegin, pcount, cc.pf_cost, prm.group_size, prm.xcds, cc.pg_batch, cc.pg_first);
    group_schedule(cc.tl_begin, cc.tl_count, cc.dn_cost, prm.group_size, prm.xcds, cc.dg_batch,
                   cc.dg_first);
}

void make_cc_plan(CcPlan& cc, const PlanParams& prm,
                  int64_t nt, const double* tx, const double* ty, const double* tz,
                  int64_t ns, const double* sx, const double* sy, const double* sz)
{
    auto t0 = std::chrono::steady_clock::now();
    cc = CcPlan();
    cc.prm = prm;
    build_tree(cc.src, ns, sx, sy, sz, prm.leaf_size);
    if (nt == ns && tx == sx && ty == sy && tz == sz && prm.batch_size == prm.leaf_size) {
        cc.tgt = cc.src;
        cc.same_tree = true;
    } else
        build_tree(cc.tgt, nt, tx, ty, tz, prm.batch_size);
    cc_plan_from_trees(cc);
    cc.setup_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace bltc
