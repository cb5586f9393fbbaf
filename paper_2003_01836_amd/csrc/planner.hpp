// planner.hpp -- host-side planning for the treecode: source tree, target
// batches, interaction lists (Alg. 1, Sec. II-D, MAC eq. 13) and the flat work
// arrays the GPU kernels consume.  Pure C++ (no HIP), compiled without FP
// contraction so that every geometric decision follows its formula exactly.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace bltc {

// Cluster tree over one point set.  Nodes are numbered breadth first; the
// children of a node are consecutive.  Particles are stored contiguously per
// node ("tree order").
struct Tree {
    int64_t n = 0;
    std::vector<int64_t> order;          // original index of tree position p
    std::vector<double> x, y, z;         // coordinates in tree order
    std::vector<int64_t> begin, count;   // per node
    std::vector<double> lo, hi;          // per node, 3 each: minimal bounding box
    std::vector<double> center;          // per node, 3 each: box midpoint
    std::vector<double> radius;          // per node: half the box diagonal
    std::vector<int32_t> first_child, nchild, level, parent;
    int32_t depth = 0;
    int64_t nodes() const { return static_cast<int64_t>(begin.size()); }
    // appends a node (box fields zero) and returns its id
    int32_t add_node(int64_t begin, int64_t count, int32_t level, int32_t parent);
    // stores the minimal box of node id with its midpoint and half diagonal
    void set_box(int64_t id, const double lo[3], const double hi[3]);
};

// Split decision of a node from its minimal box and particle count (tree rules
// in planner.cpp).  Returns false when the node is a leaf; otherwise split[l]
// tells whether dimension l is cut at the box midpoint.
bool node_split(const Tree& t, int64_t id, int64_t cap, bool split[3]);

struct PlanParams {
    double theta = 0.7;
    int32_t degree = 8;
    int64_t leaf_size = 2000;
    int64_t batch_size = 2000;
    int32_t group_size = 256;       // targets per GPU workgroup
    int64_t chunk_size = 8192;      // sources per upward-pass chunk
    int32_t xcds = 8;               // accelerator dies that round-robin the workgroups
    int32_t comps = 1;              // modified charges per grid point: 1, or 8 (Hermite)
};

struct HostPlan {
    PlanParams prm;
    int32_t np = 0;                 // n + 1
    int64_t P = 0;                  // comps (n + 1)^3: modified charges per cluster
    Tree src, tgt;

    // batches = leaves of the target tree, in tree (depth-first) order
    std::vector<int32_t> batch_node;
    std::vector<int64_t> batch_begin, batch_count;
    std::vector<double> batch_lo, batch_hi;   // [3] per batch: minimal box

    // interaction items as found by the traversal (for inspection)
    std::vector<int32_t> item_batch, item_cluster, item_kind;

    // far field: per batch, the slots of its approximated clusters
    std::vector<int32_t> far_off, far_slot;
    // near field: per batch, leaf source ranges
    std::vector<int32_t> near_off, near_leaf;
    std::vector<int64_t> near_begin, near_count;

    // clusters that need modified charges ("slots")
    std::vector<int32_t> slot_cluster;   // cluster id of each slot
    std::vector<int32_t> cluster_slot;   // slot of each cluster or -1
    std::vector<double> slot_nodes;      // [slot][3][np] Chebyshev points

    // upward-pass chunks: contiguous source ranges of one slot each
    std::vector<int32_t> chunk_slot;
    std::vector<int64_t> chunk_begin, chunk_count;
    std::vector<int32_t> slot_chunk_off; // [nslots + 1]
    std::vector<int64_t> chunk_dst;      // output row: the slot itself for single-chunk
                                         // slots, else nslots + partial index
    int64_t npartial = 0;

    // interaction workgroups: (batch, first target position); batch -1 marks an
    // empty slot.  Workgroup k runs on die k % xcds: each die gets a spatially
    // contiguous, cost-balanced segment of batches, heaviest batch first.
    std::vector<int32_t> group_batch;
    std::vector<int64_t> group_first;
    std::vector<int64_t> batch_cost;     // kernel evaluations per target of each batch

    // leaf centers (for local coordinates of the mixed-precision path)
    std::vector<int32_t> leaf_of_pos;    // source leaf id of each tree position

    // statistics
    int64_t approx_pairs = 0, direct_pairs = 0;
    int64_t far_evals = 0, near_evals = 0, upward_terms = 0;
    int64_t leaves = 0;
    double setup_seconds = 0.0;

    // targets are the sources (same arrays, same capacity): the target tree is
    // the source tree and batch b is the leaf batch_node[b]
    bool same_tree = false;
};

// Mutual direct pairs of a plan whose batches are the leaves of its source
// tree.  G(x, y) = G(y, x), so two different leaves B and C, each in the
// other's direct list, form one unit evaluated once for both directions.  A
// unit is cut into sub-units of at most `sub` of B's targets; sub-unit s
// writes the row sums of its targets (potential at B's targets from C's
// sources) to out[roff + s sub ..] and its column sums (at C's targets from
// its B sources) to out[coff + s |C| .. + |C|).
struct SymPlan {
    std::vector<int32_t> ub, uc;        // batches of a unit, ub < uc; heaviest unit first when
                                        // the caps leave some out, else in batch order
    std::vector<int64_t> roff, coff;    // out offsets of a unit's rows and first column block
    std::vector<int32_t> nsub;          // sub-units of a unit: ceil(|B| / sub)
    // 1 when the two leaves' boxes are at least 2^-500 apart in some dimension:
    // every pair of the unit then has r^2 >= 2^-1000 > 0 (no zero-distance test)
    std::vector<uint8_t> apart;
    int64_t sub = 0;                    // B targets per sub-unit
    int64_t out_size = 0;
    int64_t pair_evals = 0;             // sum over units of |B| |C|
    // per batch: the direct entries that are not mutual (leaf, range) ...
    std::vector<int32_t> near_off, near_leaf;
    std::vector<int64_t> near_begin, near_count;
    // ... and the out offsets of its rows or column blocks of every mutual
    // pair, in list order (a B side: one entry; a C side: nsub entries)
    std::vector<int32_t> pc_off;
    std::vector<int64_t> pc_base;
    std::vector<int64_t> batch_cost;    // evaluations per target left to the batch's workgroups
};

// The direct lists of a plan whose batches are the leaves of one tree (the
// targets are the sources): batch b is the leaf batch_node[b] at positions
// [batch_begin[b], + batch_count[b]); its direct entries are the leaves
// near_leaf[near_off[b] .. near_off[b + 1]); batch_cost is the work per
// target of each batch.
struct DirectLists {
    const Tree* tree;
    const std::vector<int32_t>* batch_node;
    const std::vector<int64_t>* batch_begin;
    const std::vector<int64_t>* batch_count;
    const std::vector<int32_t>* near_off;
    const std::vector<int32_t>* near_leaf;
    const std::vector<int64_t>* batch_cost;
};

// Builds sp from the direct lists with sub-units of `sub` targets; the units
// are taken heaviest first while out_size stays within max_out values, each
// with at most max_unit result values (the mutual pairs left over stay in the
// lists).  Returns false (sp untouched) when no unit is taken or a direct
// entry is not a batch's leaf.
bool plan_symmetric(const DirectLists& dl, int64_t sub, int64_t max_out, int64_t max_unit,
                    SymPlan& sp);

// Rounds of the mutual-pair results through a workspace of `cap` values: the
// units of sp in their offset order (heaviest first), cut into runs whose
// results fit in cap; round r holds units [unit_begin[r], unit_begin[r + 1])
// and result offsets [base[r], base[r + 1]).  Returns false when one unit
// alone needs more than cap values.
bool plan_pair_rounds(const SymPlan& sp, int64_t cap, std::vector<int32_t>& unit_begin,
                      std::vector<int64_t>& base);

// Builds the tree with leaf capacity `cap` (readings of the tree rules are
// documented in planner.cpp).
void build_tree(Tree& t, int64_t n, const double* x, const double* y, const double* z,
                int64_t cap);

// Full host plan.  Returns an empty string on success or an error message.
std::string make_plan(HostPlan& hp, const PlanParams& prm,
                      int64_t nt, const double* tx, const double* ty, const double* tz,
                      int64_t ns, const double* sx, const double* sy, const double* sz);

// The part of the plan that needs only the node arrays of hp.src and hp.tgt
// (batches, lists, slots, chunks, workgroup schedule); hp.prm is set first.
// Used after the trees were built on the host or on the device.
void plan_from_trees(HostPlan& hp);

// Stages of plan_from_trees, for callers that build the lists elsewhere:
// batches (and n + 1, P) from the target tree;
void plan_batches(HostPlan& hp);
// the leaves of the source tree sorted by first position, and for every node
// the run [run_lo, run_hi) of that list holding the leaves below it (in
// depth-first order);
void leaf_runs(const Tree& S, std::vector<int32_t>& leaf_list, std::vector<int64_t>& run_lo,
               std::vector<int64_t>& run_hi);
// slots (clusters with modified charges, ascending id) from per-cluster flags;
void plan_slots(HostPlan& hp, const std::vector<uint8_t>& used);
// Chebyshev points out[slot][3][n+1] of the boxes of the listed clusters
// (c + h cos(pi k / n), k = 0 at the upper end);
void grid_nodes(const Tree& t, const std::vector<int32_t>& clusters, int32_t degree,
                std::vector<double>& out);
// upward-pass chunks (<= chunk_size sources) of the listed clusters: chunk_dst
// is the slot of a single-chunk cluster, else nslots + a partial row index;
void upward_chunks(const Tree& S, const std::vector<int32_t>& slot_cluster, int64_t chunk_size,
                   std::vector<int32_t>& chunk_slot, std::vector<int64_t>& chunk_begin,
                   std::vector<int64_t>& chunk_count, std::vector<int32_t>& slot_chunk_off,
                   std::vector<int64_t>& chunk_dst, int64_t& npartial);
// upward-pass chunks and the interaction workgroup schedule (needs the slots,
// batch counts and batch_cost).
void plan_schedule(HostPlan& hp);

// Workgroups of group_size consecutive positions over batches [begin, begin +
// count), cost-ordered per die (see planner.cpp); batch -1 marks padding.
void group_schedule(const std::vector<int64_t>& begin, const std::vector<int64_t>& count,
                    const std::vector<int64_t>& cost, int32_t group_size, int32_t xcds,
                    std::vector<int32_t>& group_batch, std::vector<int64_t>& group_first);

// ---------------------------------------------------------------------------
// Cluster-particle treecode: the interpolation moves to the target side.
// Targets form the cluster tree (capacity leaf_size); the leaves of the source
// tree (capacity batch_size) are the source batches, and every source batch
// walks the target tree with the MAC of eq. 13 (roles exchanged).  An
// approximated pair (S, T) adds the potential of S's sources at T's
// Chebyshev points (the proxy potentials of T); a direct pair adds S's direct
// sum to every target of T; every target finally receives the interpolant of
// the proxy potentials of each cluster on its root-to-leaf path.
// ---------------------------------------------------------------------------
struct CpPlan {
    PlanParams prm;
    int32_t np = 0;
    int64_t P = 0;
    Tree tgt, src;
    // targets are the sources (same arrays, same capacity); same_tree once the
    // two trees (and particle orders) are known to be identical
    bool same_arrays = false;
    bool same_tree = false;

    // source batches (leaves of the source tree) and target leaves, each
    // ordered by first position
    std::vector<int32_t> sb_node, tl_node;
    std::vector<int64_t> sb_begin, sb_count, tl_begin, tl_count;

    // items as found by the walks: source batch, target cluster, kind
    std::vector<int32_t> item_batch, item_cluster, item_kind;

    // slots: target clusters with proxy potentials (ascending id)
    std::vector<int32_t> slot_cluster, cluster_slot;
    std::vector<double> slot_nodes;      // [slot][3][np]

    // proxy potentials: per slot, the source ranges (source batches)
    std::vector<int32_t> pf_off, pf_leaf;
    std::vector<int64_t> pf_begin, pf_count, pf_cost;
    // direct sums: per target leaf, the source ranges
    std::vector<int32_t> dn_off, dn_leaf;
    std::vector<int64_t> dn_begin, dn_count, dn_cost;
    // interpolation: per target leaf, the slots on its root-to-leaf path (root first)
    std::vector<int32_t> dw_off, dw_slot;

    // workgroups: over proxy points (batch = slot) and over target leaves
    std::vector<int32_t> pg_batch, dg_batch;
    std::vector<int64_t> pg_first, dg_first;

    int64_t approx_pairs = 0, direct_pairs = 0;
    int64_t proxy_evals = 0, near_evals = 0, interp_terms = 0;
    int64_t leaves = 0;
    double setup_seconds = 0.0;
};

// Everything after the two trees (cp.prm, cp.tgt, cp.src set).
void cp_plan_from_trees(CpPlan& cp);

// Host planning of the cluster-particle treecode from host coordinates.
void make_cp_plan(CpPlan& cp, const PlanParams& prm,
                  int64_t nt, const double* tx, const double* ty, const double* tz,
                  int64_t ns, const double* sx, const double* sy, const double* sz);

// ---------------------------------------------------------------------------
// Cluster-cluster treecode: both sides interpolated.  Sources form a tree of
// capacity leaf_size (modified charges), targets a tree of capacity
// batch_size (proxy potentials).  A dual walk from the roots accepts pairs
// with the MAC of eq. 13 and approximates every side larger than (n+1)^3:
// kind 0 cluster-cluster, 1 particle-cluster, 2 cluster-particle, 3 direct.
// Rejected pairs split the larger non-leaf cluster (both when the radii are
// equal) until two leaves meet, which are summed directly.
// ---------------------------------------------------------------------------
struct CcPlan {
    PlanParams prm;
    int32_t np = 0;
    int64_t P = 0;
    Tree tgt, src;

    // pairs in walk order
    std::vector<int32_t> pair_t, pair_s, pair_kind;

    // source slots: source clusters in kind 0 or 1 pairs (ascending id), their
    // grids and upward-pass chunks
    std::vector<int32_t> sslot_cluster, cluster_sslot;
    std::vector<double> sslot_nodes;
    std::vector<int32_t> chunk_slot, slot_chunk_off;
    std::vector<int64_t> chunk_begin, chunk_count, chunk_dst;
    int64_t npartial = 0;

    // target slots: target clusters in kind 0 or 2 pairs (ascending id)
    std::vector<int32_t> tslot_cluster, cluster_tslot;
    std::vector<double> tslot_nodes;

    // proxy potentials, per target slot: the source slots of its grid-grid
    // pairs (evaluated like the far field, eq. 11, at the grid points) and
    // the particle ranges (source leaves) of its sources-grid pairs
    std::vector<int32_t> gg_off, gg_slot;
    std::vector<int32_t> pf_off, pf_leaf;
    std::vector<int64_t> pf_begin, pf_count, pf_cost;

    // target leaves ordered by first position; per leaf the particle-cluster
    // source slots and the direct source ranges of every cluster on its path
    std::vector<int32_t> tl_node;
    std::vector<int64_t> tl_begin, tl_count;
    std::vector<int32_t> far_off, far_slot;
    std::vector<int32_t> dn_off, dn_leaf;
    std::vector<int64_t> dn_begin, dn_count, dn_cost;
    // interpolation: per target leaf, the target slots on its path (root first)
    std::vector<int32_t> dw_off, dw_slot;

    // workgroups: over proxy points (batch = target slot) and over target leaves
    std::vector<int32_t> pg_batch, dg_batch;
    std::vector<int64_t> pg_first, dg_first;

    // targets are the sources (same arrays, same capacity): one tree
    bool same_tree = false;

    int64_t kind_pairs[4] = {0, 0, 0, 0};
    int64_t cc_evals = 0, pc_evals = 0, cp_evals = 0, near_evals = 0;
    int64_t upward_terms = 0, interp_terms = 0;
    double setup_seconds = 0.0;
};

// Everything after the two trees (cc.prm, cc.tgt, cc.src set).
void cc_plan_from_trees(CcPlan& cc);

// Host planning of the cluster-cluster treecode from host coordinates.
void make_cc_plan(CcPlan& cc, const PlanParams& prm,
                  int64_t nt, const double* tx, const double* ty, const double* tz,
                  int64_t ns, const double* sx, const double* sy, const double* sz);

}  // namespace bltc
