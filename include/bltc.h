/*
 * bltc.h -- C ABI of the MI355X (gfx950) barycentric Lagrange treecode library.
 *
 * The library evaluates potentials
 *     phi(x_i) = sum_j G(x_i, y_j) q_j,  G = 1/r (Coulomb) or exp(-kappa r)/r (Yukawa)
 * or, since the method needs only kernel values, 1/sqrt(r^2 + delta^2)
 * (regularized Coulomb)
 * (Vaughn, Wilson, Krasny 2020, Sec. II, eqs. 1-2) with the barycentric Lagrange
 * treecode of Alg. 1: a tree of source clusters and a set of target batches
 * (Sec. II-D), modified charges on each cluster's (n+1)^3 tensor grid of
 * Chebyshev points of the 2nd kind (eqs. 6-7, 12; computed in the two-step form
 * of eqs. 14-15 with the removable-singularity rule of eq. 5), then for every
 * batch/cluster pair either the approximation of eq. 11 (MAC of eq. 13 holds)
 * or the direct sum of eq. 9 (it fails).  The same interpolation applied to
 * the target variable (the cluster-particle treecode that the paper's outlook,
 * Sec. V, names) is available as a second method, the cluster-cluster
 * treecode as a third, and the barycentric Hermite treecode (also named in
 * Sec. V: kernel derivatives on the same grids) as a fourth.
 *
 * Conventions shared by every entry point:
 *  - Counts are int64_t.  Coordinates are structure-of-arrays FP64: x, y, z are
 *    three separate arrays of length n.
 *  - Charge vectors: q[m * q_ld + j] is charge j of vector m (q_ld >= ns).
 *    Potentials: phi[m * phi_ld + i] is the potential at target i for charge
 *    vector m (phi_ld >= nt).
 *  - Unless an entry point says otherwise, every array pointer is a DEVICE
 *    pointer (HIP device memory, e.g. a ROCm torch tensor) on the current
 *    HIP device, and `stream` is a hipStream_t passed as void* (NULL = the
 *    default stream).  Work is enqueued on `stream`; results are ready when the
 *    stream is synchronised.
 *  - Ownership: the caller owns every input and output buffer.  Inputs are
 *    never modified.  Outputs are overwritten (not accumulated).  The library
 *    keeps no pointer to a caller buffer after a call returns.
 *  - Errors: a negative bltc_status is returned and a message is stored for
 *    the calling thread (bltc_last_error).  No C++ exception crosses this ABI.
 *    Faults of kernels already enqueued surface as BLTC_EHIP on a later call
 *    that synchronises.
 */
#ifndef BLTC_H
#define BLTC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BLTC_OK = 0,
    BLTC_EINVAL = -1,        /* invalid argument (message says which)              */
    BLTC_ENOMEM = -2,        /* host or device allocation failed                     */
    BLTC_EHIP = -3,          /* a HIP runtime call failed                            */
    BLTC_EUNSUPPORTED = -4,  /* valid request the library does not support           */
    BLTC_EINTERNAL = -5      /* internal consistency check failed                    */
} bltc_status;

/* Kernels (eq. 2 and one more smooth, non-oscillatory example): pairs at
 * exactly zero distance are skipped for all of them. */
typedef enum {
    BLTC_COULOMB = 0,              /* 1/r                                     */
    BLTC_YUKAWA = 1,               /* exp(-kappa r)/r                         */
    BLTC_REGULARIZED_COULOMB = 2   /* 1/sqrt(r^2 + delta^2)                   */
} bltc_kernel;

/* Arithmetic of the evaluation.
 *  BLTC_FP64        every step in FP64.
 *  BLTC_FP32_MIXED  kernel evaluations in FP32 on local coordinates, partial
 *                   sums over at most one cluster in FP32, accumulated per target
 *                   in FP64; barycentric factors, the coincidence branch and
 *                   pairs closer than a fixed cut-off stay FP64.  All points
 *                   must lie in a box of side at most 2^60 (squared FP32
 *                   distances stay finite); plan creation returns
 *                   BLTC_EUNSUPPORTED otherwise.  A target closer than about
 *                   1e-19 to a Chebyshev point of an approximated cluster
 *                   (possible only for clusters of coincident points) loses
 *                   that term: use BLTC_FP64 for such data. */
typedef enum { BLTC_FP64 = 0, BLTC_FP32_MIXED = 1 } bltc_precision;

/* Which side is interpolated.
 *  BLTC_PARTICLE_CLUSTER  the paper's BLTC (Alg. 1): source clusters carry
 *                         modified charges (eq. 12) on their Chebyshev grids,
 *                         targets are grouped in batches.
 *  BLTC_CLUSTER_PARTICLE  targets form the cluster tree and sources the
 *                         batches: an approximated (source batch S, target
 *                         cluster T) pair adds the potential of S at T's
 *                         Chebyshev points; every target then receives the
 *                         barycentric interpolant (eqs. 4-5) of the proxy
 *                         potentials of each cluster on its root-to-leaf path.
 *                         MAC of eq. 13 with the roles exchanged:
 *                         r_S + r_T < theta R and (n+1)^3 < N_T.  One charge
 *                         vector per execution; not usable in a bltc_batch.
 *  BLTC_CLUSTER_CLUSTER   both sides interpolated: source tree of capacity
 *                         N_L (modified charges), target tree of capacity N_B
 *                         (proxy potentials).  A dual walk from the roots
 *                         accepts pairs with r_T + r_S < theta R and
 *                         approximates every side with more than (n+1)^3
 *                         particles (grid to grid, grid to targets, sources
 *                         to grid, or a direct sum when neither); rejected
 *                         pairs split the larger non-leaf cluster (both when
 *                         the radii are equal) until two leaves meet, which
 *                         are summed directly.  One charge vector per
 *                         execution; not usable in a bltc_batch.
 *  BLTC_HERMITE           particle-cluster as BLTC_PARTICLE_CLUSTER, with the
 *                         tensor-product Hermite interpolant on the same
 *                         Chebyshev grids: per dimension A_k = (1 - 2 c_k (y -
 *                         s_k)) L_k^2 and B_k = (y - s_k) L_k^2, L_k of eq. 4,
 *                         c_k = sum_{j != k} 1/(s_k - s_j).  A cluster carries
 *                         8 (n+1)^3 modified charges, one per grid point k
 *                         and derivative multi-index a in {0,1}^3, and the
 *                         approximation sums d^a_y G(x, s_k) times them; the
 *                         size part of the MAC compares 8 (n+1)^3 with N_C.
 *                         BLTC_FP64 or BLTC_FP32_MIXED (the far-field terms in
 *                         FP32 from FP64-formed 1-D distances and FP32 copies
 *                         of the charges, direct sums as for the BLTC), degree
 *                         1..10, one charge vector per execution; not usable
 *                         in a bltc_batch. */
typedef enum {
    BLTC_PARTICLE_CLUSTER = 0,
    BLTC_CLUSTER_PARTICLE = 1,
    BLTC_CLUSTER_CLUSTER = 2,
    BLTC_HERMITE = 3
} bltc_method;

typedef struct {
    int32_t kernel;              /* bltc_kernel                                         */
    int32_t precision;           /* bltc_precision                                      */
    double kappa;                /* Yukawa inverse Debye length, >= 0 (eq. 2)           */
    double theta;                /* MAC parameter, 0 <= theta < 1 (eq. 13); 0 = direct  */
    int32_t degree;              /* interpolation degree n, 1..16 (eqs. 6-8)            */
    int32_t leaf_size;           /* N_L >= 1: leaf capacity of the interpolated side's  */
                                 /* cluster tree (sources; targets for CLUSTER_PARTICLE) */
    int32_t batch_size;          /* N_B >= 1: capacity of the batches of the other side */
                                 /* leaf_size = batch_size = 0: picked by the library's */
                                 /* tuner (bltc_autotune over 1000, 2000, 3000, 4000,   */
                                 /* cached) when a plan is created from device          */
                                 /* coordinates; BLTC_EUNSUPPORTED for host plans.      */
                                 /* One of them 0 and the other not: BLTC_EINVAL        */
    int32_t threads_per_target;  /* 1: one lane per target; 2 or 4: each batch's        */
                                 /* interaction lists cut into that many contiguous     */
                                 /* pieces, each evaluated by its own lane of the       */
                                 /* target (in different waves) into a partial          */
                                 /* potential, summed per target in piece order: more   */
                                 /* waves for problems with few targets.                */
                                 /* BLTC_PARTICLE_CLUSTER and BLTC_HERMITE with         */
                                 /* max_q = 1 only.  0: picked by the tuner among 1, 2, */
                                 /* 4 for those plans when created from device          */
                                 /* coordinates; one lane otherwise                     */
    int32_t method;              /* bltc_method                                         */
    double delta;                /* BLTC_REGULARIZED_COULOMB length, >= 0               */
    int32_t no_symmetry;         /* 0: when the targets are the sources (same arrays,   */
                                 /* N_B = N_L), methods BLTC_PARTICLE_CLUSTER,          */
                                 /* BLTC_HERMITE (max_q = 1) and BLTC_CLUSTER_CLUSTER   */
                                 /* evaluate each pair of different leaves that are in  */
                                 /* each other's direct lists once for both directions  */
                                 /* (G(x,y) = G(y,x)); 1: never.  Same potentials up to */
                                 /* rounding order.  The pair results take 8 B per     */
                                 /* target and pair; when they exceed 16 GiB (or what  */
                                 /* workspace_limit leaves), the pairs run in rounds   */
                                 /* through a workspace of that size, each round       */
                                 /* folded into per-target sums in a fixed order.      */
                                 /* Pairs whose results alone exceed 4 GiB stay in the */
                                 /* plain direct lists.                                 */
    int64_t workspace_limit;     /* bytes of device memory a plan may hold (requested   */
                                 /* sizes of its arrays; transient scratch of the setup */
                                 /* phase not counted); 0: no limit.  A plan whose      */
                                 /* arrays do not fit fails with BLTC_ENOMEM, also when */
                                 /* the limit leaves no room for the results of its     */
                                 /* largest mutual pair (set no_symmetry then); the     */
                                 /* mutual-pair results take what the other arrays      */
                                 /* leave, in rounds if needed.  Same potentials up to  */
                                 /* rounding order for every limit that fits.           */
} bltc_params;

/* Fills *p with the defaults: Coulomb, FP64, theta 0.7, degree 8,
 * N_L = N_B = 2000, one thread per target, BLTC_PARTICLE_CLUSTER,
 * kappa = delta = 0, no workspace limit. */
void bltc_params_default(bltc_params* p);

/* One-shot evaluation (Alg. 1): builds the tree, batches and interaction lists
 * (on the GPU, as bltc_plan_create), then computes phi[m*phi_ld + i],
 * m < num_q, on the GPU.  Synchronises `stream`.
 * nt == 0 is a no-op; ns == 0 writes zeros.  Coordinates must be finite
 * (BLTC_EINVAL otherwise). */
int bltc_potential(const bltc_params* p,
                   int64_t nt, const double* tx, const double* ty, const double* tz,
                   int64_t ns, const double* sx, const double* sy, const double* sz,
                   const double* q, int32_t num_q, int64_t q_ld,
                   double* phi, int64_t phi_ld, void* stream);

/* A plan fixes the geometry (trees, batches, lists, device copies of the
 * coordinates in tree order) so that charges can vary between executions. */
typedef struct bltc_plan bltc_plan;

/* Creates a plan from DEVICE coordinates.  The setup phase runs on the GPU
 * on `stream`: both trees are built there (only per-node data comes back to
 * the host, which takes the split decisions), and for BLTC_PARTICLE_CLUSTER
 * the interaction lists of Alg. 1 are built there as well; particles are
 * written in tree order directly into the plan's device arrays.  The result
 * equals the plan bltc_plan_create_host builds from the same coordinates.
 * Synchronises `stream`.  max_q >= 1 bounds num_q of later executions
 * (max_q must be 1 for every method but BLTC_PARTICLE_CLUSTER).  At most 2^31 - 1 particles
 * per side.  Non-finite coordinates: BLTC_EINVAL. */
int bltc_plan_create(bltc_plan** out, const bltc_params* p,
                     int64_t nt, const double* tx, const double* ty, const double* tz,
                     int64_t ns, const double* sx, const double* sy, const double* sz,
                     int32_t max_q, void* stream);

/* Same as bltc_plan_create but the coordinates are HOST pointers and no HIP
 * call is made: the plan holds only its host side (trees, batches, lists) and
 * uploads its device side on its first execution.  Usable without a GPU for
 * inspection (bltc_plan_view, bltc_plan_stats). */
int bltc_plan_create_host(bltc_plan** out, const bltc_params* p,
                          int64_t nt, const double* tx, const double* ty, const double* tz,
                          int64_t ns, const double* sx, const double* sy, const double* sz,
                          int32_t max_q);

/* Evaluates the upward pass (eqs. 14-15) and all batch/cluster interactions
 * (eqs. 9 and 11) for num_q <= max_q charge vectors q (device, caller order),
 * writing phi (device, caller order).  Enqueued on `stream`; does not
 * synchronise. */
int bltc_plan_execute(bltc_plan* plan, const double* q, int32_t num_q, int64_t q_ld,
                      double* phi, int64_t phi_ld, void* stream);

/* Copies the modified charges (eq. 12) that the last execution formed for
 * source cluster `cluster` (an index into the cluster arrays of
 * bltc_plan_view) and charge vector `qi` into the HOST buffer out[(n+1)^3],
 * ordered k = (k1*(n+1) + k2)*(n+1) + k3.  Synchronises `stream`.
 * BLTC_EINVAL if the cluster is in no approximation list (no charges formed).
 * For BLTC_CLUSTER_PARTICLE plans `cluster` is a target cluster and out
 * receives its proxy potentials (qi = 0); for BLTC_CLUSTER_CLUSTER plans it is
 * a node of the target tree (a batch index of bltc_plan_view) and out
 * receives its proxy potentials.  For BLTC_HERMITE plans out holds
 * 8 (n+1)^3 values, out[8 k + a] with a = 4 a1 + 2 a2 + a3 the derivative
 * multi-index. */
int bltc_plan_modified_charges(bltc_plan* plan, int64_t cluster, int32_t qi,
                               double* out, void* stream);

/* For BLTC_CLUSTER_PARTICLE plans the cluster fields describe the target
 * tree, the batches are the source batches, far_evals counts the proxy
 * potential evaluations (sum over approx pairs of (n+1)^3 * N_S) and
 * upward_terms the interpolation terms (sum over approx clusters of
 * N_T * (n+1)^3). */
typedef struct {
    int64_t clusters;        /* source clusters in the tree                         */
    int64_t leaves;          /* leaf clusters                                       */
    int64_t batches;         /* target batches                                      */
    int64_t approx_pairs;    /* batch/cluster pairs evaluated with eq. 11           */
    int64_t direct_pairs;    /* batch/cluster pairs evaluated with eq. 9            */
    int64_t approx_clusters; /* clusters that need modified charges                 */
    int64_t far_evals;       /* sum over approx pairs of N_B * (n+1)^3               */
    int64_t near_evals;      /* sum over direct pairs of N_B * N_C                   */
    int64_t upward_terms;    /* sum over approx clusters of N_C * (n+1)^3            */
    int32_t depth;           /* deepest cluster-tree level (root = 0)               */
    int32_t degree;
    int32_t leaf_size;
    int32_t batch_size;
    double setup_seconds;    /* planning time (trees and lists)                     */
    int64_t mutual_pair_evals; /* kernel values computed once for two direct terms:   */
                             /* sum over mutual leaf pairs of N_B * N_C (no_symmetry */
                             /* = 0; counted once the device side exists), else 0    */
    int32_t threads_per_target; /* lanes per target of the interaction launch (1, 2, 4) */
    int64_t workspace_bytes; /* device memory the plan holds (requested bytes; 0 before */
                             /* the device side exists)                              */
    int64_t mutual_pairs;    /* mutual leaf pairs evaluated once (no_symmetry = 0)      */
    int64_t pair_workspace_bytes; /* part of workspace_bytes for their results         */
    int32_t pair_rounds;     /* rounds of mutual-pair results (1: all at once)          */
} bltc_stats;

int bltc_plan_stats(const bltc_plan* plan, bltc_stats* out);

/* Phase timing of executions (the paper's precompute / compute split,
 * Sec. IV).  With timing enabled, bltc_plan_execute records HIP events on its
 * stream around each phase; bltc_plan_phase_times waits for the last
 * execution's events and writes its device milliseconds:
 *   ms[0] charges gathered into tree order, ms[1] upward pass (eqs. 14-15),
 *   ms[2] batch/cluster interactions (eqs. 9, 11), ms[3] total, ms[4] the
 *   part of ms[2] spent on mutual direct leaf pairs (see no_symmetry; 0 when
 *   the execution had none).
 * BLTC_EINVAL if timing is off or nothing was executed since it was enabled. */
int bltc_plan_set_timing(bltc_plan* plan, int32_t enable);
int bltc_plan_phase_times(bltc_plan* plan, double* ms /* [5] */);

/* Read-only HOST view of a plan's structure (valid until the plan is
 * destroyed).  Cluster ids index the cluster arrays; the children of cluster c
 * are cluster_first_child[c] .. + cluster_nchild[c] - 1.  For plans built on
 * the GPU the orders and items are copied to the host on the first call.
 * For BLTC_CLUSTER_PARTICLE plans the clusters are the target tree's nodes
 * (cluster_begin/count index target_order), the batches are the source
 * batches (batch_begin/count index source_order) and an item is (source
 * batch, target cluster, kind).  For BLTC_CLUSTER_CLUSTER plans the clusters
 * are the source tree's nodes, the batches ALL nodes of the target tree, and
 * an item is a pair of the dual walk (target node, source node, kind 0
 * grid-grid, 1 grid-targets, 2 sources-grid, 3 direct). */
typedef struct {
    int64_t nt, ns, n_clusters, n_batches, n_items;
    const int64_t* source_order;        /* [ns] original index at tree position    */
    const int64_t* target_order;        /* [nt] original index at batch position   */
    const int64_t* cluster_begin;       /* [n_clusters] first tree position        */
    const int64_t* cluster_count;       /* [n_clusters]                           */
    const double* cluster_lo;           /* [3*n_clusters] minimal box, x,y,z      */
    const double* cluster_hi;           /* [3*n_clusters]                         */
    const int32_t* cluster_first_child; /* [n_clusters] -1 for leaves             */
    const int32_t* cluster_nchild;      /* [n_clusters]                           */
    const int32_t* cluster_level;       /* [n_clusters]                           */
    const int64_t* batch_begin;         /* [n_batches] first batch position       */
    const int64_t* batch_count;         /* [n_batches]                            */
    const double* batch_lo;             /* [3*n_batches]                          */
    const double* batch_hi;             /* [3*n_batches]                          */
    const int32_t* item_batch;          /* [n_items]                              */
    const int32_t* item_cluster;        /* [n_items]                              */
    const int32_t* item_kind;           /* [n_items] 0 = approximation, 1 = direct */
} bltc_plan_view;

int bltc_plan_view_get(const bltc_plan* plan, bltc_plan_view* out);

void bltc_plan_destroy(bltc_plan* plan);

/* Many independent systems in one evaluation.  A batch is built from plans
 * (one per system; each created with max_q >= 2, all with the same kernel and
 * precision; the plans stay owned by the caller and must outlive the batch).
 * bltc_batch_execute evaluates, for every system i, num_q[i] <= min(16, max_q)
 * charge vectors q[i] (device, q_ld[i]) into phi[i] (device, phi_ld[i]):
 * per-system charge gathers, one matrix-core upward pass (eqs. 14-15) over
 * the chunks of all systems, and ONE persistent work-queue launch over every
 * batch/cluster work unit of every system (eqs. 9, 11), heaviest first.  The
 * sequence is captured into a hipGraph the first time a given set of
 * buffers/counts is seen and replayed afterwards (a new set of buffers is
 * re-captured; that call synchronises `stream`).  Enqueued on `stream`.
 * Calls on one batch must not overlap.  BLTC_EINVAL on mismatched plans,
 * counts or NULL buffers; BLTC_ENOMEM when a host or device allocation of the
 * batch tables fails (no C++ exception leaves any bltc_* call). */
typedef struct bltc_batch bltc_batch;

typedef struct {
    int32_t systems;         /* plans in the batch                                  */
    int32_t units;           /* work-queue units (system, 256-target group)         */
    int32_t upward_units;    /* upward-pass chunks over all systems                 */
    int32_t workgroups;      /* persistent workgroups of the work-queue launch      */
    int64_t graph_captures;  /* hipGraphs captured so far                           */
    int64_t launches;        /* executions so far                                   */
} bltc_batch_info;

int bltc_batch_create(bltc_batch** out, bltc_plan* const* plans, int32_t count, void* stream);
/* One-shot form over plans[]: builds a batch of the `count` plans, evaluates
 * it once as bltc_batch_execute (no hipGraph), synchronises `stream` and
 * frees the batch.  For repeated evaluations keep a bltc_batch, which owns
 * the work-queue tables and the captured graph between calls. */
int bltc_batch_potential(bltc_plan* const* plans, int32_t count, const double* const* q,
                         const int32_t* num_q, const int64_t* q_ld, double* const* phi,
                         const int64_t* phi_ld, void* stream);
int bltc_batch_execute(bltc_batch* batch, const double* const* q, const int32_t* num_q,
                       const int64_t* q_ld, double* const* phi, const int64_t* phi_ld,
                       void* stream);
/* enable (default) or disable the hipGraph; without it every call enqueues
 * the launches directly */
int bltc_batch_set_graph(bltc_batch* batch, int32_t enable);
int bltc_batch_info_get(const bltc_batch* batch, bltc_batch_info* out);
void bltc_batch_destroy(bltc_batch* batch);

/* The library's tuner for the leaf and batch size (kept equal) and the
 * threads per target: for the given DEVICE coordinates it builds a plan for
 * each of the `ncand` candidate sizes, times one evaluation of `num_q`
 * (1..16) charge vectors on `stream` after a warm-up, and writes the fastest
 * into out->leaf_size and out->batch_size (the other fields are copied from
 * *p) and its device time into *best_ms.  For BLTC_PARTICLE_CLUSTER and
 * BLTC_HERMITE with num_q = 1 and p->threads_per_target = 0 it then times 2
 * and 4 threads per target at that size and writes the fastest of 1, 2, 4
 * into out->threads_per_target.  With use_cache != 0 the choice is looked up
 * in / appended to a text cache keyed by the problem class (method, log2 of
 * the counts, theta, degree, kernel, precision, one or several vectors,
 * whether threads per target are searched); the file is
 * $BLTC_TUNE_CACHE, else $HOME/.bltc_tune_cache.  Synchronises `stream`.
 * Theta and n set the accuracy; the leaf size only moves which pairs are
 * approximated.  Candidates below (n+1)^3 can never be approximated as
 * leaves. */
int bltc_autotune(const bltc_params* p,
                  int64_t nt, const double* tx, const double* ty, const double* tz,
                  int64_t ns, const double* sx, const double* sy, const double* sz,
                  int32_t num_q, const int32_t* candidates, int32_t ncand, int32_t use_cache,
                  bltc_params* out, double* best_ms, void* stream);

/* GPU direct sum of eq. 1 (all pairs, pairs at zero distance skipped), FP64:
 * phi[m*phi_ld + i] for m < num_q.  Diagnostic / baseline path.  Enqueued on
 * `stream`. */
int bltc_direct(const bltc_params* p,
                int64_t nt, const double* tx, const double* ty, const double* tz,
                int64_t ns, const double* sx, const double* sy, const double* sz,
                const double* q, int32_t num_q, int64_t q_ld,
                double* phi, int64_t phi_ld, void* stream);

/* bltc_direct without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, checks and results as bltc_direct; the
 * per-vector staging of the sources (x, y, z, q records, 32 B per source)
 * goes to a fixed array of 2^20 records (32 MiB) in device memory, one per GPU,
 * that the library holds until the process ends.  ns > 2^20 returns
 * BLTC_EUNSUPPORTED (use bltc_direct).  Calls no hipMalloc/hipFree; the first
 * call on a device looks up that device's address of the array.  All calls on
 * one GPU share its array: calls that overlap in time on one GPU (different
 * streams, or host threads) race and must be serialised by the caller.
 * Enqueued on `stream`. */
int bltc_direct_noalloc(const bltc_params* p,
                        int64_t nt, const double* tx, const double* ty, const double* tz,
                        int64_t ns, const double* sx, const double* sy, const double* sz,
                        const double* q, int32_t num_q, int64_t q_ld,
                        double* phi, int64_t phi_ld, void* stream);

const char* bltc_status_string(int code);
const char* bltc_last_error(void);     /* message of the calling thread's last failure */
const char* bltc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BLTC_H */
