/*
 * bltc_oracle.c -- CPU oracle for the barycentric Lagrange treecode (BLTC).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, FP64 reference that
 * the GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library, and it never reads anything the GPU
 * library produced.
 *
 * What it computes (Vaughn, Wilson, Krasny, "A GPU-Accelerated Barycentric
 * Lagrange Treecode", 2020):
 *   - the direct sum phi_i = sum_j G(x_i, y_j) q_j                 (Sec. II, eq. 1)
 *     with G = 1/r (Coulomb) or exp(-kappa r)/r (Yukawa)             (eq. 2),
 *     or the regularized Coulomb kernel 1/sqrt(r^2 + delta^2);
 *   - the BLTC of Alg. 1: source-cluster tree and target batches
 *     (Sec. II-D), modified charges on each cluster's tensor grid of
 *     Chebyshev points of the 2nd kind (eqs. 4-7, 12) with the
 *     removable-singularity rule (eq. 5, Sec. II-C), and the recursive
 *     ComputePotential with the two-part MAC (eq. 13): the approximation
 *     (eq. 11) when it holds, the direct particle sum (eq. 9) when it fails.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   R1  pairs at exactly zero distance are skipped (self term, duplicates);
 *   R2  cluster/batch center = midpoint of its minimal bounding box,
 *       radius = half the box diagonal;
 *   R3  MAC evaluated as r_B + r_C < theta * R (false when R = 0), strict "<"
 *       in both parts, R = sqrt(dx*dx + dy*dy + dz*dz) summed x, y, z;
 *   R4  branch order of Alg. 1 as printed: a geometric failure recurses into
 *       the children of a non-leaf cluster even when the size test also fails;
 *       a size-only failure is a direct sum over the whole cluster;
 *   R5  a coordinate on the split plane (y_l >= c_l) goes to the upper child;
 *   R6  aspect-ratio rule (Sec. III-A) applied to every node: dimension l is
 *       split iff 2 L_l^2 >= L_max^2, L_l = hi_l - lo_l;
 *   R7  every node shrinks to the minimal box of its own particles;
 *   R8  leaf iff N_C <= N_L, or L_max = 0, or the split leaves every particle
 *       in one child (possible only for boxes a few ulps wide);
 *   R9  a source coordinate coincides with a node when |y - s| < DBL_MIN
 *       (the smallest positive normal double); the lowest such k wins;
 *   R10 nodes s_k = c + h cos(pi k / n), h = (hi - lo)/2, k = 0..n (k = 0 at
 *       the upper end), weights w_k = (-1)^k delta_k;
 *   R11 modified charges are formed for every cluster that appears in some
 *       approximation list (the same values Alg. 1 forms for all clusters);
 *   R24 the regularized Coulomb kernel 1/sqrt(r^2 + delta^2) follows R1 as
 *       well (pairs at exactly zero distance are skipped).
 *
 * Floating point: plain FP64, compiled without contraction so that the tree
 * and MAC decisions follow the formulas above operation by operation.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_COULOMB 0
#define ORACLE_YUKAWA 1
#define ORACLE_REGULARIZED 2

static double wall_seconds(void)
{
#ifdef _OPENMP
    return omp_get_wtime();
#else
    return 0.0;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Kernel G(x, y) as a function of r = |x - y|: Coulomb 1/r and Yukawa        */
/* exp(-kappa r)/r (eq. 2).  The method needs only kernel values (Sec. II),   */
/* so any kernel smooth away from r = 0 and not oscillatory fits; the         */
/* regularized Coulomb kernel 1/sqrt(r^2 + delta^2) (reading R24; delta is    */
/* passed as the kernel parameter in place of kappa) is the third one built.  */
/* ------------------------------------------------------------------------- */
static double kernel_of_distance(double r, int kernel, double kappa)
{
    if (kernel == ORACLE_YUKAWA)
        return exp(-kappa * r) / r;
    if (kernel == ORACLE_REGULARIZED)
        return 1.0 / sqrt(r * r + kappa * kappa);
    return 1.0 / r;
}

/* ------------------------------------------------------------------------- */
/* Direct sum, eq. (1): phi[m*phi_ld + i] = sum_j G(x_i, y_j) q[m*q_ld + j],  */
/* skipping pairs at exactly zero distance (reading R1).                      */
/* ------------------------------------------------------------------------- */
void oracle_direct(int64_t nt, const double *tx, const double *ty, const double *tz,
                   int64_t ns, const double *sx, const double *sy, const double *sz,
                   const double *q, int32_t m, int64_t q_ld,
                   int32_t kernel, double kappa, double *phi, int64_t phi_ld)
{
    int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < nt; ++i) {
        for (int32_t c = 0; c < m; ++c) {
            double sum = 0.0;
            for (int64_t j = 0; j < ns; ++j) {
                double dx = tx[i] - sx[j];
                double dy = ty[i] - sy[j];
                double dz = tz[i] - sz[j];
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                if (r == 0.0)
                    continue;
                sum += kernel_of_distance(r, kernel, kappa) * q[(int64_t)c * q_ld + j];
            }
            phi[(int64_t)c * phi_ld + i] = sum;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* 1-D Chebyshev points of the 2nd kind on [a, b] and their barycentric       */
/* weights, eqs. (6)-(7) with the linear map of Sec. II-A (reading R10).      */
/* ------------------------------------------------------------------------- */
void oracle_chebyshev(int32_t n, double a, double b, double *s, double *w)
{
    double c = (a + b) / 2.0;
    double h = (b - a) / 2.0;
    for (int32_t k = 0; k <= n; ++k) {
        s[k] = c + h * cos(M_PI * (double)k / (double)n);
        double delta = (k == 0 || k == n) ? 0.5 : 1.0;
        w[k] = ((k % 2) ? -1.0 : 1.0) * delta;
    }
}

/* L_k(x), k = 0..n, by the barycentric formula eq. (4), with the removable
 * singularity eq. (5) enforced when |x - s_k'| < DBL_MIN (reading R9). */
void oracle_lagrange(int32_t n, const double *s, const double *w, double x, double *L)
{
    for (int32_t k = 0; k <= n; ++k) {
        if (fabs(x - s[k]) < DBL_MIN) {
            for (int32_t kk = 0; kk <= n; ++kk)
                L[kk] = (kk == k) ? 1.0 : 0.0;
            return;
        }
    }
    double denom = 0.0;
    for (int32_t k = 0; k <= n; ++k)
        denom += w[k] / (x - s[k]);
    for (int32_t k = 0; k <= n; ++k)
        L[k] = (w[k] / (x - s[k])) / denom;
}

/* ------------------------------------------------------------------------- */
/* Trees (Sec. II-D, Sec. III-A), readings R2, R5-R8.                         */
/* ------------------------------------------------------------------------- */
typedef struct {
    double lo[3], hi[3], center[3], radius;
    int64_t begin, count;   /* range in the tree's permuted index array */
    int32_t child[8];
    int32_t nchild;
    int32_t level;
} onode;

typedef struct {
    onode *nodes;
    int64_t n_nodes, cap_nodes;
    int64_t *idx;           /* idx[p] = original index of the particle at tree position p */
    int64_t n;
} otree;

static int32_t tree_new_node(otree *t)
{
    if (t->n_nodes == t->cap_nodes) {
        t->cap_nodes = t->cap_nodes ? 2 * t->cap_nodes : 64;
        t->nodes = (onode *)realloc(t->nodes, (size_t)t->cap_nodes * sizeof(onode));
    }
    memset(&t->nodes[t->n_nodes], 0, sizeof(onode));
    return (int32_t)t->n_nodes++;
}

static void tree_split(otree *t, const double *const p[3], int32_t id, int64_t cap,
                       int64_t *scratch)
{
    onode *nd = &t->nodes[id];
    int64_t begin = nd->begin, count = nd->count;

    /* minimal bounding box of this node's particles (R7) */
    for (int l = 0; l < 3; ++l) {
        nd->lo[l] = INFINITY;
        nd->hi[l] = -INFINITY;
    }
    for (int64_t a = begin; a < begin + count; ++a) {
        int64_t i = t->idx[a];
        for (int l = 0; l < 3; ++l) {
            double v = p[l][i];
            if (v < nd->lo[l]) nd->lo[l] = v;
            if (v > nd->hi[l]) nd->hi[l] = v;
        }
    }
    double L[3];
    for (int l = 0; l < 3; ++l) {
        nd->center[l] = (nd->lo[l] + nd->hi[l]) / 2.0;
        L[l] = nd->hi[l] - nd->lo[l];
    }
    nd->radius = 0.5 * sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
    nd->nchild = 0;
    double Lmax = L[0];
    if (L[1] > Lmax) Lmax = L[1];
    if (L[2] > Lmax) Lmax = L[2];
    if (count <= cap || Lmax == 0.0)
        return;

    int split[3];
    for (int l = 0; l < 3; ++l)
        split[l] = (2.0 * L[l] * L[l] >= Lmax * Lmax);

    /* child code: bit l set iff dimension l is split and y_l >= c_l (R5) */
    int64_t nb[8] = {0};
    for (int64_t a = begin; a < begin + count; ++a) {
        int64_t i = t->idx[a];
        int code = 0;
        for (int l = 0; l < 3; ++l)
            if (split[l] && p[l][i] >= nd->center[l])
                code |= 1 << l;
        scratch[a - begin] = code;
        nb[code]++;
    }
    int nonempty = 0;
    for (int c = 0; c < 8; ++c)
        nonempty += nb[c] > 0;
    if (nonempty <= 1)
        return; /* degenerate split: leaf (R8) */

    /* stable partition of this node's range by child code */
    int64_t off[8], pos = 0;
    for (int c = 0; c < 8; ++c) {
        off[c] = pos;
        pos += nb[c];
    }
    int64_t *tmp = (int64_t *)malloc((size_t)count * sizeof(int64_t));
    for (int64_t a = 0; a < count; ++a)
        tmp[off[scratch[a]]++] = t->idx[begin + a];
    memcpy(t->idx + begin, tmp, (size_t)count * sizeof(int64_t));
    free(tmp);

    int64_t start = begin;
    int32_t kids[8];
    int nk = 0;
    int32_t level = nd->level;
    for (int c = 0; c < 8; ++c) {
        if (nb[c] == 0)
            continue;
        int32_t cid = tree_new_node(t);     /* may move t->nodes */
        t->nodes[cid].begin = start;
        t->nodes[cid].count = nb[c];
        t->nodes[cid].level = level + 1;
        kids[nk++] = cid;
        start += nb[c];
    }
    nd = &t->nodes[id];
    nd->nchild = nk;
    for (int c = 0; c < nk; ++c)
        nd->child[c] = kids[c];
    for (int c = 0; c < nk; ++c)
        tree_split(t, p, kids[c], cap, scratch);
}

static void tree_build(otree *t, int64_t n, const double *x, const double *y, const double *z,
                       int64_t cap)
{
    memset(t, 0, sizeof(*t));
    t->n = n;
    t->idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        t->idx[i] = i;
    if (n == 0)
        return;
    const double *p[3] = {x, y, z};
    int64_t *scratch = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int32_t root = tree_new_node(t);
    t->nodes[root].begin = 0;
    t->nodes[root].count = n;
    t->nodes[root].level = 0;
    tree_split(t, p, root, cap, scratch);
    free(scratch);
}

static void tree_free(otree *t)
{
    free(t->nodes);
    free(t->idx);
    memset(t, 0, sizeof(*t));
}

/* ------------------------------------------------------------------------- */
/* The treecode object: source tree, target batches, interaction lists,      */
/* and modified charges formed on demand.                                     */
/* ------------------------------------------------------------------------- */
typedef struct {
    int32_t cluster;
    int32_t kind;   /* 0 = approximation (eq. 11), 1 = direct sum (eq. 9) */
} oitem;

typedef struct {
    /* caller data (not owned) */
    int64_t nt, ns;
    const double *tx, *ty, *tz, *sx, *sy, *sz;
    double theta;
    int32_t n;       /* interpolation degree */
    int32_t comps;   /* values per grid node: 1 (Lagrange), 8 (Hermite, R25) */
    int64_t leaf, batch;
    otree src, tgt;
    int32_t *batch_node;     /* target-tree node id of each batch (leaves, DFS order) */
    int64_t n_batches;
    int64_t *batch_of_pos;   /* batch id of each target tree position */
    int64_t *target_pos;     /* target tree position of each original target index */
    oitem **items;           /* per batch */
    int64_t *n_items, *cap_items;
    double t_setup;
} otc;

static void push_item(otc *tc, int64_t b, int32_t cluster, int32_t kind)
{
    if (tc->n_items[b] == tc->cap_items[b]) {
        tc->cap_items[b] = tc->cap_items[b] ? 2 * tc->cap_items[b] : 16;
        tc->items[b] = (oitem *)realloc(tc->items[b], (size_t)tc->cap_items[b] * sizeof(oitem));
    }
    tc->items[b][tc->n_items[b]].cluster = cluster;
    tc->items[b][tc->n_items[b]].kind = kind;
    tc->n_items[b]++;
}

/* ComputePotential of Alg. 1, recording what it would compute (R3, R4). */
static void compute_potential(otc *tc, int64_t b, const onode *B, int32_t cid)
{
    const onode *C = &tc->src.nodes[cid];
    double dx = B->center[0] - C->center[0];
    double dy = B->center[1] - C->center[1];
    double dz = B->center[2] - C->center[2];
    double R = sqrt(dx * dx + dy * dy + dz * dz);
    int64_t P = (int64_t)tc->comps * (tc->n + 1) * (tc->n + 1) * (tc->n + 1);
    int geometric = (B->radius + C->radius < tc->theta * R);
    int size = (P < C->count);
    if (geometric && size) {
        push_item(tc, b, cid, 0);
    } else if (!geometric) {
        if (C->nchild == 0) {
            push_item(tc, b, cid, 1);
        } else {
            int32_t nk = C->nchild;
            int32_t kids[8];
            memcpy(kids, C->child, sizeof(kids));
            for (int32_t c = 0; c < nk; ++c)
                compute_potential(tc, b, B, kids[c]);
        }
    } else {
        push_item(tc, b, cid, 1);
    }
}

static otc *tc_create(int64_t nt, const double *tx, const double *ty, const double *tz,
                      int64_t ns, const double *sx, const double *sy, const double *sz,
                      double theta, int32_t degree, int64_t leaf, int64_t batch, int32_t comps)
{
    double t0 = wall_seconds();
    otc *tc = (otc *)calloc(1, sizeof(otc));
    tc->nt = nt; tc->ns = ns;
    tc->tx = tx; tc->ty = ty; tc->tz = tz;
    tc->sx = sx; tc->sy = sy; tc->sz = sz;
    tc->theta = theta; tc->n = degree; tc->leaf = leaf; tc->batch = batch;
    tc->comps = comps;

    tree_build(&tc->src, ns, sx, sy, sz, leaf);
    tree_build(&tc->tgt, nt, tx, ty, tz, batch);

    /* batches = leaves of the target tree, in depth-first order */
    int64_t nb = 0;
    for (int64_t i = 0; i < tc->tgt.n_nodes; ++i)
        nb += tc->tgt.nodes[i].nchild == 0;
    tc->n_batches = nb;
    tc->batch_node = (int32_t *)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(int32_t));
    {
        /* depth-first walk with an explicit stack */
        int64_t sp = 0, k = 0;
        int32_t *stack = (int32_t *)malloc((size_t)(tc->tgt.n_nodes + 1) * sizeof(int32_t));
        if (tc->tgt.n_nodes > 0)
            stack[sp++] = 0;
        while (sp > 0) {
            int32_t id = stack[--sp];
            const onode *nd = &tc->tgt.nodes[id];
            if (nd->nchild == 0) {
                tc->batch_node[k++] = id;
            } else {
                for (int32_t c = nd->nchild - 1; c >= 0; --c)
                    stack[sp++] = nd->child[c];
            }
        }
        free(stack);
    }
    tc->batch_of_pos = (int64_t *)malloc((size_t)(nt > 0 ? nt : 1) * sizeof(int64_t));
    tc->target_pos = (int64_t *)malloc((size_t)(nt > 0 ? nt : 1) * sizeof(int64_t));
    for (int64_t b = 0; b < nb; ++b) {
        const onode *B = &tc->tgt.nodes[tc->batch_node[b]];
        for (int64_t a = B->begin; a < B->begin + B->count; ++a)
            tc->batch_of_pos[a] = b;
    }
    for (int64_t a = 0; a < nt; ++a)
        tc->target_pos[tc->tgt.idx[a]] = a;

    tc->items = (oitem **)calloc((size_t)(nb > 0 ? nb : 1), sizeof(oitem *));
    tc->n_items = (int64_t *)calloc((size_t)(nb > 0 ? nb : 1), sizeof(int64_t));
    tc->cap_items = (int64_t *)calloc((size_t)(nb > 0 ? nb : 1), sizeof(int64_t));
    if (ns > 0) {
        int64_t b;
#pragma omp parallel for schedule(dynamic, 1)
        for (b = 0; b < nb; ++b)
            compute_potential(tc, b, &tc->tgt.nodes[tc->batch_node[b]], 0);
    }
    tc->t_setup = wall_seconds() - t0;
    return tc;
}

otc *oracle_tc_create(int64_t nt, const double *tx, const double *ty, const double *tz,
                      int64_t ns, const double *sx, const double *sy, const double *sz,
                      double theta, int32_t degree, int64_t leaf, int64_t batch)
{
    return tc_create(nt, tx, ty, tz, ns, sx, sy, sz, theta, degree, leaf, batch, 1);
}

void oracle_tc_destroy(otc *tc)
{
    if (!tc)
        return;
    for (int64_t b = 0; b < tc->n_batches; ++b)
        free(tc->items[b]);
    free(tc->items);
    free(tc->n_items);
    free(tc->cap_items);
    free(tc->batch_node);
    free(tc->batch_of_pos);
    free(tc->target_pos);
    tree_free(&tc->src);
    tree_free(&tc->tgt);
    free(tc);
}

/* ---- structure export (for structural comparisons in tests) ------------ */
void oracle_tc_sizes(const otc *tc, int64_t *out /* [5] */)
{
    int64_t total = 0;
    for (int64_t b = 0; b < tc->n_batches; ++b)
        total += tc->n_items[b];
    out[0] = tc->src.n_nodes;
    out[1] = tc->n_batches;
    out[2] = total;
    out[3] = tc->tgt.n_nodes;
    out[4] = (int64_t)(tc->t_setup * 1e9);
}

/* node i of the source tree: lo[3], hi[3], begin, count, nchild, child[8], level */
void oracle_tc_source_node(const otc *tc, int64_t i, double *lo, double *hi,
                           int64_t *begin_count, int32_t *nchild_children_level)
{
    const onode *nd = &tc->src.nodes[i];
    for (int l = 0; l < 3; ++l) {
        lo[l] = nd->lo[l];
        hi[l] = nd->hi[l];
    }
    begin_count[0] = nd->begin;
    begin_count[1] = nd->count;
    nchild_children_level[0] = nd->nchild;
    for (int c = 0; c < 8; ++c)
        nchild_children_level[1 + c] = c < nd->nchild ? nd->child[c] : -1;
    nchild_children_level[9] = nd->level;
}

void oracle_tc_source_order(const otc *tc, int64_t *out)
{
    memcpy(out, tc->src.idx, (size_t)tc->ns * sizeof(int64_t));
}

void oracle_tc_target_order(const otc *tc, int64_t *out)
{
    memcpy(out, tc->tgt.idx, (size_t)tc->nt * sizeof(int64_t));
}

/* batch b: lo[3], hi[3], begin/count in target tree order */
void oracle_tc_batch(const otc *tc, int64_t b, double *lo, double *hi, int64_t *begin_count)
{
    const onode *nd = &tc->tgt.nodes[tc->batch_node[b]];
    for (int l = 0; l < 3; ++l) {
        lo[l] = nd->lo[l];
        hi[l] = nd->hi[l];
    }
    begin_count[0] = nd->begin;
    begin_count[1] = nd->count;
}

/* all items, batch-major: batch id, cluster (source node id), kind */
void oracle_tc_items(const otc *tc, int64_t *batch, int32_t *cluster, int32_t *kind)
{
    int64_t k = 0;
    for (int64_t b = 0; b < tc->n_batches; ++b)
        for (int64_t t = 0; t < tc->n_items[b]; ++t) {
            batch[k] = b;
            cluster[k] = tc->items[b][t].cluster;
            kind[k] = tc->items[b][t].kind;
            ++k;
        }
}

/* Chebyshev nodes of source cluster c: out[l*(n+1) + k] = s_{l,k} (R10) */
void oracle_tc_cluster_nodes(const otc *tc, int32_t c, double *out)
{
    const onode *nd = &tc->src.nodes[c];
    double w[64];
    for (int l = 0; l < 3; ++l)
        oracle_chebyshev(tc->n, nd->lo[l], nd->hi[l], out + l * (tc->n + 1), w);
}

/* ------------------------------------------------------------------------- */
/* Modified charges of one cluster, eq. (12):                                  */
/*   qhat[k*m_count + m] = sum_{j in C} L_k1(y_j1) L_k2(y_j2) L_k3(y_j3) q_jm, */
/*   k = (k1*(n+1) + k2)*(n+1) + k3, L from eq. (4) with the rule of eq. (5).  */
/* ------------------------------------------------------------------------- */
void oracle_tc_modified_charges(const otc *tc, int32_t c, const double *q, int32_t m,
                                int64_t q_ld, double *qhat)
{
    const onode *nd = &tc->src.nodes[c];
    int32_t n = tc->n, np = n + 1;
    int64_t P = (int64_t)np * np * np;
    double s[3][64], w[64], L[3][64];
    for (int l = 0; l < 3; ++l)
        oracle_chebyshev(n, nd->lo[l], nd->hi[l], s[l], w);
    memset(qhat, 0, (size_t)(P * m) * sizeof(double));
    const double *p[3] = {tc->sx, tc->sy, tc->sz};
    for (int64_t a = nd->begin; a < nd->begin + nd->count; ++a) {
        int64_t j = tc->src.idx[a];
        for (int l = 0; l < 3; ++l)
            oracle_lagrange(n, s[l], w, p[l][j], L[l]);
        for (int32_t k1 = 0; k1 < np; ++k1)
            for (int32_t k2 = 0; k2 < np; ++k2)
                for (int32_t k3 = 0; k3 < np; ++k3) {
                    double L123 = L[0][k1] * L[1][k2] * L[2][k3];
                    int64_t k = ((int64_t)k1 * np + k2) * np + k3;
                    for (int32_t mm = 0; mm < m; ++mm)
                        qhat[k * m + mm] += L123 * q[(int64_t)mm * q_ld + j];
                }
    }
}

/* ------------------------------------------------------------------------- */
/* Evaluation (Alg. 1): phi at the targets listed in `sample` (original      */
/* indices; all targets when sample == NULL), each through its own batch's   */
/* interaction list:                                                          */
/*   phi = sum_{C approx} sum_k G(x, s_k) qhat_k  (eq. 11)                    */
/*       + sum_{C direct} sum_{j in C, r != 0} G(x, y_j) q_j  (eq. 9).        */
/* phi[mm*phi_ld + s] for charge vector mm and sample s.                      */
/* times[0] = modified-charge seconds, times[1] = evaluation seconds.         */
/* ------------------------------------------------------------------------- */
int oracle_tc_potential(const otc *tc, const double *q, int32_t m, int64_t q_ld,
                        int32_t kernel, double kappa, int64_t n_sample, const int64_t *sample,
                        double *phi, int64_t phi_ld, double *times)
{
    int32_t n = tc->n, np = n + 1;
    int64_t P = (int64_t)np * np * np;
    int64_t n_eval = sample ? n_sample : tc->nt;
    double t0 = wall_seconds();

    /* which batches are touched, then which clusters need modified charges */
    char *batch_used = (char *)calloc((size_t)(tc->n_batches > 0 ? tc->n_batches : 1), 1);
    for (int64_t s = 0; s < n_eval; ++s) {
        int64_t i = sample ? sample[s] : s;
        if (i < 0 || i >= tc->nt) {
            free(batch_used);
            return -1;
        }
        batch_used[tc->batch_of_pos[tc->target_pos[i]]] = 1;
    }
    int64_t nn = tc->src.n_nodes;
    int32_t *need = (int32_t *)calloc((size_t)(nn > 0 ? nn : 1), sizeof(int32_t));
    for (int64_t b = 0; b < tc->n_batches; ++b)
        if (batch_used[b])
            for (int64_t t = 0; t < tc->n_items[b]; ++t)
                if (tc->items[b][t].kind == 0)
                    need[tc->items[b][t].cluster] = 1;
    int64_t n_need = 0;
    for (int64_t c = 0; c < nn; ++c)
        n_need += need[c];
    int32_t *need_list = (int32_t *)malloc((size_t)(n_need > 0 ? n_need : 1) * sizeof(int32_t));
    double **qhat = (double **)calloc((size_t)(nn > 0 ? nn : 1), sizeof(double *));
    {
        int64_t k = 0;
        for (int64_t c = 0; c < nn; ++c)
            if (need[c])
                need_list[k++] = (int32_t)c;
    }
    {
        int64_t u;
#pragma omp parallel for schedule(dynamic, 1)
        for (u = 0; u < n_need; ++u) {
            int32_t c = need_list[u];
            double *buf = (double *)malloc((size_t)(P * m) * sizeof(double));
            oracle_tc_modified_charges(tc, c, q, m, q_ld, buf);
            qhat[c] = buf;
        }
    }
    double t1 = wall_seconds();

    {
        int64_t s;
#pragma omp parallel for schedule(dynamic, 8)
        for (s = 0; s < n_eval; ++s) {
            int64_t i = sample ? sample[s] : s;
            int64_t b = tc->batch_of_pos[tc->target_pos[i]];
            double x = tc->tx[i], y = tc->ty[i], z = tc->tz[i];
            double acc[64];
            double nodes[3][64], w[64];
            for (int32_t mm = 0; mm < m; ++mm)
                acc[mm] = 0.0;
            for (int64_t t = 0; t < tc->n_items[b]; ++t) {
                const oitem *it = &tc->items[b][t];
                const onode *C = &tc->src.nodes[it->cluster];
                if (it->kind == 0) {
                    for (int l = 0; l < 3; ++l)
                        oracle_chebyshev(n, C->lo[l], C->hi[l], nodes[l], w);
                    const double *qh = qhat[it->cluster];
                    for (int32_t k1 = 0; k1 < np; ++k1)
                        for (int32_t k2 = 0; k2 < np; ++k2)
                            for (int32_t k3 = 0; k3 < np; ++k3) {
                                double dx = x - nodes[0][k1];
                                double dy = y - nodes[1][k2];
                                double dz = z - nodes[2][k3];
                                double r = sqrt(dx * dx + dy * dy + dz * dz);
                                double g = kernel_of_distance(r, kernel, kappa);
                                int64_t k = ((int64_t)k1 * np + k2) * np + k3;
                                for (int32_t mm = 0; mm < m; ++mm)
                                    acc[mm] += g * qh[k * m + mm];
                            }
                } else {
                    for (int64_t a = C->begin; a < C->begin + C->count; ++a) {
                        int64_t j = tc->src.idx[a];
                        double dx = x - tc->sx[j];
                        double dy = y - tc->sy[j];
                        double dz = z - tc->sz[j];
                        double r = sqrt(dx * dx + dy * dy + dz * dz);
                        if (r == 0.0)
                            continue;
                        double g = kernel_of_distance(r, kernel, kappa);
                        for (int32_t mm = 0; mm < m; ++mm)
                            acc[mm] += g * q[(int64_t)mm * q_ld + j];
                    }
                }
            }
            for (int32_t mm = 0; mm < m; ++mm)
                phi[(int64_t)mm * phi_ld + s] = acc[mm];
        }
    }
    double t2 = wall_seconds();
    if (times) {
        times[0] = t1 - t0;
        times[1] = t2 - t1;
    }
    for (int64_t c = 0; c < nn; ++c)
        free(qhat[c]);
    free(qhat);
    free(need_list);
    free(need);
    free(batch_used);
    return 0;
}

/* ========================================================================= */
/* Barycentric cluster-particle treecode (CP).                                */
/*                                                                            */
/* Sec. V names the cluster-particle variant as a GPU extension: the same     */
/* barycentric interpolation (eqs. 4-7) applied in the target variable.       */
/* Readings (listed with the others in the design notes):                     */
/*   R16 targets form the cluster tree (capacity leaf = N_L, the interpolated */
/*       side); sources form a tree of capacity batch = N_B whose leaves are  */
/*       the source batches; both trees follow R2 and R5-R8;                  */
/*   R17 for a source batch S and target cluster T the MAC of eq. 13 reads    */
/*       r_S + r_T < theta R and (n+1)^3 < N_T, with the branch order of R4   */
/*       (ComputePotential with the roles of the two trees exchanged);        */
/*   R18 an approximated pair adds to the proxy potentials of T,              */
/*       phihat_T(t_k) += sum_{j in S} G(t_k, y_j) q_j, and every target      */
/*       x in T receives sum_k L_k(x) phihat_T(t_k), L_k the tensor product  */
/*       of eq. 4 over T's grid (eq. 5 rule for a coordinate on a node);      */
/*   R19 a direct pair adds sum_{j in S, r != 0} G(x_i, y_j) q_j to every     */
/*       target of T (R1).                                                    */
/* For a symmetric kernel the CP matrix is the transpose of the BLTC matrix  */
/* with targets and sources exchanged (same trees, same MAC decisions).       */
/* ========================================================================= */
typedef struct {
    int64_t nt, ns;
    const double *tx, *ty, *tz, *sx, *sy, *sz;
    double theta;
    int32_t n;
    int64_t leaf, batch;
    otree tgt;               /* target clusters (interpolated side) */
    otree src;               /* source tree; its leaves are the source batches */
    int32_t *batch_node;     /* source-tree node of each source batch, depth-first order */
    int64_t n_batches;
    oitem **items;           /* per source batch: (target cluster, kind) */
    int64_t *n_items, *cap_items;
    double t_setup;
} ocp;

static void cp_push(ocp *cp, int64_t b, int32_t cluster, int32_t kind)
{
    if (cp->n_items[b] == cp->cap_items[b]) {
        cp->cap_items[b] = cp->cap_items[b] ? 2 * cp->cap_items[b] : 16;
        cp->items[b] = (oitem *)realloc(cp->items[b], (size_t)cp->cap_items[b] * sizeof(oitem));
    }
    cp->items[b][cp->n_items[b]].cluster = cluster;
    cp->items[b][cp->n_items[b]].kind = kind;
    cp->n_items[b]++;
}

/* ComputePotential with the target tree traversed for a source batch (R17). */
static void cp_traverse(ocp *cp, int64_t b, const onode *S, int32_t tid)
{
    const onode *T = &cp->tgt.nodes[tid];
    double dx = S->center[0] - T->center[0];
    double dy = S->center[1] - T->center[1];
    double dz = S->center[2] - T->center[2];
    double R = sqrt(dx * dx + dy * dy + dz * dz);
    int64_t P = (int64_t)(cp->n + 1) * (cp->n + 1) * (cp->n + 1);
    int geometric = (S->radius + T->radius < cp->theta * R);
    int size = (P < T->count);
    if (geometric && size) {
        cp_push(cp, b, tid, 0);
    } else if (!geometric) {
        if (T->nchild == 0) {
            cp_push(cp, b, tid, 1);
        } else {
            int32_t nk = T->nchild;
            int32_t kids[8];
            memcpy(kids, T->child, sizeof(kids));
            for (int32_t c = 0; c < nk; ++c)
                cp_traverse(cp, b, S, kids[c]);
        }
    } else {
        cp_push(cp, b, tid, 1);
    }
}

ocp *oracle_cp_create(int64_t nt, const double *tx, const double *ty, const double *tz,
                      int64_t ns, const double *sx, const double *sy, const double *sz,
                      double theta, int32_t degree, int64_t leaf, int64_t batch)
{
    double t0 = wall_seconds();
    ocp *cp = (ocp *)calloc(1, sizeof(ocp));
    cp->nt = nt; cp->ns = ns;
    cp->tx = tx; cp->ty = ty; cp->tz = tz;
    cp->sx = sx; cp->sy = sy; cp->sz = sz;
    cp->theta = theta; cp->n = degree; cp->leaf = leaf; cp->batch = batch;
    tree_build(&cp->tgt, nt, tx, ty, tz, leaf);
    tree_build(&cp->src, ns, sx, sy, sz, batch);

    int64_t nb = 0;
    for (int64_t i = 0; i < cp->src.n_nodes; ++i)
        nb += cp->src.nodes[i].nchild == 0;
    cp->n_batches = nb;
    cp->batch_node = (int32_t *)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(int32_t));
    {
        int64_t sp = 0, k = 0;
        int32_t *stack = (int32_t *)malloc((size_t)(cp->src.n_nodes + 1) * sizeof(int32_t));
        if (cp->src.n_nodes > 0)
            stack[sp++] = 0;
        while (sp > 0) {
            int32_t id = stack[--sp];
            const onode *nd = &cp->src.nodes[id];
            if (nd->nchild == 0) {
                cp->batch_node[k++] = id;
            } else {
                for (int32_t c = nd->nchild - 1; c >= 0; --c)
                    stack[sp++] = nd->child[c];
            }
        }
        free(stack);
    }
    cp->items = (oitem **)calloc((size_t)(nb > 0 ? nb : 1), sizeof(oitem *));
    cp->n_items = (int64_t *)calloc((size_t)(nb > 0 ? nb : 1), sizeof(int64_t));
    cp->cap_items = (int64_t *)calloc((size_t)(nb > 0 ? nb : 1), sizeof(int64_t));
    if (nt > 0) {
        int64_t b;
#pragma omp parallel for schedule(dynamic, 1)
        for (b = 0; b < nb; ++b)
            cp_traverse(cp, b, &cp->src.nodes[cp->batch_node[b]], 0);
    }
    cp->t_setup = wall_seconds() - t0;
    return cp;
}

void oracle_cp_destroy(ocp *cp)
{
    if (!cp)
        return;
    for (int64_t b = 0; b < cp->n_batches; ++b)
        free(cp->items[b]);
    free(cp->items);
    free(cp->n_items);
    free(cp->cap_items);
    free(cp->batch_node);
    tree_free(&cp->tgt);
    tree_free(&cp->src);
    free(cp);
}

/* sizes: target clusters, source batches, items, source-tree nodes */
void oracle_cp_sizes(const ocp *cp, int64_t *out /* [4] */)
{
    int64_t total = 0;
    for (int64_t b = 0; b < cp->n_batches; ++b)
        total += cp->n_items[b];
    out[0] = cp->tgt.n_nodes;
    out[1] = cp->n_batches;
    out[2] = total;
    out[3] = cp->src.n_nodes;
}

void oracle_cp_target_order(const ocp *cp, int64_t *out)
{
    memcpy(out, cp->tgt.idx, (size_t)cp->nt * sizeof(int64_t));
}

void oracle_cp_source_order(const ocp *cp, int64_t *out)
{
    memcpy(out, cp->src.idx, (size_t)cp->ns * sizeof(int64_t));
}

/* target cluster i: lo[3], hi[3], begin, count (target tree order), nchild, children, level */
void oracle_cp_cluster(const ocp *cp, int64_t i, double *lo, double *hi, int64_t *begin_count,
                       int32_t *nchild_children_level)
{
    const onode *nd = &cp->tgt.nodes[i];
    for (int l = 0; l < 3; ++l) {
        lo[l] = nd->lo[l];
        hi[l] = nd->hi[l];
    }
    begin_count[0] = nd->begin;
    begin_count[1] = nd->count;
    nchild_children_level[0] = nd->nchild;
    for (int c = 0; c < 8; ++c)
        nchild_children_level[1 + c] = c < nd->nchild ? nd->child[c] : -1;
    nchild_children_level[9] = nd->level;
}

/* source batch b: begin, count in source tree order */
void oracle_cp_batch(const ocp *cp, int64_t b, int64_t *begin_count)
{
    const onode *nd = &cp->src.nodes[cp->batch_node[b]];
    begin_count[0] = nd->begin;
    begin_count[1] = nd->count;
}

/* all items, source-batch-major: batch, target cluster, kind */
void oracle_cp_items(const ocp *cp, int64_t *batch, int32_t *cluster, int32_t *kind)
{
    int64_t k = 0;
    for (int64_t b = 0; b < cp->n_batches; ++b)
        for (int64_t t = 0; t < cp->n_items[b]; ++t) {
            batch[k] = b;
            cluster[k] = cp->items[b][t].cluster;
            kind[k] = cp->items[b][t].kind;
            ++k;
        }
}

/* Proxy potentials of target cluster c (R18): out[k] = sum over the source   */
/* batches S approximated with c, sum_{j in S, r != 0} G(t_k, y_j) q_j,        */
/* k = (k1*(n+1) + k2)*(n+1) + k3, t_k from R10 on c's box.                   */
void oracle_cp_proxy_potentials(const ocp *cp, int32_t c, const double *q, int32_t kernel,
                                double kappa, double *out)
{
    const onode *T = &cp->tgt.nodes[c];
    int32_t n = cp->n, np = n + 1;
    int64_t P = (int64_t)np * np * np;
    double t[3][64], w[64];
    for (int l = 0; l < 3; ++l)
        oracle_chebyshev(n, T->lo[l], T->hi[l], t[l], w);
    memset(out, 0, (size_t)P * sizeof(double));
    for (int64_t b = 0; b < cp->n_batches; ++b)
        for (int64_t it = 0; it < cp->n_items[b]; ++it) {
            if (cp->items[b][it].cluster != c || cp->items[b][it].kind != 0)
                continue;
            const onode *S = &cp->src.nodes[cp->batch_node[b]];
            for (int64_t a = S->begin; a < S->begin + S->count; ++a) {
                int64_t j = cp->src.idx[a];
                for (int32_t k1 = 0; k1 < np; ++k1)
                    for (int32_t k2 = 0; k2 < np; ++k2)
                        for (int32_t k3 = 0; k3 < np; ++k3) {
                            double dx = t[0][k1] - cp->sx[j];
                            double dy = t[1][k2] - cp->sy[j];
                            double dz = t[2][k3] - cp->sz[j];
                            double r = sqrt(dx * dx + dy * dy + dz * dz);
                            if (r == 0.0)
                                continue;
                            out[((int64_t)k1 * np + k2) * np + k3] +=
                                kernel_of_distance(r, kernel, kappa) * q[j];
                        }
            }
        }
}

/* Evaluation: phi[s] at target sample[s] (all targets when sample == NULL):  */
/* for every target cluster T on the path from the root to the target's leaf, */
/* the direct sums of T's direct source batches (R19) and the interpolant of  */
/* T's proxy potentials (R18).  times[0] = proxy potentials, times[1] = rest. */
int oracle_cp_potential(const ocp *cp, const double *q, int32_t kernel, double kappa,
                        int64_t n_sample, const int64_t *sample, double *phi, double *times)
{
    int32_t n = cp->n, np = n + 1;
    int64_t P = (int64_t)np * np * np;
    int64_t n_eval = sample ? n_sample : cp->nt;
    int64_t nn = cp->tgt.n_nodes;
    double t0 = wall_seconds();

    /* target tree position of each target */
    int64_t *pos = (int64_t *)malloc((size_t)(cp->nt > 0 ? cp->nt : 1) * sizeof(int64_t));
    for (int64_t a = 0; a < cp->nt; ++a)
        pos[cp->tgt.idx[a]] = a;
    /* per target cluster: approximated and direct source batches */
    int64_t *n_far = (int64_t *)calloc((size_t)(nn > 0 ? nn : 1), sizeof(int64_t));
    int64_t *n_dir = (int64_t *)calloc((size_t)(nn > 0 ? nn : 1), sizeof(int64_t));
    for (int64_t b = 0; b < cp->n_batches; ++b)
        for (int64_t it = 0; it < cp->n_items[b]; ++it)
            (cp->items[b][it].kind == 0 ? n_far : n_dir)[cp->items[b][it].cluster]++;
    int64_t **dir = (int64_t **)calloc((size_t)(nn > 0 ? nn : 1), sizeof(int64_t *));
    int64_t *fill = (int64_t *)calloc((size_t)(nn > 0 ? nn : 1), sizeof(int64_t));
    for (int64_t c = 0; c < nn; ++c)
        dir[c] = (int64_t *)malloc((size_t)(n_dir[c] > 0 ? n_dir[c] : 1) * sizeof(int64_t));
    for (int64_t b = 0; b < cp->n_batches; ++b)
        for (int64_t it = 0; it < cp->n_items[b]; ++it)
            if (cp->items[b][it].kind == 1) {
                int32_t c = cp->items[b][it].cluster;
                dir[c][fill[c]++] = b;
            }
    /* proxy potentials of the clusters on the sampled targets' paths */
    char *need = (char *)calloc((size_t)(nn > 0 ? nn : 1), 1);
    for (int64_t s = 0; s < n_eval; ++s) {
        int64_t i = sample ? sample[s] : s;
        if (i < 0 || i >= cp->nt) {
            free(need);
            free(pos);
            free(n_far);
            free(n_dir);
            for (int64_t c = 0; c < nn; ++c)
                free(dir[c]);
            free(dir);
            free(fill);
            return -1;
        }
        int64_t a = pos[i];
        for (int32_t c = 0; c >= 0;) {
            if (n_far[c] > 0)
                need[c] = 1;
            int32_t next = -1;
            const onode *nd = &cp->tgt.nodes[c];
            for (int32_t k = 0; k < nd->nchild; ++k) {
                const onode *ch = &cp->tgt.nodes[nd->child[k]];
                if (a >= ch->begin && a < ch->begin + ch->count)
                    next = nd->child[k];
            }
            c = next;
        }
    }
    double **phat = (double **)calloc((size_t)(nn > 0 ? nn : 1), sizeof(double *));
    {
        int64_t c;
#pragma omp parallel for schedule(dynamic, 1)
        for (c = 0; c < nn; ++c)
            if (need[c]) {
                double *buf = (double *)malloc((size_t)P * sizeof(double));
                oracle_cp_proxy_potentials(cp, (int32_t)c, q, kernel, kappa, buf);
                phat[c] = buf;
            }
    }
    double t1 = wall_seconds();
    {
        int64_t s;
#pragma omp parallel for schedule(dynamic, 8)
        for (s = 0; s < n_eval; ++s) {
            int64_t i = sample ? sample[s] : s;
            int64_t a = pos[i];
            double x[3] = {cp->tx[i], cp->ty[i], cp->tz[i]};
            double acc = 0.0;
            double nodes[64], w[64], L[3][64];
            for (int32_t c = 0; c >= 0;) {
                const onode *T = &cp->tgt.nodes[c];
                for (int64_t u = 0; u < n_dir[c]; ++u) {
                    const onode *S = &cp->src.nodes[cp->batch_node[dir[c][u]]];
                    for (int64_t e = S->begin; e < S->begin + S->count; ++e) {
                        int64_t j = cp->src.idx[e];
                        double dx = x[0] - cp->sx[j];
                        double dy = x[1] - cp->sy[j];
                        double dz = x[2] - cp->sz[j];
                        double r = sqrt(dx * dx + dy * dy + dz * dz);
                        if (r == 0.0)
                            continue;
                        acc += kernel_of_distance(r, kernel, kappa) * q[j];
                    }
                }
                if (phat[c]) {
                    for (int l = 0; l < 3; ++l) {
                        oracle_chebyshev(n, T->lo[l], T->hi[l], nodes, w);
                        oracle_lagrange(n, nodes, w, x[l], L[l]);
                    }
                    for (int32_t k1 = 0; k1 < np; ++k1)
                        for (int32_t k2 = 0; k2 < np; ++k2)
                            for (int32_t k3 = 0; k3 < np; ++k3)
                                acc += L[0][k1] * L[1][k2] * L[2][k3] *
                                       phat[c][((int64_t)k1 * np + k2) * np + k3];
                }
                int32_t next = -1;
                for (int32_t k = 0; k < T->nchild; ++k) {
                    const onode *ch = &cp->tgt.nodes[T->child[k]];
                    if (a >= ch->begin && a < ch->begin + ch->count)
                        next = T->child[k];
                }
                c = next;
            }
            phi[s] = acc;
        }
    }
    double t2 = wall_seconds();
    if (times) {
        times[0] = t1 - t0;
        times[1] = t2 - t1;
    }
    for (int64_t c = 0; c < nn; ++c) {
        free(phat[c]);
        free(dir[c]);
    }
    free(phat);
    free(dir);
    free(fill);
    free(need);
    free(pos);
    free(n_far);
    free(n_dir);
    return 0;
}

/* ========================================================================= */
/* Barycentric cluster-cluster treecode (CC), named with the CP variant in    */
/* the paper's outlook (Sec. V).  Both sides are interpolated.                */
/* Readings (listed with the others in the design notes):                     */
/*   R20 sources form a tree of capacity leaf (N_L), targets a tree of         */
/*       capacity batch (N_B); both follow R2 and R5-R8;                       */
/*   R21 a dual walk starts at the pair of roots.  For a pair (T, S) with     */
/*       r_T + r_S < theta R (R3) the interaction is approximated on every    */
/*       side larger than (n+1)^3: CC when P < N_T and P < N_S (proxy         */
/*       potentials of T from the modified charges of S), PC when only        */
/*       P < N_S (targets of T from S's modified charges, eq. 11), CP when    */
/*       only P < N_T (proxy potentials of T from S's particles), a direct    */
/*       sum when neither;                                                    */
/*   R22 otherwise two leaves interact directly; else a leaf is never split,  */
/*       of two non-leaves the one with the larger radius is split, and equal */
/*       radii split both (child pairs in target-major order);                */
/*   R23 every target receives its direct and PC terms from all clusters on   */
/*       its root-to-leaf path and the interpolant (R18) of the proxy         */
/*       potentials of each of them.                                          */
/* Exchanging targets and sources (and N_L with N_B) mirrors every decision,  */
/* so for a symmetric kernel the matrix is the transpose of the exchanged     */
/* problem's.                                                                 */
/* ========================================================================= */
typedef struct {
    int32_t t, s;     /* target node, source node */
    int32_t kind;     /* 0 CC, 1 PC, 2 CP, 3 direct */
} opair;

typedef struct {
    int64_t nt, ns;
    const double *tx, *ty, *tz, *sx, *sy, *sz;
    double theta;
    int32_t n;
    int64_t leaf, batch;
    otree tgt, src;
    opair *pairs;
    int64_t n_pairs, cap_pairs;
    double t_setup;
} occ;

static void cc_push(occ *cc, int32_t t, int32_t s, int32_t kind)
{
    if (cc->n_pairs == cc->cap_pairs) {
        cc->cap_pairs = cc->cap_pairs ? 2 * cc->cap_pairs : 64;
        cc->pairs = (opair *)realloc(cc->pairs, (size_t)cc->cap_pairs * sizeof(opair));
    }
    cc->pairs[cc->n_pairs].t = t;
    cc->pairs[cc->n_pairs].s = s;
    cc->pairs[cc->n_pairs].kind = kind;
    cc->n_pairs++;
}

/* the dual walk (R21, R22) */
static void cc_walk(occ *cc, int32_t t, int32_t s)
{
    const onode *T = &cc->tgt.nodes[t];
    const onode *S = &cc->src.nodes[s];
    double dx = T->center[0] - S->center[0];
    double dy = T->center[1] - S->center[1];
    double dz = T->center[2] - S->center[2];
    double R = sqrt(dx * dx + dy * dy + dz * dz);
    int64_t P = (int64_t)(cc->n + 1) * (cc->n + 1) * (cc->n + 1);
    if (T->radius + S->radius < cc->theta * R) {
        int big_t = P < T->count, big_s = P < S->count;
        cc_push(cc, t, s, big_t && big_s ? 0 : (big_s ? 1 : (big_t ? 2 : 3)));
        return;
    }
    int leaf_t = T->nchild == 0, leaf_s = S->nchild == 0;
    if (leaf_t && leaf_s) {
        cc_push(cc, t, s, 3);
        return;
    }
    int split_t, split_s;
    if (leaf_s) {
        split_t = 1; split_s = 0;
    } else if (leaf_t) {
        split_t = 0; split_s = 1;
    } else if (T->radius > S->radius) {
        split_t = 1; split_s = 0;
    } else if (S->radius > T->radius) {
        split_t = 0; split_s = 1;
    } else {
        split_t = 1; split_s = 1;
    }
    int32_t kt[8], ks[8], nkt = 1, nks = 1;
    kt[0] = t;
    ks[0] = s;
    if (split_t) {
        nkt = T->nchild;
        memcpy(kt, T->child, sizeof(kt));
    }
    if (split_s) {
        nks = S->nchild;
        memcpy(ks, S->child, sizeof(ks));
    }
    for (int32_t a = 0; a < nkt; ++a)
        for (int32_t b = 0; b < nks; ++b)
            cc_walk(cc, kt[a], ks[b]);
}

occ *oracle_cc_create(int64_t nt, const double *tx, const double *ty, const double *tz,
                      int64_t ns, const double *sx, const double *sy, const double *sz,
                      double theta, int32_t degree, int64_t leaf, int64_t batch)
{
    double t0 = wall_seconds();
    occ *cc = (occ *)calloc(1, sizeof(occ));
    cc->nt = nt; cc->ns = ns;
    cc->tx = tx; cc->ty = ty; cc->tz = tz;
    cc->sx = sx; cc->sy = sy; cc->sz = sz;
    cc->theta = theta; cc->n = degree; cc->leaf = leaf; cc->batch = batch;
    tree_build(&cc->tgt, nt, tx, ty, tz, batch);
    tree_build(&cc->src, ns, sx, sy, sz, leaf);
    if (nt > 0 && ns > 0)
        cc_walk(cc, 0, 0);
    cc->t_setup = wall_seconds() - t0;
    return cc;
}

void oracle_cc_destroy(occ *cc)
{
    if (!cc)
        return;
    free(cc->pairs);
    tree_free(&cc->tgt);
    tree_free(&cc->src);
    free(cc);
}

/* sizes: target nodes, source nodes, pairs */
void oracle_cc_sizes(const occ *cc, int64_t *out /* [3] */)
{
    out[0] = cc->tgt.n_nodes;
    out[1] = cc->src.n_nodes;
    out[2] = cc->n_pairs;
}

void oracle_cc_orders(const occ *cc, int64_t *target_order, int64_t *source_order)
{
    memcpy(target_order, cc->tgt.idx, (size_t)cc->nt * sizeof(int64_t));
    memcpy(source_order, cc->src.idx, (size_t)cc->ns * sizeof(int64_t));
}

/* node i of the target (side 0) or source (side 1) tree: lo, hi, begin, count */
void oracle_cc_node(const occ *cc, int32_t side, int64_t i, double *lo, double *hi,
                    int64_t *begin_count)
{
    const onode *nd = side == 0 ? &cc->tgt.nodes[i] : &cc->src.nodes[i];
    for (int l = 0; l < 3; ++l) {
        lo[l] = nd->lo[l];
        hi[l] = nd->hi[l];
    }
    begin_count[0] = nd->begin;
    begin_count[1] = nd->count;
}

void oracle_cc_pairs(const occ *cc, int32_t *t, int32_t *s, int32_t *kind)
{
    for (int64_t k = 0; k < cc->n_pairs; ++k) {
        t[k] = cc->pairs[k].t;
        s[k] = cc->pairs[k].s;
        kind[k] = cc->pairs[k].kind;
    }
}

/* modified charges of source node c by eq. 12 (as oracle_tc_modified_charges) */
static void cc_modified_charges(const occ *cc, int32_t c, const double *q, double *qhat)
{
    const onode *nd = &cc->src.nodes[c];
    int32_t n = cc->n, np = n + 1;
    int64_t P = (int64_t)np * np * np;
    double s[3][64], w[64], L[3][64];
    for (int l = 0; l < 3; ++l)
        oracle_chebyshev(n, nd->lo[l], nd->hi[l], s[l], w);
    memset(qhat, 0, (size_t)P * sizeof(double));
    const double *p[3] = {cc->sx, cc->sy, cc->sz};
    for (int64_t a = nd->begin; a < nd->begin + nd->count; ++a) {
        int64_t j = cc->src.idx[a];
        for (int l = 0; l < 3; ++l)
            oracle_lagrange(n, s[l], w, p[l][j], L[l]);
        for (int32_t k1 = 0; k1 < np; ++k1)
            for (int32_t k2 = 0; k2 < np; ++k2)
                for (int32_t k3 = 0; k3 < np; ++k3)
                    qhat[((int64_t)k1 * np + k2) * np + k3] +=
                        L[0][k1] * L[1][k2] * L[2][k3] * q[j];
    }
}

/* sum over the grid of source node s of G(x, s_m) qhat_m (eq. 11) */
static double cc_from_grid(const occ *cc, int32_t s, const double *qhat, const double x[3],
                           int32_t kernel, double kappa)
{
    const onode *S = &cc->src.nodes[s];
    int32_t n = cc->n, np = n + 1;
    double g[3][64], w[64];
    for (int l = 0; l < 3; ++l)
        oracle_chebyshev(n, S->lo[l], S->hi[l], g[l], w);
    double acc = 0.0;
    for (int32_t k1 = 0; k1 < np; ++k1)
        for (int32_t k2 = 0; k2 < np; ++k2)
            for (int32_t k3 = 0; k3 < np; ++k3) {
                double dx = x[0] - g[0][k1], dy = x[1] - g[1][k2], dz = x[2] - g[2][k3];
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                acc += kernel_of_distance(r, kernel, kappa) * qhat[((int64_t)k1 * np + k2) * np + k3];
            }
    return acc;
}

/* sum over the particles of source node s of G(x, y_j) q_j, r != 0 (R1) */
static double cc_from_particles(const occ *cc, int32_t s, const double *q, const double x[3],
                                int32_t kernel, double kappa)
{
    const onode *S = &cc->src.nodes[s];
    double acc = 0.0;
    for (int64_t a = S->begin; a < S->begin + S->count; ++a) {
        int64_t j = cc->src.idx[a];
        double dx = x[0] - cc->sx[j], dy = x[1] - cc->sy[j], dz = x[2] - cc->sz[j];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r == 0.0)
            continue;
        acc += kernel_of_distance(r, kernel, kappa) * q[j];
    }
    return acc;
}

/* Proxy potentials of target node c (R21): CC pairs through the source      */
/* cluster's modified charges, CP pairs through its particles.                */
void oracle_cc_proxy_potentials(const occ *cc, int32_t c, const double *q, int32_t kernel,
                                double kappa, double *out)
{
    const onode *T = &cc->tgt.nodes[c];
    int32_t n = cc->n, np = n + 1;
    int64_t P = (int64_t)np * np * np;
    double t[3][64], w[64];
    for (int l = 0; l < 3; ++l)
        oracle_chebyshev(n, T->lo[l], T->hi[l], t[l], w);
    memset(out, 0, (size_t)P * sizeof(double));
    double *qhat = (double *)malloc((size_t)P * sizeof(double));
    for (int64_t k = 0; k < cc->n_pairs; ++k) {
        const opair *pr = &cc->pairs[k];
        if (pr->t != c || (pr->kind != 0 && pr->kind != 2))
            continue;
        if (pr->kind == 0)
            cc_modified_charges(cc, pr->s, q, qhat);
        for (int32_t k1 = 0; k1 < np; ++k1)
            for (int32_t k2 = 0; k2 < np; ++k2)
                for (int32_t k3 = 0; k3 < np; ++k3) {
                    double x[3] = {t[0][k1], t[1][k2], t[2][k3]};
                    out[((int64_t)k1 * np + k2) * np + k3] +=
                        pr->kind == 0 ? cc_from_grid(cc, pr->s, qhat, x, kernel, kappa)
                                      : cc_from_particles(cc, pr->s, q, x, kernel, kappa);
                }
    }
    free(qhat);
}

/* Evaluation (R23): phi[s] at target sample[s] (all targets when NULL). */
int oracle_cc_potential(const occ *cc, const double *q, int32_t kernel, double kappa,
                        int64_t n_sample, const int64_t *sample, double *phi, double *times)
{
    int32_t n = cc->n, np = n + 1;
    int64_t P = (int64_t)np * np * np;
    int64_t n_eval = sample ? n_sample : cc->nt;
    int64_t nn = cc->tgt.n_nodes, ms = cc->src.n_nodes;
    double t0 = wall_seconds();
    for (int64_t s = 0; s < n_eval; ++s) {
        int64_t i = sample ? sample[s] : s;
        if (i < 0 || i >= cc->nt)
            return -1;
    }
    int64_t *pos = (int64_t *)malloc((size_t)(cc->nt > 0 ? cc->nt : 1) * sizeof(int64_t));
    for (int64_t a = 0; a < cc->nt; ++a)
        pos[cc->tgt.idx[a]] = a;
    /* pairs grouped by target node */
    int64_t *off = (int64_t *)calloc((size_t)(nn + 1), sizeof(int64_t));
    for (int64_t k = 0; k < cc->n_pairs; ++k)
        off[cc->pairs[k].t + 1]++;
    for (int64_t c = 0; c < nn; ++c)
        off[c + 1] += off[c];
    int64_t *by_t = (int64_t *)malloc((size_t)(cc->n_pairs > 0 ? cc->n_pairs : 1) * sizeof(int64_t));
    {
        int64_t *fill = (int64_t *)malloc((size_t)(nn > 0 ? nn : 1) * sizeof(int64_t));
        for (int64_t c = 0; c < nn; ++c)
            fill[c] = off[c];
        for (int64_t k = 0; k < cc->n_pairs; ++k)
            by_t[fill[cc->pairs[k].t]++] = k;
        free(fill);
    }
    /* modified charges of the sources in CC or PC pairs */
    char *need_s = (char *)calloc((size_t)(ms > 0 ? ms : 1), 1);
    char *need_t = (char *)calloc((size_t)(nn > 0 ? nn : 1), 1);
    for (int64_t k = 0; k < cc->n_pairs; ++k) {
        if (cc->pairs[k].kind <= 1)
            need_s[cc->pairs[k].s] = 1;
        if (cc->pairs[k].kind == 0 || cc->pairs[k].kind == 2)
            need_t[cc->pairs[k].t] = 1;
    }
    double **qhat = (double **)calloc((size_t)(ms > 0 ? ms : 1), sizeof(double *));
    double **phat = (double **)calloc((size_t)(nn > 0 ? nn : 1), sizeof(double *));
    {
        int64_t c;
#pragma omp parallel for schedule(dynamic, 1)
        for (c = 0; c < ms; ++c)
            if (need_s[c]) {
                qhat[c] = (double *)malloc((size_t)P * sizeof(double));
                cc_modified_charges(cc, (int32_t)c, q, qhat[c]);
            }
#pragma omp parallel for schedule(dynamic, 1)
        for (c = 0; c < nn; ++c)
            if (need_t[c]) {
                phat[c] = (double *)malloc((size_t)P * sizeof(double));
                oracle_cc_proxy_potentials(cc, (int32_t)c, q, kernel, kappa, phat[c]);
            }
    }
    double t1 = wall_seconds();
    {
        int64_t s;
#pragma omp parallel for schedule(dynamic, 8)
        for (s = 0; s < n_eval; ++s) {
            int64_t i = sample ? sample[s] : s;
            int64_t a = pos[i];
            double x[3] = {cc->tx[i], cc->ty[i], cc->tz[i]};
            double acc = 0.0;
            double nodes[64], w[64], L[3][64];
            for (int32_t c = 0; c >= 0;) {
                const onode *T = &cc->tgt.nodes[c];
                for (int64_t u = off[c]; u < off[c + 1]; ++u) {
                    const opair *pr = &cc->pairs[by_t[u]];
                    if (pr->kind == 1)
                        acc += cc_from_grid(cc, pr->s, qhat[pr->s], x, kernel, kappa);
                    else if (pr->kind == 3)
                        acc += cc_from_particles(cc, pr->s, q, x, kernel, kappa);
                }
                if (phat[c]) {
                    for (int l = 0; l < 3; ++l) {
                        oracle_chebyshev(n, T->lo[l], T->hi[l], nodes, w);
                        oracle_lagrange(n, nodes, w, x[l], L[l]);
                    }
                    for (int32_t k1 = 0; k1 < np; ++k1)
                        for (int32_t k2 = 0; k2 < np; ++k2)
                            for (int32_t k3 = 0; k3 < np; ++k3)
                                acc += L[0][k1] * L[1][k2] * L[2][k3] *
                                       phat[c][((int64_t)k1 * np + k2) * np + k3];
                }
                int32_t next = -1;
                for (int32_t k = 0; k < T->nchild; ++k) {
                    const onode *ch = &cc->tgt.nodes[T->child[k]];
                    if (a >= ch->begin && a < ch->begin + ch->count)
                        next = T->child[k];
                }
                c = next;
            }
            phi[s] = acc;
        }
    }
    double t2 = wall_seconds();
    if (times) {
        times[0] = t1 - t0;
        times[1] = t2 - t1;
    }
    for (int64_t c = 0; c < ms; ++c)
        free(qhat[c]);
    for (int64_t c = 0; c < nn; ++c)
        free(phat[c]);
    free(qhat);
    free(phat);
    free(need_s);
    free(need_t);
    free(by_t);
    free(off);
    free(pos);
    return 0;
}

/* ========================================================================= */
/* Barycentric Hermite treecode (the paper's outlook, Sec. V: like the BLTC   */
/* but with low-order partial derivatives of the kernel).                     */
/* Readings (listed with the others in the design notes):                     */
/*   R25 the interpolant in y is the tensor-product Hermite interpolant on    */
/*       the same Chebyshev grid (eqs. 6-7): per dimension                    */
/*         f(y) ~ sum_k f(s_k) A_k(y) + f'(s_k) B_k(y),                       */
/*         A_k = (1 - 2 c_k (y - s_k)) L_k(y)^2,  B_k = (y - s_k) L_k(y)^2,    */
/*       L_k from eq. 4 (eq. 5 rule at a node), c_k = L_k'(s_k) =             */
/*       sum_{j != k} 1 / (s_k - s_j); exact for degree <= 2n + 1;            */
/*   R26 a cluster carries 8 (n+1)^3 modified charges                         */
/*         qhat^a_k = sum_j q_j prod_l (a_l ? B_kl(y_jl) : A_kl(y_jl)),       */
/*       a in {0,1}^3, and the approximation is                               */
/*         phi(x) ~ sum_k sum_a d^a_y G(x, s_k) qhat^a_k;                     */
/*   R27 the size part of the MAC compares 8 (n+1)^3 with N_C.                */
/* For a radial kernel G(r), with d = x - y, g1 = G'/r, g2 = g1'/r,           */
/* g3 = g2'/r:  d_yi G = -d_i g1,  d_yi d_yj G = d_i d_j g2 (i != j),          */
/* d_y1 d_y2 d_y3 G = -d_1 d_2 d_3 g3.                                        */
/* ========================================================================= */

/* G, g1, g2, g3 of the kernels at distance r > 0 */
void oracle_kernel_derivatives(double r, int32_t kernel, double kappa, double *g)
{
    if (kernel == ORACLE_YUKAWA) {
        double e = exp(-kappa * r), kr = kappa * r;
        g[0] = e / r;
        g[1] = -e * (1.0 + kr) / (r * r * r);
        g[2] = e * (3.0 + 3.0 * kr + kr * kr) / pow(r, 5.0);
        g[3] = -e * (15.0 + 15.0 * kr + 6.0 * kr * kr + kr * kr * kr) / pow(r, 7.0);
    } else if (kernel == ORACLE_REGULARIZED) {
        double u = r * r + kappa * kappa;
        g[0] = 1.0 / sqrt(u);
        g[1] = -pow(u, -1.5);
        g[2] = 3.0 * pow(u, -2.5);
        g[3] = -15.0 * pow(u, -3.5);
    } else {
        g[0] = 1.0 / r;
        g[1] = -1.0 / (r * r * r);
        g[2] = 3.0 / pow(r, 5.0);
        g[3] = -15.0 / pow(r, 7.0);
    }
}

/* 1-D Hermite basis A_k(x), B_k(x), k = 0..n, on nodes s (R25); at a node    */
/* (R9, lowest k) A is one-hot and B zero, also when the nodes coincide.      */
void oracle_hermite_basis(int32_t n, const double *s, const double *w, double x, double *A,
                          double *B)
{
    double L[64];
    int32_t hit = -1;
    for (int32_t k = n; k >= 0; --k)
        if (fabs(x - s[k]) < DBL_MIN)
            hit = k;
    if (hit >= 0) {
        for (int32_t k = 0; k <= n; ++k) {
            A[k] = k == hit ? 1.0 : 0.0;
            B[k] = 0.0;
        }
        return;
    }
    oracle_lagrange(n, s, w, x, L);
    for (int32_t k = 0; k <= n; ++k) {
        double c = 0.0;
        for (int32_t j = 0; j <= n; ++j)
            if (j != k)
                c += 1.0 / (s[k] - s[j]);
        double d = x - s[k];
        A[k] = (1.0 - 2.0 * c * d) * L[k] * L[k];
        B[k] = d * L[k] * L[k];
    }
}

otc *oracle_tc_create_hermite(int64_t nt, const double *tx, const double *ty, const double *tz,
                              int64_t ns, const double *sx, const double *sy, const double *sz,
                              double theta, int32_t degree, int64_t leaf, int64_t batch)
{
    return tc_create(nt, tx, ty, tz, ns, sx, sy, sz, theta, degree, leaf, batch, 8);
}

/* Hermite modified charges of cluster c (R26): out[a * P + k], a = 4 a1 + 2 a2 + a3,
 * k = (k1*(n+1) + k2)*(n+1) + k3. */
void oracle_tc_hermite_charges(const otc *tc, int32_t c, const double *q, double *out)
{
    const onode *nd = &tc->src.nodes[c];
    int32_t n = tc->n, np = n + 1;
    int64_t P = (int64_t)np * np * np;
    double s[3][64], w[64], A[3][64], B[3][64];
    for (int l = 0; l < 3; ++l)
        oracle_chebyshev(n, nd->lo[l], nd->hi[l], s[l], w);
    memset(out, 0, (size_t)(8 * P) * sizeof(double));
    const double *p[3] = {tc->sx, tc->sy, tc->sz};
    for (int64_t e = nd->begin; e < nd->begin + nd->count; ++e) {
        int64_t j = tc->src.idx[e];
        for (int l = 0; l < 3; ++l)
            oracle_hermite_basis(n, s[l], w, p[l][j], A[l], B[l]);
        for (int a = 0; a < 8; ++a)
            for (int32_t k1 = 0; k1 < np; ++k1)
                for (int32_t k2 = 0; k2 < np; ++k2)
                    for (int32_t k3 = 0; k3 < np; ++k3) {
                        double h = ((a & 4) ? B[0][k1] : A[0][k1]) * ((a & 2) ? B[1][k2] : A[1][k2]) *
                                   ((a & 1) ? B[2][k3] : A[2][k3]);
                        out[a * P + ((int64_t)k1 * np + k2) * np + k3] += h * q[j];
                    }
    }
}

/* Evaluation with the Hermite approximation for the approximated clusters  */
/* (R26) and the direct sum (eq. 9) for the others; phi[s] at sample[s].     */
int oracle_tc_hermite_potential(const otc *tc, const double *q, int32_t kernel, double kappa,
                                int64_t n_sample, const int64_t *sample, double *phi,
                                double *times)
{
    int32_t n = tc->n, np = n + 1;
    int64_t P = (int64_t)np * np * np;
    int64_t n_eval = sample ? n_sample : tc->nt;
    int64_t nn = tc->src.n_nodes;
    double t0 = wall_seconds();
    for (int64_t s = 0; s < n_eval; ++s) {
        int64_t i = sample ? sample[s] : s;
        if (i < 0 || i >= tc->nt)
            return -1;
    }
    char *need = (char *)calloc((size_t)(nn > 0 ? nn : 1), 1);
    for (int64_t s = 0; s < n_eval; ++s) {
        int64_t b = tc->batch_of_pos[tc->target_pos[sample ? sample[s] : s]];
        for (int64_t t = 0; t < tc->n_items[b]; ++t)
            if (tc->items[b][t].kind == 0)
                need[tc->items[b][t].cluster] = 1;
    }
    double **qh = (double **)calloc((size_t)(nn > 0 ? nn : 1), sizeof(double *));
    {
        int64_t c;
#pragma omp parallel for schedule(dynamic, 1)
        for (c = 0; c < nn; ++c)
            if (need[c]) {
                qh[c] = (double *)malloc((size_t)(8 * P) * sizeof(double));
                oracle_tc_hermite_charges(tc, (int32_t)c, q, qh[c]);
            }
    }
    double t1 = wall_seconds();
    {
        int64_t s;
#pragma omp parallel for schedule(dynamic, 8)
        for (s = 0; s < n_eval; ++s) {
            int64_t i = sample ? sample[s] : s;
            int64_t b = tc->batch_of_pos[tc->target_pos[i]];
            double x = tc->tx[i], y = tc->ty[i], z = tc->tz[i];
            double acc = 0.0, nodes[3][64], w[64], g[4];
            for (int64_t t = 0; t < tc->n_items[b]; ++t) {
                const oitem *it = &tc->items[b][t];
                const onode *C = &tc->src.nodes[it->cluster];
                if (it->kind == 0) {
                    for (int l = 0; l < 3; ++l)
                        oracle_chebyshev(n, C->lo[l], C->hi[l], nodes[l], w);
                    const double *Q = qh[it->cluster];
                    for (int32_t k1 = 0; k1 < np; ++k1)
                        for (int32_t k2 = 0; k2 < np; ++k2)
                            for (int32_t k3 = 0; k3 < np; ++k3) {
                                double d1 = x - nodes[0][k1], d2 = y - nodes[1][k2],
                                       d3 = z - nodes[2][k3];
                                double r = sqrt(d1 * d1 + d2 * d2 + d3 * d3);
                                oracle_kernel_derivatives(r, kernel, kappa, g);
                                int64_t k = ((int64_t)k1 * np + k2) * np + k3;
                                /* d^a_y G for a = (a1, a2, a3), index 4 a1 + 2 a2 + a3 */
                                acc += g[0] * Q[0 * P + k];
                                acc += -d3 * g[1] * Q[1 * P + k];
                                acc += -d2 * g[1] * Q[2 * P + k];
                                acc += d2 * d3 * g[2] * Q[3 * P + k];
                                acc += -d1 * g[1] * Q[4 * P + k];
                                acc += d1 * d3 * g[2] * Q[5 * P + k];
                                acc += d1 * d2 * g[2] * Q[6 * P + k];
                                acc += -d1 * d2 * d3 * g[3] * Q[7 * P + k];
                            }
                } else {
                    for (int64_t e = C->begin; e < C->begin + C->count; ++e) {
                        int64_t j = tc->src.idx[e];
                        double d1 = x - tc->sx[j], d2 = y - tc->sy[j], d3 = z - tc->sz[j];
                        double r = sqrt(d1 * d1 + d2 * d2 + d3 * d3);
                        if (r == 0.0)
                            continue;
                        acc += kernel_of_distance(r, kernel, kappa) * q[j];
                    }
                }
            }
            phi[s] = acc;
        }
    }
    double t2 = wall_seconds();
    if (times) {
        times[0] = t1 - t0;
        times[1] = t2 - t1;
    }
    for (int64_t c = 0; c < nn; ++c)
        free(qh[c]);
    free(qh);
    free(need);
    return 0;
}
