/*
 * CPU oracle for kNN-graph construction by repeated two-means bisection.
 *
 * Method: Zhao, Yang, Deng, "Scalable Nearest Neighbor Search based on kNN
 * Graph" (arXiv 1701.08475), Sec. 3.1 and Algorithm 1 (kNN graph construction).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, FP64 reference
 * that the tests, the GPU smoke check and the benchmark's CPU-baseline leg
 * compare against.  The GPU library never links, loads or calls it, and it
 * shares no code, header or constant table with the GPU path.
 *
 * Readings of the paper that this oracle fixes (the paper leaves them open):
 *   R1  d(x_i, x_j) is the squared Euclidean distance, summed in FP64 over the
 *       exact FP32 inputs in increasing dimension order (Sec. 1 names l1 or
 *       l2; Eqn 2 works with squared l2).
 *   R2  The two-means clustering is plain Lloyd 2-means on the sum-of-squares
 *       objective (the boost k-means objective of Sec. 3.1 is not defined in
 *       the paper).
 *   R3  The two starting centres are two distinct members drawn with a keyed
 *       SplitMix64 hash of (seed, tree, smallest member id, node size, j);
 *       the tree index in the key makes every round different (Sec. 3.1
 *       states that the clustering differs from round to round).
 *   R4  At most I_max assignment passes; stop when no label changes or a
 *       side is empty.  A point equidistant from both centres goes left.
 *   R5  A node is split iff it holds more than leaf_max points (Sec. 3.1
 *       bounds the cluster size by a threshold).  A side smaller than min_leaf is
 *       repaired by re-splitting on the rank of the margin
 *       mu = |x-c0|^2 - |x-c1|^2 (ties by id), left size clamped to
 *       [min_leaf, m-min_leaf]; if every margin is equal the left size is
 *       floor(m/2).
 *   R6  The initial G of Alg. 1 is an empty list per row, (-1, +inf) padding.
 *   R7  Alg. 1 skips pairs compared before; this is realised as de-duplication by id when
 *       a candidate is inserted: G[i] is the k smallest (d, id) over the
 *       distinct co-leaf members seen in all rounds, which is exactly what
 *       Algorithm 1's update produces (a rejected pair stays rejected since
 *       the k-th distance of a row never grows).
 *   R8  Rows are ordered by ascending (d, id).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Keyed random pair (reading R3).                                     */
/* SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014).       */
/* ------------------------------------------------------------------ */
#define ORC_GAMMA 0x9e3779b97f4a7c15ULL

uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

/* One SplitMix64 step from state (h xor w): absorb each key word in turn. */
uint64_t orc_key_hash(uint64_t seed, uint64_t tree, uint64_t min_id,
                      uint64_t size, uint64_t j)
{
    uint64_t words[4] = {tree, min_id, size, j};
    uint64_t h = seed;
    for (int i = 0; i < 4; ++i)
        h = orc_mix64((h ^ words[i]) + ORC_GAMMA);
    return h;
}

/* Indices a != b in [0, m) of the two starting centres (m >= 2). */
void orc_init_pair(uint64_t seed, int tree, int min_id, int64_t m,
                   int64_t *a_out, int64_t *b_out)
{
    uint64_t u0 = orc_key_hash(seed, (uint64_t)tree, (uint64_t)min_id, (uint64_t)m, 0);
    uint64_t u1 = orc_key_hash(seed, (uint64_t)tree, (uint64_t)min_id, (uint64_t)m, 1);
    int64_t a = (int64_t)(u0 % (uint64_t)m);
    int64_t b = (int64_t)(u1 % (uint64_t)(m - 1));
    if (b >= a) b += 1;
    *a_out = a;
    *b_out = b;
}

/* ------------------------------------------------------------------ */
/* Distances (reading R1).                                             */
/* ------------------------------------------------------------------ */
double orc_d64(const float *X, int D, int64_t i, int64_t j)
{
    const float *xi = X + (size_t)i * D, *xj = X + (size_t)j * D;
    double s = 0.0;
    for (int d = 0; d < D; ++d) {
        double t = (double)xi[d] - (double)xj[d];
        s += t * t;
    }
    return s;
}

static double dist_to_centre(const float *x, const double *c, int D)
{
    double s = 0.0;
    for (int d = 0; d < D; ++d) {
        double t = (double)x[d] - c[d];
        s += t * t;
    }
    return s;
}

/* (d, id) lexicographic order, ids as signed ints. */
static int pair_less(double da, int ia, double db, int ib)
{
    return da < db || (da == db && ia < ib);
}

/* Keep row (ids, ds, *cnt) as the k smallest (d, id) seen so far, distinct
 * ids only.  Plain insertion into a sorted array. */
static void row_insert(int *ids, double *ds, int *cnt, int k, int j, double d)
{
    for (int p = 0; p < *cnt; ++p)
        if (ids[p] == j) return; /* already present (reading R7) */
    if (*cnt == k && !pair_less(d, j, ds[k - 1], ids[k - 1])) return;
    int p = (*cnt < k) ? *cnt : k - 1; /* slot that is freed */
    while (p > 0 && pair_less(d, j, ds[p - 1], ids[p - 1])) {
        ids[p] = ids[p - 1];
        ds[p] = ds[p - 1];
        --p;
    }
    ids[p] = j;
    ds[p] = d;
    if (*cnt < k) ++*cnt;
}

/* ------------------------------------------------------------------ */
/* Exact k nearest neighbours of selected rows (brute force, FP64).    */
/* ids/dists are [nq, k]; padded with (-1, +inf) when n-1 < k.          */
/* ------------------------------------------------------------------ */
int orc_exact_knn(const float *X, int64_t n, int D, int k, const int64_t *rows,
                  int64_t nq, int32_t *ids, double *dists)
{
    if (n < 1 || D < 1 || k < 1) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nq; ++q) {
        int64_t i = rows[q];
        int *ri = (int *)ids + q * k;
        double *rd = dists + q * k;
        int cnt = 0;
        for (int p = 0; p < k; ++p) { ri[p] = -1; rd[p] = INFINITY; }
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            row_insert(ri, rd, &cnt, k, (int)j, orc_d64(X, D, i, j));
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* One two-means bisection of a member set (Sec. 3.1; readings R2-R5). */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t assign_rows;   /* sum over assignment passes of members assigned */
    int64_t passes;        /* assignment passes */
    int64_t splits;        /* bisections performed */
    int64_t repairs;       /* bisections repaired by margin rank */
} orc_stats;

static void assign_pass(const float *X, int D, const int32_t *mem, int64_t m,
                        const double *c0, const double *c1, unsigned char *lab)
{
    for (int64_t p = 0; p < m; ++p) {
        const float *x = X + (size_t)mem[p] * D;
        double d0 = dist_to_centre(x, c0, D);
        double d1 = dist_to_centre(x, c1, D);
        lab[p] = (d1 < d0) ? 1 : 0; /* ties go left (R4) */
    }
}

typedef struct { double mu; int32_t id; } mu_rec;

static int mu_cmp(const void *a, const void *b)
{
    const mu_rec *x = (const mu_rec *)a, *y = (const mu_rec *)b;
    if (x->mu < y->mu) return -1;
    if (x->mu > y->mu) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* mem: member ids in increasing order, m >= 2*min_leaf.
 * lab: output label per member (0 = left, 1 = right).
 * c_out (optional, 2*D): the final centres (c0 then c1).
 * Returns the number of members labelled 0. */
/* Same as orc_split with the starting centres given as member positions
 * a != b (orc_split draws them with the keyed hash, reading R3). */
int64_t orc_split_init(const float *X, int D, const int32_t *mem, int64_t m,
                       int min_leaf, int max_iter, int64_t a, int64_t b,
                       unsigned char *lab, double *c_out, int *repaired_out,
                       orc_stats *st)
{
    double *c0 = (double *)malloc(sizeof(double) * D);
    double *c1 = (double *)malloc(sizeof(double) * D);
    double *s0 = (double *)malloc(sizeof(double) * D);
    double *s1 = (double *)malloc(sizeof(double) * D);
    unsigned char *nl = (unsigned char *)malloc((size_t)m);

    for (int d = 0; d < D; ++d) {
        c0[d] = (double)X[(size_t)mem[a] * D + d];
        c1[d] = (double)X[(size_t)mem[b] * D + d];
    }
    assign_pass(X, D, mem, m, c0, c1, lab);
    int64_t passes = 1;

    for (int it = 1; it < max_iter; ++it) {
        int64_t n1 = 0;
        for (int64_t p = 0; p < m; ++p) n1 += lab[p];
        if (n1 == 0 || n1 == m) break; /* one side empty: nothing to move */
        /* centres <- means of the two sides */
        for (int d = 0; d < D; ++d) { s0[d] = 0.0; s1[d] = 0.0; }
        for (int64_t p = 0; p < m; ++p) {
            const float *x = X + (size_t)mem[p] * D;
            double *s = lab[p] ? s1 : s0;
            for (int d = 0; d < D; ++d) s[d] += (double)x[d];
        }
        for (int d = 0; d < D; ++d) {
            c0[d] = s0[d] / (double)(m - n1);
            c1[d] = s1[d] / (double)n1;
        }
        assign_pass(X, D, mem, m, c0, c1, nl);
        ++passes;
        int changed = memcmp(nl, lab, (size_t)m) != 0;
        memcpy(lab, nl, (size_t)m);
        if (!changed) break; /* converged */
    }

    int64_t n0 = 0;
    for (int64_t p = 0; p < m; ++p) n0 += (lab[p] == 0);
    int repaired = 0;
    if (n0 < min_leaf || m - n0 < min_leaf) {
        /* margin-rank repair (R5) */
        repaired = 1;
        mu_rec *r = (mu_rec *)malloc(sizeof(mu_rec) * (size_t)m);
        for (int64_t p = 0; p < m; ++p) {
            const float *x = X + (size_t)mem[p] * D;
            r[p].mu = dist_to_centre(x, c0, D) - dist_to_centre(x, c1, D);
            r[p].id = mem[p];
        }
        int all_equal = 1;
        for (int64_t p = 1; p < m; ++p)
            if (r[p].mu != r[0].mu) { all_equal = 0; break; }
        int64_t s;
        if (all_equal) {
            s = m / 2;
        } else {
            s = n0;
            if (s < min_leaf) s = min_leaf;
            if (s > m - min_leaf) s = m - min_leaf;
        }
        qsort(r, (size_t)m, sizeof(mu_rec), mu_cmp);
        /* members are sorted by id, so rank -> position by binary search */
        for (int64_t q = 0; q < m; ++q) {
            int64_t lo = 0, hi = m - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (mem[mid] < r[q].id) lo = mid + 1; else hi = mid;
            }
            lab[lo] = (q < s) ? 0 : 1;
        }
        n0 = s;
        free(r);
    }

    if (c_out) {
        memcpy(c_out, c0, sizeof(double) * D);
        memcpy(c_out + D, c1, sizeof(double) * D);
    }
    if (repaired_out) *repaired_out = repaired;
    if (st) {
        st->passes += passes;
        st->assign_rows += passes * m;
        st->splits += 1;
        st->repairs += repaired;
    }
    free(c0); free(c1); free(s0); free(s1); free(nl);
    return n0;
}

int64_t orc_split(const float *X, int D, const int32_t *mem, int64_t m,
                  int min_leaf, int max_iter, uint64_t seed, int tree,
                  unsigned char *lab, double *c_out, int *repaired_out,
                  orc_stats *st)
{
    int64_t a, b; /* starting centres: two distinct members (R3) */
    orc_init_pair(seed, tree, mem[0], m, &a, &b);
    return orc_split_init(X, D, mem, m, min_leaf, max_iter, a, b, lab, c_out,
                          repaired_out, st);
}

/* ------------------------------------------------------------------ */
/* One tree: recursive bisection down to leaves (Alg. 1: clustering    */
/* by two-means, then the collection of the clusters).                 */
/* perm is filled in depth-first order, left child first, so that      */
/* every node is a contiguous run of perm and every leaf too.          */
/* ------------------------------------------------------------------ */
typedef struct {
    const float *X;
    int D, leaf_max, min_leaf, max_iter, tree;
    uint64_t seed;
    int32_t *perm;
    int32_t *leaf_off;   /* leaf start positions; count in n_leaves */
    int64_t n_leaves;
    int32_t *nodes;      /* internal nodes: (start, size, n_left, depth) */
    int64_t n_nodes, nodes_cap;
    int depth_max;
    orc_stats st;
} tree_ctx;

static void build_rec(tree_ctx *cx, int32_t *mem, int64_t m, int64_t start, int depth)
{
    if (depth > cx->depth_max) cx->depth_max = depth;
    if (m <= cx->leaf_max) {
        memcpy(cx->perm + start, mem, sizeof(int32_t) * (size_t)m);
        cx->leaf_off[cx->n_leaves++] = (int32_t)start;
        return;
    }
    unsigned char *lab = (unsigned char *)malloc((size_t)m);
    int64_t n0 = orc_split(cx->X, cx->D, mem, m, cx->min_leaf, cx->max_iter,
                           cx->seed, cx->tree, lab, NULL, NULL, &cx->st);
    int32_t *left = (int32_t *)malloc(sizeof(int32_t) * (size_t)n0);
    int32_t *right = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m - n0));
    int64_t a = 0, b = 0;
    for (int64_t p = 0; p < m; ++p) { /* stable: keeps ids increasing */
        if (lab[p] == 0) left[a++] = mem[p]; else right[b++] = mem[p];
    }
    free(lab);
    if (cx->nodes && cx->n_nodes < cx->nodes_cap) {
        int32_t *r = cx->nodes + 4 * cx->n_nodes;
        r[0] = (int32_t)start; r[1] = (int32_t)m; r[2] = (int32_t)n0; r[3] = depth;
    }
    cx->n_nodes++;
    build_rec(cx, left, n0, start, depth + 1);
    build_rec(cx, right, m - n0, start + n0, depth + 1);
    free(left);
    free(right);
}

/* Build tree `tree`.  perm: [n]; leaf_off: capacity n+1, receives the
 * n_leaves+1 leaf boundaries (ascending, last = n); nodes (optional,
 * capacity nodes_cap records of 4 ints): internal nodes in pre-order.
 * stats (optional, 6 int64): assign_rows, passes, splits, repairs,
 * internal node count, maximum depth.  Returns the number of leaves. */
int64_t orc_tree(const float *X, int64_t n, int D, int leaf_max, int min_leaf,
                 int max_iter, uint64_t seed, int tree, int32_t *perm,
                 int32_t *leaf_off, int32_t *nodes, int64_t nodes_cap,
                 int64_t *stats)
{
    tree_ctx cx;
    memset(&cx, 0, sizeof(cx));
    cx.X = X; cx.D = D; cx.leaf_max = leaf_max; cx.min_leaf = min_leaf;
    cx.max_iter = max_iter; cx.tree = tree; cx.seed = seed;
    cx.perm = perm; cx.leaf_off = leaf_off; cx.nodes = nodes; cx.nodes_cap = nodes_cap;
    int32_t *all = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) all[i] = (int32_t)i;
    build_rec(&cx, all, n, 0, 0);
    free(all);
    leaf_off[cx.n_leaves] = (int32_t)n;
    if (stats) {
        stats[0] = cx.st.assign_rows; stats[1] = cx.st.passes;
        stats[2] = cx.st.splits; stats[3] = cx.st.repairs;
        stats[4] = cx.n_nodes; stats[5] = cx.depth_max;
    }
    return cx.n_leaves;
}

/* ------------------------------------------------------------------ */
/* Exhaustive comparison inside each cluster and update of G (Alg. 1,  */
/* inner loops over S_m and <i, j>, readings R6-R8).                   */
/* ------------------------------------------------------------------ */
static void graph_init(int32_t *ids, double *ds, int *cnt, int64_t n, int k)
{
    for (int64_t i = 0; i < n * k; ++i) { ids[i] = -1; ds[i] = INFINITY; }
    memset(cnt, 0, sizeof(int) * (size_t)n);
}

/* Every unordered pair of a leaf updates both rows.  Leaves of one tree are
 * disjoint, so distinct leaves touch distinct rows. */
static void graph_update_tree(const float *X, int D, int k, const int32_t *perm,
                              const int32_t *leaf_off, int64_t n_leaves,
                              int32_t *ids, double *ds, int *cnt)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t l = 0; l < n_leaves; ++l) {
        int64_t s = leaf_off[l], e = leaf_off[l + 1];
        for (int64_t p = s; p < e; ++p) {
            for (int64_t q = p + 1; q < e; ++q) {
                int i = perm[p], j = perm[q];
                double d = orc_d64(X, D, i, j);
                row_insert(ids + (size_t)i * k, ds + (size_t)i * k, cnt + i, k, j, d);
                row_insert(ids + (size_t)j * k, ds + (size_t)j * k, cnt + j, k, i, d);
            }
        }
    }
}

/* Graph from given leaves.  perm: [n_trees, n]; leaf_off: the per-tree
 * boundary arrays concatenated (n_leaves[t] + 1 entries each). */
int orc_graph_from_leaves(const float *X, int64_t n, int D, int k, int n_trees,
                          const int32_t *perm, const int32_t *leaf_off,
                          const int64_t *n_leaves, int32_t *ids, double *ds)
{
    int *cnt = (int *)malloc(sizeof(int) * (size_t)n);
    if (!cnt) return -1;
    graph_init(ids, ds, cnt, n, k);
    int64_t off = 0;
    for (int t = 0; t < n_trees; ++t) {
        graph_update_tree(X, D, k, perm + (size_t)t * n, leaf_off + off,
                          n_leaves[t], ids, ds, cnt);
        off += n_leaves[t] + 1;
    }
    free(cnt);
    return 0;
}

/* Full Algorithm 1: n_trees rounds of bisection + leaf comparison.
 * stats (optional, 6 int64): summed tree stats (max for depth). */
int orc_graph(const float *X, int64_t n, int D, int k, int n_trees, int leaf_max,
              int min_leaf, int max_iter, uint64_t seed, int32_t *ids, double *ds,
              int64_t *stats)
{
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * n_trees);
    int32_t *loff = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1) * n_trees);
    int64_t *nl = (int64_t *)malloc(sizeof(int64_t) * n_trees);
    int64_t *st = (int64_t *)calloc((size_t)6 * n_trees, sizeof(int64_t));
    int *cnt = (int *)malloc(sizeof(int) * (size_t)n);
    if (!perm || !loff || !nl || !st || !cnt) return -1;
    /* the rounds' partitions are independent of each other */
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < n_trees; ++t)
        nl[t] = orc_tree(X, n, D, leaf_max, min_leaf, max_iter, seed, t,
                         perm + (size_t)t * n, loff + (size_t)t * (n + 1),
                         NULL, 0, st + 6 * t);
    graph_init(ids, ds, cnt, n, k);
    for (int t = 0; t < n_trees; ++t)
        graph_update_tree(X, D, k, perm + (size_t)t * n, loff + (size_t)t * (n + 1),
                          nl[t], ids, ds, cnt);
    if (stats) {
        for (int c = 0; c < 6; ++c) stats[c] = 0;
        for (int t = 0; t < n_trees; ++t) {
            for (int c = 0; c < 5; ++c) stats[c] += st[6 * t + c];
            if (st[6 * t + 5] > stats[5]) stats[5] = st[6 * t + 5];
        }
    }
    free(perm); free(loff); free(nl); free(st); free(cnt);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t)
{
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Rows `rows[q]` of the graph from given leaves (same result as
 * orc_graph_from_leaves restricted to those rows).  Used where n is too large
 * for the full graph.  perm / leaf_off / n_leaves as in orc_graph_from_leaves. */
int orc_rows_from_leaves(const float *X, int64_t n, int D, int k, int n_trees,
                         const int32_t *perm, const int32_t *leaf_off,
                         const int64_t *n_leaves, const int64_t *rows, int64_t nq,
                         int32_t *ids, double *ds)
{
    int32_t *inv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * n_trees);
    const int32_t **offs = (const int32_t **)malloc(sizeof(int32_t *) * n_trees);
    if (!inv || !offs) return -1;
    int64_t o = 0;
    for (int t = 0; t < n_trees; ++t) {
        for (int64_t p = 0; p < n; ++p) inv[(size_t)t * n + perm[(size_t)t * n + p]] = (int32_t)p;
        offs[t] = leaf_off + o;
        o += n_leaves[t] + 1;
    }
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t q = 0; q < nq; ++q) {
        int64_t i = rows[q];
        int32_t *ri = ids + q * k;
        double *rd = ds + q * k;
        int cnt = 0;
        for (int p = 0; p < k; ++p) { ri[p] = -1; rd[p] = INFINITY; }
        for (int t = 0; t < n_trees; ++t) {
            int64_t pos = inv[(size_t)t * n + i];
            /* leaf l with offs[l] <= pos < offs[l+1] */
            int64_t lo = 0, hi = n_leaves[t] - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) / 2;
                if (offs[t][mid] <= pos) lo = mid; else hi = mid - 1;
            }
            for (int64_t p = offs[t][lo]; p < offs[t][lo + 1]; ++p) {
                int32_t j = perm[(size_t)t * n + p];
                if (j != i) row_insert(ri, rd, &cnt, k, j, orc_d64(X, D, i, j));
            }
        }
    }
    free(inv);
    free(offs);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Reduced-precision first pass (the leaf distances of the reduced     */
/* path), emulated: reading R9.                                        */
/*   R9  x~_i = rnd(sigma_i x_i) in the format (round to nearest, ties */
/*       to even, with the format's subnormals); sigma_i = 1 for BF16, */
/*       else 2^(E - floor(log2 max_d |x_id|) - 1), E = 15 (FP16) or 8 */
/*       (FP8-e4m3), so |sigma x| < 2^E.  d~(i,j) = |x~_i/s_i - x~_j/s_j|^2  */
/*       computed as n~_i + n~_j - 2 <x~_i/s_i, x~_j/s_j> in FP64.  Per */
/*       row and leaf the c smallest (d~, j) are re-ranked by d64 and the */
/*       k smallest (d64, j) kept; rows are then merged as in R7.       */
/* ------------------------------------------------------------------ */
enum { ORC_BF16 = 1, ORC_FP16 = 2, ORC_FP8 = 3 };

/* Nearest value with `mant` fraction bits and smallest normal exponent
 * emin (evenly spaced subnormals below it); ties to even.  Every step is
 * exact in double for mant <= 10. */
double orc_round_fmt(double x, int mant, int emin)
{
    if (x == 0.0) return x;
    int e;
    frexp(x, &e);
    e -= 1; /* |x| in [2^e, 2^(e+1)) */
    if (e < emin) e = emin;
    double ulp = ldexp(1.0, e - mant);
    return nearbyint(x / ulp) * ulp; /* default rounding mode: ties to even */
}

double orc_quantize(int fmt, double x)
{
    switch (fmt) {
    case ORC_BF16: return orc_round_fmt(x, 7, -126);
    case ORC_FP16: return orc_round_fmt(x, 10, -14);
    case ORC_FP8: return orc_round_fmt(x, 3, -6);
    default: return x;
    }
}

/* Power-of-two scale sigma of one row (R9). */
double orc_row_scale(int fmt, const float *x, int D)
{
    if (fmt == ORC_BF16) return 1.0;
    double mx = 0.0;
    for (int d = 0; d < D; ++d) {
        double a = fabs((double)x[d]);
        if (a > mx) mx = a;
    }
    if (mx == 0.0) return 1.0;
    int e;
    frexp(mx, &e); /* mx in [2^(e-1), 2^e): floor(log2 mx) = e-1 */
    int E = (fmt == ORC_FP16) ? 15 : 8;
    return ldexp(1.0, E - (e - 1) - 1);
}

/* Dequantised reduced row x~/sigma. */
static void reduced_row(int fmt, const float *x, int D, double *out)
{
    double s = orc_row_scale(fmt, x, D);
    for (int d = 0; d < D; ++d) out[d] = orc_quantize(fmt, (double)x[d] * s) / s;
}

typedef struct { double d; int32_t j; } dj_rec;

static int dj_cmp(const void *a, const void *b)
{
    const dj_rec *x = (const dj_rec *)a, *y = (const dj_rec *)b;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    return (x->j > y->j) - (x->j < y->j);
}

/* First-pass distances (R9) of member a of a leaf to every other member:
 * the n~_a + n~_b - 2 <x~_a/s_a, x~_b/s_b> of the dequantised rows q
 * (m x D) with squared norms nq, in FP64; r receives (d~, id) for every
 * b != a, sorted by (d~, id).  Returns the number of entries, m - 1. */
static int reduced_first_pass(const int32_t *ids, int64_t m, int D, int64_t a,
                              const double *q, const double *nq, dj_rec *r)
{
    int nr = 0;
    for (int64_t b = 0; b < m; ++b) {
        if (b == a) continue;
        double g = 0.0;
        for (int d = 0; d < D; ++d) g += q[a * D + d] * q[b * D + d];
        r[nr].d = nq[a] + nq[b] - 2.0 * g;
        r[nr].j = ids[b];
        ++nr;
    }
    qsort(r, (size_t)nr, sizeof(dj_rec), dj_cmp);
    return nr;
}

/* Dequantised rows (R9) of the m points ids[0..m) into q (m x D) and their
 * squared norms into nq. */
static void reduced_leaf_rows(int fmt, const float *X, int D, const int32_t *ids, int64_t m,
                              double *q, double *nq)
{
    for (int64_t a = 0; a < m; ++a) {
        reduced_row(fmt, X + (size_t)ids[a] * D, D, q + a * D);
        double acc = 0.0;
        for (int d = 0; d < D; ++d) acc += q[a * D + d] * q[a * D + d];
        nq[a] = acc;
    }
}

/* Re-rank (R9): the first cc = min(c, nr) entries of the sorted first pass
 * take the exact d64 of their pair and are sorted by (d64, id). */
static int reduced_rerank(const float *X, int D, int64_t i, dj_rec *r, int nr, int c)
{
    int cc = nr < c ? nr : c;
    for (int p = 0; p < cc; ++p) r[p].d = orc_d64(X, D, i, r[p].j);
    qsort(r, (size_t)cc, sizeof(dj_rec), dj_cmp);
    return cc;
}

/* Graph from given leaves with the reduced first pass (R9); arguments as
 * orc_graph_from_leaves plus the format and c candidates per row and leaf. */
int orc_graph_from_leaves_reduced(const float *X, int64_t n, int D, int k, int n_trees,
                                  const int32_t *perm, const int32_t *leaf_off,
                                  const int64_t *n_leaves, int fmt, int c,
                                  int32_t *ids, double *ds)
{
    int *cnt = (int *)malloc(sizeof(int) * (size_t)n);
    if (!cnt) return -1;
    graph_init(ids, ds, cnt, n, k);
    int64_t off = 0;
    for (int t = 0; t < n_trees; ++t) {
        const int32_t *pm = perm + (size_t)t * n;
        const int32_t *lo = leaf_off + off;
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t l = 0; l < n_leaves[t]; ++l) {
            int64_t s = lo[l], m = lo[l + 1] - lo[l];
            double *q = (double *)malloc(sizeof(double) * (size_t)(m * D));
            double *nq = (double *)malloc(sizeof(double) * (size_t)m);
            dj_rec *r = (dj_rec *)malloc(sizeof(dj_rec) * (size_t)m);
            reduced_leaf_rows(fmt, X, D, pm + s, m, q, nq);
            for (int64_t a = 0; a < m; ++a) {
                int i = pm[s + a];
                int nr = reduced_first_pass(pm + s, m, D, a, q, nq, r);
                int cc = reduced_rerank(X, D, i, r, nr, c);
                for (int p = 0; p < cc && p < k; ++p)
                    row_insert(ids + (size_t)i * k, ds + (size_t)i * k, cnt + i, k, r[p].j, r[p].d);
            }
            free(q); free(nq); free(r);
        }
        off += n_leaves[t] + 1;
    }
    free(cnt);
    return 0;
}

/* First-pass distance d~(i, j) of one pair (R9), FP64. */
double orc_dtilde(const float *X, int D, int fmt, int64_t i, int64_t j)
{
    double *q = (double *)malloc(sizeof(double) * (size_t)(2 * D));
    if (!q) return NAN;
    reduced_row(fmt, X + (size_t)i * D, D, q);
    reduced_row(fmt, X + (size_t)j * D, D, q + D);
    double ni = 0.0, nj = 0.0, g = 0.0;
    for (int d = 0; d < D; ++d) ni += q[d] * q[d];
    for (int d = 0; d < D; ++d) nj += q[D + d] * q[D + d];
    for (int d = 0; d < D; ++d) g += q[d] * q[D + d];
    free(q);
    return ni + nj - 2.0 * g;
}

/* First-pass distances d~(i, js[p]) for p < nj (R9), FP64, into out. */
int orc_dtilde_row(const float *X, int D, int fmt, int64_t i, const int32_t *js, int64_t nj,
                   double *out)
{
    double *qi = (double *)malloc(sizeof(double) * (size_t)D);
    double *qj = (double *)malloc(sizeof(double) * (size_t)D);
    if (!qi || !qj) { free(qi); free(qj); return -1; }
    reduced_row(fmt, X + (size_t)i * D, D, qi);
    double ni = 0.0;
    for (int d = 0; d < D; ++d) ni += qi[d] * qi[d];
    for (int64_t p = 0; p < nj; ++p) {
        reduced_row(fmt, X + (size_t)js[p] * D, D, qj);
        double nj2 = 0.0, g = 0.0;
        for (int d = 0; d < D; ++d) nj2 += qj[d] * qj[d];
        for (int d = 0; d < D; ++d) g += qi[d] * qj[d];
        out[p] = ni + nj2 - 2.0 * g;
    }
    free(qi); free(qj);
    return 0;
}

/* Rows `rows[q]` of orc_graph_from_leaves_reduced (same result restricted to
 * those rows), for n too large for the full graph.  thr (nullable, [nq][n_trees][2])
 * receives, per row and tree, the first-pass distances of the c-th and the
 * (c+1)-th entry of the row's sorted first pass in its leaf: the last
 * candidate kept and the first one dropped (+inf where the leaf has no such
 * entry). */
int orc_rows_from_leaves_reduced(const float *X, int64_t n, int D, int k, int n_trees,
                                 const int32_t *perm, const int32_t *leaf_off,
                                 const int64_t *n_leaves, int fmt, int c,
                                 const int64_t *rows, int64_t nq, int32_t *ids, double *ds,
                                 double *thr)
{
    int32_t *inv = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * n_trees);
    const int32_t **offs = (const int32_t **)malloc(sizeof(int32_t *) * n_trees);
    if (!inv || !offs) return -1;
    int64_t o = 0;
    for (int t = 0; t < n_trees; ++t) {
        for (int64_t p = 0; p < n; ++p) inv[(size_t)t * n + perm[(size_t)t * n + p]] = (int32_t)p;
        offs[t] = leaf_off + o;
        o += n_leaves[t] + 1;
    }
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t qi = 0; qi < nq; ++qi) {
        int64_t i = rows[qi];
        int32_t *ri = ids + qi * k;
        double *rd = ds + qi * k;
        int cnt = 0;
        for (int p = 0; p < k; ++p) { ri[p] = -1; rd[p] = INFINITY; }
        for (int t = 0; t < n_trees; ++t) {
            const int32_t *pm = perm + (size_t)t * n;
            int64_t pos = inv[(size_t)t * n + i];
            int64_t lo = 0, hi = n_leaves[t] - 1;
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) / 2;
                if (offs[t][mid] <= pos) lo = mid; else hi = mid - 1;
            }
            int64_t s = offs[t][lo], m = offs[t][lo + 1] - s;
            double *q = (double *)malloc(sizeof(double) * (size_t)(m * D));
            double *nqv = (double *)malloc(sizeof(double) * (size_t)m);
            dj_rec *r = (dj_rec *)malloc(sizeof(dj_rec) * (size_t)m);
            if (!q || !nqv || !r) {
#pragma omp atomic write
                fail = 1;
                free(q); free(nqv); free(r);
                continue;
            }
            reduced_leaf_rows(fmt, X, D, pm + s, m, q, nqv);
            int nr = reduced_first_pass(pm + s, m, D, pos - s, q, nqv, r);
            if (thr) {
                thr[(qi * n_trees + t) * 2] = c <= nr ? r[c - 1].d : INFINITY;
                thr[(qi * n_trees + t) * 2 + 1] = c < nr ? r[c].d : INFINITY;
            }
            int cc = reduced_rerank(X, D, i, r, nr, c);
            for (int p = 0; p < cc && p < k; ++p) row_insert(ri, rd, &cnt, k, r[p].j, r[p].d);
            free(q); free(nqv); free(r);
        }
    }
    free(inv);
    free(offs);
    return fail ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Enhanced hill-climbing search over a kNN graph (Alg. 2, E-GNNS).    */
/*   R10 A node is visited once its distance to the query has been     */
/*       taken (seeds included); each node enters the rank list once;  */
/*       seed ids outside [0, n) are ignored.                          */
/*   R11 The rank list R is ordered by ascending (d, id).  Only its k   */
/*       best entries are kept: an entry outside them can never return, */
/*       since the k-th distance of R never grows.                     */
/*   R12 Each round expands every member of the top-k of R as R stood   */
/*       at the start of the round; the new neighbours T are merged     */
/*       after the round (R <- R u T).  A member expanded in an earlier */
/*       round adds nothing (its neighbours are visited), and a round   */
/*       without an unexpanded member ends the search (later rounds add */
/*       nothing either).  Graph entries < 0 are padding.               */
/*   R13 The output is the top-k of R, padded with (-1, +inf).  The     */
/*       rank order is taken in d64 (dist_mode 0, R1) or in the         */
/*       canonical FP32 d32 (dist_mode 1): per block of 32 dimensions a */
/*       sequential fused multiply-add of (q_d - x_d)^2 from 0, blocks  */
/*       added in increasing order in FP32 -- the GPU search's order.   */
/* ------------------------------------------------------------------ */
static float d32_canonical(const float *a, const float *b, int D)
{
    float tot = 0.0f;
    for (int d0 = 0; d0 < D; d0 += 32) {
        int dn = D - d0 < 32 ? D - d0 : 32;
        float blk = 0.0f;
        for (int dd = 0; dd < dn; ++dd) {
            float df = a[d0 + dd] - b[d0 + dd];
            blk = fmaf(df, df, blk);
        }
        tot = tot + blk;
    }
    return tot;
}

double orc_d32(const float *a, const float *b, int D) { return (double)d32_canonical(a, b, D); }

static double query_dist(const float *q, const float *x, int D, int dist_mode)
{
    if (dist_mode == 1) return (double)d32_canonical(q, x, D);
    double s = 0.0;
    for (int d = 0; d < D; ++d) {
        double df = (double)q[d] - (double)x[d];
        s += df * df;
    }
    return s;
}

/* Insert (j, d) unexpanded into the rank list (rid, rd, rx, *rn <= k). */
static void rank_insert(int32_t *rid, double *rd, unsigned char *rx, int *rn, int k,
                        int32_t j, double d)
{
    if (*rn == k && !pair_less(d, j, rd[k - 1], rid[k - 1])) return;
    int p = (*rn < k) ? *rn : k - 1;
    while (p > 0 && pair_less(d, j, rd[p - 1], rid[p - 1])) {
        rid[p] = rid[p - 1];
        rd[p] = rd[p - 1];
        rx[p] = rx[p - 1];
        --p;
    }
    rid[p] = j;
    rd[p] = d;
    rx[p] = 0;
    if (*rn < k) ++*rn;
}

/* Queries Q [nq, D], graph G [n, kg], seeds [nq, ns]; outputs [nq, k].
 * work_out (nullable, [2]): distances taken over all queries (each visited
 * node once, seeds included) and nodes expanded. */
int orc_egnns(const float *X, int64_t n, int D, const int32_t *G, int kg, const float *Q,
              int64_t nq, const int32_t *seeds, int ns, int k, int rounds, int dist_mode,
              int32_t *ids_out, double *d_out, int64_t *work_out)
{
    int fail = 0;
    int64_t n_dist = 0, n_exp = 0;
#pragma omp parallel
    {
        unsigned char *vis = (unsigned char *)calloc((size_t)n, 1);
        int32_t *touched = (int32_t *)malloc(sizeof(int32_t) *
                                             ((size_t)ns + (size_t)rounds * k * kg + 1));
        int32_t *rid = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        double *rd = (double *)malloc(sizeof(double) * (size_t)k);
        unsigned char *rx = (unsigned char *)malloc((size_t)k);
        int32_t *front = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
        int32_t *tid = (int32_t *)malloc(sizeof(int32_t) * (size_t)k * kg);
        double *td = (double *)malloc(sizeof(double) * (size_t)k * kg);
        if (!vis || !touched || !rid || !rd || !rx || !front || !tid || !td) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 4) reduction(+ : n_dist, n_exp)
            for (int64_t qi = 0; qi < nq; ++qi) {
                const float *q = Q + (size_t)qi * D;
                int rn = 0, nt = 0;
                for (int s = 0; s < ns; ++s) {
                    int32_t j = seeds[(size_t)qi * ns + s];
                    if (j < 0 || j >= n || vis[j]) continue;
                    vis[j] = 1;
                    touched[nt++] = j;
                    rank_insert(rid, rd, rx, &rn, k, j, query_dist(q, X + (size_t)j * D, D, dist_mode));
                }
                for (int t = 0; t < rounds; ++t) {
                    int nf = 0;
                    for (int p = 0; p < rn; ++p)
                        if (!rx[p]) {
                            front[nf++] = rid[p];
                            rx[p] = 1;
                        }
                    if (nf == 0) break;
                    n_exp += nf;
                    int nT = 0;
                    for (int f = 0; f < nf; ++f)
                        for (int e = 0; e < kg; ++e) {
                            int32_t j = G[(size_t)front[f] * kg + e];
                            if (j < 0 || j >= n || vis[j]) continue;
                            vis[j] = 1;
                            touched[nt++] = j;
                            tid[nT] = j;
                            td[nT] = query_dist(q, X + (size_t)j * D, D, dist_mode);
                            ++nT;
                        }
                    for (int e = 0; e < nT; ++e) rank_insert(rid, rd, rx, &rn, k, tid[e], td[e]);
                }
                for (int p = 0; p < k; ++p) {
                    ids_out[(size_t)qi * k + p] = p < rn ? rid[p] : -1;
                    d_out[(size_t)qi * k + p] = p < rn ? rd[p] : INFINITY;
                }
                n_dist += nt;
                for (int e = 0; e < nt; ++e) vis[touched[e]] = 0;
            }
        }
        free(vis); free(touched); free(rid); free(rd); free(rx); free(front); free(tid); free(td);
    }
    if (work_out) {
        work_out[0] = n_dist;
        work_out[1] = n_exp;
    }
    return fail ? -1 : 0;
}

/* Exact k nearest reference points of external query points (brute force,
 * FP64, R1; ascending (d, id)); ground truth for the search's recall. */
int orc_exact_knn_points(const float *X, int64_t n, int D, const float *Q, int64_t nq, int k,
                         int32_t *ids, double *dists)
{
    if (n < 1 || D < 1 || k < 1) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nq; ++q) {
        int *ri = (int *)ids + q * k;
        double *rd = dists + q * k;
        int cnt = 0;
        for (int p = 0; p < k; ++p) { ri[p] = -1; rd[p] = INFINITY; }
        for (int64_t j = 0; j < n; ++j)
            row_insert(ri, rd, &cnt, k, (int)j,
                       query_dist(Q + (size_t)q * D, X + (size_t)j * D, D, 0));
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Inverted index from residue vector quantisation, feeding search     */
/* seeds (Sec. 4.1-4.2, Eqns 1-3).  Readings:                          */
/*   R14 Two RVQ stages (Eqn 1 with two terms): a vocabulary V1 of K1  */
/*       words trained on sample rows of X, and V2 of K2 words trained */
/*       on the sample's stage-1 residues r = x - w1[c1(x)].  Each is  */
/*       trained by Lloyd k-means (the paper names no trainer).  The   */
/*       sample (row ids) and the starting words (distinct positions in */
/*       the sample, one list per stage) are inputs.                   */
/*   R15 Quantiser distance: FP64 squared Euclidean, each term added   */
/*       by a fused multiply-add, dimensions in increasing order from  */
/*       0 (d64f).  The nearest word is the lowest index among equals. */
/*   R16 Lloyd: assign; then up to `iters` rounds of (update, assign), */
/*       stopping after a round whose codes equal the previous ones.   */
/*       Sums run over the sample in increasing position; a word with  */
/*       no member keeps its value; the new word is sum / count.       */
/*   R17 Encoding: c1 = nearest V1 word of x, c2 = nearest V2 word of  */
/*       x - w1[c1]; the index key is I = c1 * K2 + c2, and the list   */
/*       of I holds the ids with that key in increasing id order.      */
/*   R18 Eqn 3 as printed loses signs and a factor 2; its two terms    */
/*       are read as the expansion of Eqn 2:                           */
/*         term1 = (q.q - 2 w1.q) + w1.w1                              */
/*         term2 = (2 w1.w2 + w2.w2) - 2 w2.q,   d(q, I) = term1+term2 */
/*       with every dot product an FP64 fma chain in dimension order   */
/*       over the FP32 query taken exactly; the factors 2 are exact,   */
/*       so the order of each sum is the one written.                  */
/*   R19 Cascade: keep the n1 first-stage words with the smallest      */
/*       (term1, c1); rank their n1 * K2 keys by (d(q, I), I); walk    */
/*       the lists in that order and take their ids as seeds until ns  */
/*       are taken; fewer than ns are padded with -1.                  */
/* ------------------------------------------------------------------ */
static double d64f(const double *v, const double *w, int D)
{
    double s = 0.0;
    for (int d = 0; d < D; ++d) {
        double t = v[d] - w[d];
        s = fma(t, t, s);
    }
    return s;
}

static double dot64f(const double *a, const double *b, int D)
{
    double s = 0.0;
    for (int d = 0; d < D; ++d) s = fma(a[d], b[d], s);
    return s;
}

static int nearest_word(const double *v, const double *W, int K, int D)
{
    int best = 0;
    double bd = d64f(v, W, D);
    for (int j = 1; j < K; ++j) {
        double dj = d64f(v, W + (size_t)j * D, D);
        if (dj < bd) {
            bd = dj;
            best = j;
        }
    }
    return best;
}

static int64_t assign_words(const double *P, int64_t m, int D, const double *W, int K,
                            int32_t *codes)
{
    int64_t changed = 0;
#pragma omp parallel for schedule(static) reduction(+ : changed)
    for (int64_t p = 0; p < m; ++p) {
        int c = nearest_word(P + (size_t)p * D, W, K, D);
        if (c != codes[p]) ++changed;
        codes[p] = c;
    }
    return changed;
}

/* Lloyd k-means (R15, R16) on the rows P [m, D]; W [K, D] starts from the
 * rows init[K] of P; codes [m] = the nearest word of each row under the
 * final W.  Returns the number of update rounds taken, or -1. */
int orc_kmeans(const double *P, int64_t m, int D, int K, const int32_t *init, int iters,
               double *W, int32_t *codes)
{
    if (m < 1 || D < 1 || K < 1 || iters < 0) return -1;
    for (int j = 0; j < K; ++j) {
        if (init[j] < 0 || init[j] >= m) return -1;
        memcpy(W + (size_t)j * D, P + (size_t)init[j] * D, sizeof(double) * (size_t)D);
    }
    for (int64_t p = 0; p < m; ++p) codes[p] = -1;
    assign_words(P, m, D, W, K, codes);
    double *sum = (double *)malloc(sizeof(double) * (size_t)K * D);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    if (!sum || !cnt) {
        free(sum);
        free(cnt);
        return -1;
    }
    int rounds = 0;
    while (rounds < iters) {
        memset(sum, 0, sizeof(double) * (size_t)K * D);
        memset(cnt, 0, sizeof(int64_t) * (size_t)K);
        for (int64_t p = 0; p < m; ++p) {
            int c = codes[p];
            ++cnt[c];
            for (int d = 0; d < D; ++d) sum[(size_t)c * D + d] += P[(size_t)p * D + d];
        }
        for (int j = 0; j < K; ++j)
            if (cnt[j] > 0)
                for (int d = 0; d < D; ++d)
                    W[(size_t)j * D + d] = sum[(size_t)j * D + d] / (double)cnt[j];
        ++rounds;
        if (assign_words(P, m, D, W, K, codes) == 0) break;
    }
    free(sum);
    free(cnt);
    return rounds;
}

/* Two-stage RVQ training (R14): sample rows train_ids[m] of X, starting
 * positions init1[K1], init2[K2] in the sample.  Outputs W1 [K1, D],
 * W2 [K2, D] (FP64), the sample's codes (nullable) and rounds [2]
 * (nullable).  Returns 0 or -1. */
int orc_rvq_train(const float *X, int64_t n, int D, const int32_t *train_ids, int64_t m,
                  int K1, int K2, const int32_t *init1, const int32_t *init2, int iters,
                  double *W1, double *W2, int32_t *codes1, int32_t *codes2, int32_t *rounds)
{
    if (m < 1 || D < 1) return -1;
    double *P = (double *)malloc(sizeof(double) * (size_t)m * D);
    int32_t *c1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    int32_t *c2 = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    int rc = -1;
    if (!P || !c1 || !c2) goto out;
    for (int64_t p = 0; p < m; ++p) {
        if (train_ids[p] < 0 || train_ids[p] >= n) goto out;
        for (int d = 0; d < D; ++d)
            P[(size_t)p * D + d] = (double)X[(size_t)train_ids[p] * D + d];
    }
    int r1 = orc_kmeans(P, m, D, K1, init1, iters, W1, c1);
    if (r1 < 0) goto out;
    for (int64_t p = 0; p < m; ++p)
        for (int d = 0; d < D; ++d) P[(size_t)p * D + d] -= W1[(size_t)c1[p] * D + d];
    int r2 = orc_kmeans(P, m, D, K2, init2, iters, W2, c2);
    if (r2 < 0) goto out;
    if (codes1) memcpy(codes1, c1, sizeof(int32_t) * (size_t)m);
    if (codes2) memcpy(codes2, c2, sizeof(int32_t) * (size_t)m);
    if (rounds) {
        rounds[0] = r1;
        rounds[1] = r2;
    }
    rc = 0;
out:
    free(P);
    free(c1);
    free(c2);
    return rc;
}

/* RVQ encoding and index key of every row (R17): key [n]. */
int orc_rvq_encode(const float *X, int64_t n, int D, const double *W1, int K1,
                   const double *W2, int K2, int32_t *key)
{
    if (n < 0 || D < 1 || K1 < 1 || K2 < 1) return -1;
    int fail = 0;
#pragma omp parallel
    {
        double *v = (double *)malloc(sizeof(double) * (size_t)D);
        if (!v) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                for (int d = 0; d < D; ++d) v[d] = (double)X[(size_t)i * D + d];
                int c1 = nearest_word(v, W1, K1, D);
                for (int d = 0; d < D; ++d) v[d] -= W1[(size_t)c1 * D + d];
                int c2 = nearest_word(v, W2, K2, D);
                key[i] = c1 * K2 + c2;
            }
        }
        free(v);
    }
    return fail ? -1 : 0;
}

/* Inverted lists of the keys (R17): offsets [nkeys + 1], ids [n]. */
int orc_ivf_lists(const int32_t *key, int64_t n, int nkeys, int32_t *offsets, int32_t *ids)
{
    if (n < 0 || nkeys < 1) return -1;
    for (int j = 0; j <= nkeys; ++j) offsets[j] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (key[i] < 0 || key[i] >= nkeys) return -1;
        ++offsets[key[i] + 1];
    }
    for (int j = 0; j < nkeys; ++j) offsets[j + 1] += offsets[j];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)nkeys);
    if (!fill) return -1;
    memcpy(fill, offsets, sizeof(int32_t) * (size_t)nkeys);
    for (int64_t i = 0; i < n; ++i) ids[fill[key[i]]++] = (int32_t)i;
    free(fill);
    return 0;
}

/* term1 [K1] and d(q, I) [K1 * K2] of one query (R18), for every key. */
int orc_ivf_key_dist(const float *q, int D, const double *W1, int K1, const double *W2, int K2,
                     double *term1, double *dist)
{
    double *qv = (double *)malloc(sizeof(double) * (size_t)D);
    if (!qv) return -1;
    for (int d = 0; d < D; ++d) qv[d] = (double)q[d];
    const double qq = dot64f(qv, qv, D);
    for (int j = 0; j < K1; ++j) {
        const double *w1 = W1 + (size_t)j * D;
        term1[j] = (qq - 2.0 * dot64f(w1, qv, D)) + dot64f(w1, w1, D);
        for (int l = 0; l < K2; ++l) {
            const double *w2 = W2 + (size_t)l * D;
            double term2 = (2.0 * dot64f(w1, w2, D) + dot64f(w2, w2, D)) - 2.0 * dot64f(w2, qv, D);
            dist[(size_t)j * K2 + l] = term1[j] + term2;
        }
    }
    free(qv);
    return 0;
}

typedef struct {
    double d;
    int32_t key;
} key_rank;

static int key_rank_cmp(const void *a, const void *b)
{
    const key_rank *x = (const key_rank *)a, *y = (const key_rank *)b;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    return (x->key > y->key) - (x->key < y->key);
}

/* Cascaded seeds of each query (R18, R19): seeds [nq, ns]. */
int orc_ivf_seeds(const float *Q, int64_t nq, int D, const double *W1, int K1, const double *W2,
                  int K2, const int32_t *offsets, const int32_t *ids, int n1, int ns,
                  int32_t *seeds)
{
    if (n1 < 1 || n1 > K1 || ns < 0) return -1;
    int fail = 0;
#pragma omp parallel
    {
        double *t1 = (double *)malloc(sizeof(double) * (size_t)K1);
        double *dist = (double *)malloc(sizeof(double) * (size_t)K1 * K2);
        key_rank *first = (key_rank *)malloc(sizeof(key_rank) * (size_t)K1);
        key_rank *keys = (key_rank *)malloc(sizeof(key_rank) * (size_t)n1 * K2);
        if (!t1 || !dist || !first || !keys) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 4)
            for (int64_t qi = 0; qi < nq; ++qi) {
                int32_t *out = seeds + (size_t)qi * ns;
                orc_ivf_key_dist(Q + (size_t)qi * D, D, W1, K1, W2, K2, t1, dist);
                for (int j = 0; j < K1; ++j) {
                    first[j].d = t1[j];
                    first[j].key = j;
                }
                qsort(first, (size_t)K1, sizeof(key_rank), key_rank_cmp);
                for (int a = 0; a < n1; ++a)
                    for (int l = 0; l < K2; ++l) {
                        const int32_t I = first[a].key * K2 + l;
                        keys[(size_t)a * K2 + l].d = dist[I];
                        keys[(size_t)a * K2 + l].key = I;
                    }
                qsort(keys, (size_t)n1 * K2, sizeof(key_rank), key_rank_cmp);
                int s = 0;
                for (int64_t e = 0; e < (int64_t)n1 * K2 && s < ns; ++e)
                    for (int32_t p = offsets[keys[e].key]; p < offsets[keys[e].key + 1] && s < ns; ++p)
                        out[s++] = ids[p];
                for (; s < ns; ++s) out[s] = -1;
            }
        }
        free(t1);
        free(dist);
        free(first);
        free(keys);
    }
    return fail ? -1 : 0;
}
