/*
 * hm_oracle.c -- plain, slow CPU FP64 oracle for the H^2 evaluation Y = K~ * W.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code with the GPU library: it writes
 * the compressed-representation file from its own code and evaluates K~ * W
 * with its own loops.
 *
 * What it follows (MatRox, arXiv 1812.07152):
 *   - kernel matrix K(i,j) = kernel(x_i, x_j), Gaussian exp(-|x-y|^2/(2h^2))
 *     (Section 1);
 *   - cluster tree by recursive partition of the points down to leaf size m
 *     (Section 3.1, "Tree construction and interaction computation");
 *   - near/far interactions by the admissibility condition
 *     tau * dist(a,b) > diam(a) + diam(b) (Section 2.1, "Compression"), or the
 *     HSS structure where every off-diagonal block is low-rank (Section 4.1);
 *   - interpolative decomposition (ID) giving nested bases (the V / U generators)
 *     and coupling blocks B, near blocks D stored full (Section 3.1,
 *     "Low-rank approximation and sampling"; Section 2.1);
 *   - evaluation as reduction loops over near (D) and far (B) interactions
 *     plus a bottom-up (V) and top-down (U) tree traversal (Section 2.1,
 *     "Evaluation").
 * Readings where the paper is silent (tree split rule, distance/diameter,
 * rank rule, row sampling, ID form) are documented at each function.
 *
 * Everything is row-major FP64.  Points are N x d.  Tree positions t = 0..N-1
 * index the points after the partition; perm[t] is the original index.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR (-1)

typedef struct {
    /* inputs */
    int64_t N;
    int d;
    int kernel;     /* 0 Gaussian exp(-r^2/(2h^2)), 1 Laplace exp(-r/h) */
    double h;
    int m;          /* leaf size */
    double tol;     /* ID tolerance (relative to |R_11|) */
    int rmax;       /* rank cap */
    int adm;        /* 0 distance admissibility, 1 HSS, 2 budget (H^2-b) */
    double tau;
    int part;       /* 0 median of the widest coordinate, 1 two-means direction */
    double budget;  /* budget admissibility: near leaves per leaf = floor(budget * #leaves) */
    int64_t S;      /* row-sample cap */
    uint64_t seed;  /* sample seed */
    double *X;      /* N x d copy of the points (original order) */

    /* tree */
    int L;          /* depth: leaves at level L */
    int n_nodes;
    int64_t *perm;  /* tree position -> original index */
    int64_t *start, *size;
    int *parent, *left, *right, *level;
    double *centroid; /* n_nodes x d */
    double *radius;
    double *split_c;  /* n_nodes x 2d: the two means of a two-means split (tests) */
    unsigned char *leafnear; /* n_leaves x n_leaves near relation (budget admissibility) */

    /* interaction lists (CSR by row node, sorted by column node) */
    int64_t *far_ptr;  int *far_col;  int64_t n_far;
    int64_t *near_ptr; int *near_col; int64_t n_near;

    /* nested basis: P (leaf, k x size) or T (internal, k x (k_l+k_r)) */
    int *rank;
    int64_t *basis_off; double *basis; int64_t basis_len;
    int64_t *skel_ptr;  int64_t *skel; int64_t skel_len; /* original indices */
    int *cap_hit;       /* 1 where the rank cap decided the rank */

    /* coupling blocks B (k_a x k_b) and near blocks D (size_a x size_b) */
    int64_t *far_off;  double *B; int64_t B_len;
    int64_t *near_off; double *D; int64_t D_len;
} orc_h2;

/* ------------------------------------------------------------------------ */
/* Kernel function (Section 1: K(i,j) = kernel(x_i, x_j); the Gaussian is the
 * paper's example; the Laplace-type exp(-r/h) is a second smooth SPD kernel).
 * r^2 is summed in coordinate order, so kernel(x,y) == kernel(y,x) bitwise. */
static double orc_kernel(const orc_h2 *H, const double *x, const double *y)
{
    double r2 = 0.0;
    for (int t = 0; t < H->d; t++) {
        double df = x[t] - y[t];
        r2 += df * df;
    }
    if (H->kernel == 0)
        return exp(-r2 / (2.0 * H->h * H->h));
    return exp(-sqrt(r2) / H->h);
}

static double orc_kernel_idx(const orc_h2 *H, int64_t i, int64_t j)
{
    return orc_kernel(H, H->X + i * H->d, H->X + j * H->d);
}

/* ------------------------------------------------------------------------ */
/* Cluster tree (Section 3.1).  Reading: a perfect binary tree of depth
 * L = smallest L with ceil(N / 2^L) <= m, nodes numbered breadth-first (root 0,
 * children of i are 2i+1 and 2i+2).  A node is split along the coordinate of
 * largest bounding-box extent (lowest coordinate on a tie) at the median: the
 * points are ordered by (coordinate value, original index) and the left child
 * takes the first floor(n/2) of them. */
typedef struct { double v; int64_t idx; } orc_key;

static int orc_key_cmp(const void *a, const void *b)
{
    const orc_key *x = (const orc_key *)a, *y = (const orc_key *)b;
    if (x->v < y->v) return -1;
    if (x->v > y->v) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Two-means split of the points at tree positions [s, s + sz) (Section 3.1:
 * two-means partitioning for high-dimensional data).  Reading: the two means
 * of the node's points are found by Lloyd's iteration started from the point
 * farthest from the node's centroid and the point farthest from that one
 * (lowest original index on ties); a point goes to the second mean only if it
 * is strictly nearer to it.  The iteration stops when the assignment repeats
 * (the means are then a fixed point), when a group would be empty, or after
 * 100 rounds.  To keep the perfect tree (leaves of at most m points, all on
 * level L), the node is then cut at the median along the direction between
 * the two means: points ordered by (x . (c2 - c1), original index), the left
 * child takes the first floor(n/2).  c1 and c2 are kept in split_c. */
static double orc_d2(const double *x, const double *y, int d)
{
    double r2 = 0.0;
    for (int t = 0; t < d; t++) {
        double df = x[t] - y[t];
        r2 += df * df;
    }
    return r2;
}

static void orc_two_means_keys(orc_h2 *H, int node, int64_t s, int64_t sz, orc_key *keys)
{
    int d = H->d;
    double *cen = calloc((size_t)d, sizeof(double));
    double *c1 = H->split_c + (size_t)node * 2 * d, *c2 = c1 + d;
    for (int64_t p = s; p < s + sz; p++)
        for (int t = 0; t < d; t++) cen[t] += H->X[H->perm[p] * d + t];
    for (int t = 0; t < d; t++) cen[t] /= (double)sz;
    /* farthest point from the centroid, then farthest point from it */
    int64_t i1 = -1, i2 = -1;
    double best = -1.0;
    for (int64_t p = s; p < s + sz; p++) {
        int64_t i = H->perm[p];
        double r2 = orc_d2(H->X + i * d, cen, d);
        if (r2 > best || (r2 == best && i < i1)) { best = r2; i1 = i; }
    }
    best = -1.0;
    for (int64_t p = s; p < s + sz; p++) {
        int64_t i = H->perm[p];
        double r2 = orc_d2(H->X + i * d, H->X + i1 * d, d);
        if (r2 > best || (r2 == best && i < i2)) { best = r2; i2 = i; }
    }
    memcpy(c1, H->X + i1 * d, sizeof(double) * d);
    memcpy(c2, H->X + i2 * d, sizeof(double) * d);
    unsigned char *grp = malloc((size_t)sz), *prev = malloc((size_t)sz);
    for (int64_t p = 0; p < sz; p++) {
        const double *x = H->X + H->perm[s + p] * d;
        grp[p] = orc_d2(x, c2, d) < orc_d2(x, c1, d);
    }
    double *m1 = malloc(sizeof(double) * d), *m2 = malloc(sizeof(double) * d);
    for (int it = 0; it < 100; it++) {
        int64_t n1 = 0, n2 = 0;
        for (int t = 0; t < d; t++) m1[t] = m2[t] = 0.0;
        for (int64_t p = 0; p < sz; p++) {
            const double *x = H->X + H->perm[s + p] * d;
            double *m = grp[p] ? m2 : m1;
            for (int t = 0; t < d; t++) m[t] += x[t];
            if (grp[p]) n2++; else n1++;
        }
        if (n1 == 0 || n2 == 0) break;
        for (int t = 0; t < d; t++) { c1[t] = m1[t] / (double)n1; c2[t] = m2[t] / (double)n2; }
        memcpy(prev, grp, (size_t)sz);
        int changed = 0;
        for (int64_t p = 0; p < sz; p++) {
            const double *x = H->X + H->perm[s + p] * d;
            grp[p] = orc_d2(x, c2, d) < orc_d2(x, c1, d);
            changed |= grp[p] != prev[p];
        }
        if (!changed) break;
    }
    for (int64_t p = 0; p < sz; p++) {
        int64_t i = H->perm[s + p];
        double v = 0.0;
        for (int t = 0; t < d; t++) v += H->X[i * d + t] * (c2[t] - c1[t]);
        keys[p].idx = i;
        keys[p].v = v;
    }
    free(cen); free(grp); free(prev); free(m1); free(m2);
}

static void orc_build_tree(orc_h2 *H)
{
    int L = 0;
    while (((H->N + ((int64_t)1 << L) - 1) >> L) > H->m) L++;
    H->L = L;
    H->n_nodes = (int)(((int64_t)2 << L) - 1);
    int n = H->n_nodes;
    H->perm = malloc(sizeof(int64_t) * H->N);
    H->start = malloc(sizeof(int64_t) * n);
    H->size = malloc(sizeof(int64_t) * n);
    H->parent = malloc(sizeof(int) * n);
    H->left = malloc(sizeof(int) * n);
    H->right = malloc(sizeof(int) * n);
    H->level = malloc(sizeof(int) * n);
    H->split_c = calloc((size_t)n * 2 * H->d, sizeof(double));
    for (int64_t t = 0; t < H->N; t++) H->perm[t] = t;
    H->start[0] = 0;
    H->size[0] = H->N;
    H->parent[0] = -1;
    orc_key *keys = malloc(sizeof(orc_key) * H->N);
    for (int i = 0; i < n; i++) {
        int lev = 0;
        while (((int64_t)2 << lev) - 1 <= i) lev++;
        H->level[i] = lev;
        if (lev == L) { H->left[i] = H->right[i] = -1; continue; }
        int l = 2 * i + 1, r = 2 * i + 2;
        H->left[i] = l; H->right[i] = r;
        H->parent[l] = H->parent[r] = i;
        int64_t s = H->start[i], sz = H->size[i];
        if (H->part == 1) {
            orc_two_means_keys(H, i, s, sz, keys);
            qsort(keys, (size_t)sz, sizeof(orc_key), orc_key_cmp);
            for (int64_t p = 0; p < sz; p++) H->perm[s + p] = keys[p].idx;
            H->start[l] = s;        H->size[l] = sz / 2;
            H->start[r] = s + sz / 2; H->size[r] = sz - sz / 2;
            continue;
        }
        /* widest coordinate of the bounding box */
        int jstar = 0;
        double best = -1.0;
        for (int t = 0; t < H->d; t++) {
            double lo = INFINITY, hi = -INFINITY;
            for (int64_t p = s; p < s + sz; p++) {
                double v = H->X[H->perm[p] * H->d + t];
                if (v < lo) lo = v;
                if (v > hi) hi = v;
            }
            double ext = sz > 0 ? hi - lo : 0.0;
            if (ext > best) { best = ext; jstar = t; }
        }
        for (int64_t p = 0; p < sz; p++) {
            keys[p].idx = H->perm[s + p];
            keys[p].v = H->X[keys[p].idx * H->d + jstar];
        }
        qsort(keys, (size_t)sz, sizeof(orc_key), orc_key_cmp);
        for (int64_t p = 0; p < sz; p++) H->perm[s + p] = keys[p].idx;
        H->start[l] = s;        H->size[l] = sz / 2;
        H->start[r] = s + sz / 2; H->size[r] = sz - sz / 2;
    }
    free(keys);
}

/* Geometry for admissibility (Section 2.1).  Reading: dist(a,b) is the
 * distance between the centroids, diam(a) = 2 * max distance of a's points to
 * its centroid (the enclosing ball). */
static void orc_geometry(orc_h2 *H)
{
    int n = H->n_nodes, d = H->d;
    H->centroid = calloc((size_t)n * d, sizeof(double));
    H->radius = calloc((size_t)n, sizeof(double));
    for (int i = 0; i < n; i++) {
        double *c = H->centroid + (size_t)i * d;
        for (int64_t p = H->start[i]; p < H->start[i] + H->size[i]; p++)
            for (int t = 0; t < d; t++) c[t] += H->X[H->perm[p] * d + t];
        for (int t = 0; t < d; t++) c[t] /= (double)H->size[i];
        double rmax2 = 0.0;
        for (int64_t p = H->start[i]; p < H->start[i] + H->size[i]; p++) {
            double r2 = 0.0;
            for (int t = 0; t < d; t++) {
                double df = H->X[H->perm[p] * d + t] - c[t];
                r2 += df * df;
            }
            if (r2 > rmax2) rmax2 = r2;
        }
        H->radius[i] = sqrt(rmax2);
    }
}

static double orc_dist(const orc_h2 *H, int a, int b)
{
    double r2 = 0.0;
    for (int t = 0; t < H->d; t++) {
        double df = H->centroid[(size_t)a * H->d + t] - H->centroid[(size_t)b * H->d + t];
        r2 += df * df;
    }
    return sqrt(r2);
}

/* ------------------------------------------------------------------------ */
/* Interaction computation (Section 3.1; admissibility of Section 2.1).
 * Dual traversal from (root, root) over ordered pairs:
 *   a == b: a leaf gives a near pair, otherwise all four child pairs;
 *   admissible(a,b): far pair;  two leaves: near pair;
 *   otherwise split the non-leaf side(s).
 * Distance mode: admissible iff a != b and tau*dist > diam(a)+diam(b).
 * HSS mode (Section 4.1): admissible iff a != b, so Far(a) = {sibling}. */
typedef struct { int a, b; } orc_pair;
typedef struct { orc_pair *v; int64_t n, cap; } orc_pairs;

static void orc_push(orc_pairs *P, int a, int b)
{
    if (P->n == P->cap) {
        P->cap = P->cap ? 2 * P->cap : 1024;
        P->v = realloc(P->v, sizeof(orc_pair) * P->cap);
    }
    P->v[P->n].a = a; P->v[P->n].b = b; P->n++;
}

/* Far clusters / leaves ordered by centroid distance, ties by node number. */
typedef struct { double dist; int node; } orc_fc;

static int orc_fc_cmp(const void *x, const void *y)
{
    const orc_fc *p = (const orc_fc *)x, *q = (const orc_fc *)y;
    if (p->dist != q->dist) return p->dist < q->dist ? -1 : 1;
    return (p->node > q->node) - (p->node < q->node);
}

/* Budget admissibility (Section 4.1: the budget parameter of GOFMM, 0.03 for
 * H^2-b, 0 for HSS).  Reading: every leaf is near itself and the
 * floor(budget * #leaves) other leaves with the nearest centroids (ties by
 * node number); the relation is made symmetric.  Two distinct nodes are
 * admissible iff no leaf below one is near a leaf below the other.  Leaves
 * below a node of level l are the 2^(L-l) consecutive leaves starting at
 * (a + 1) 2^(L-l) - 1 (breadth-first numbering of a perfect tree). */
static void orc_budget_near(orc_h2 *H)
{
    int L = H->L, first = (1 << L) - 1, nl = 1 << L;
    H->leafnear = calloc((size_t)nl * nl, 1);
    int64_t kb = (int64_t)floor(H->budget * nl);
    if (kb > nl - 1) kb = nl - 1;
    orc_fc *fc = malloc(sizeof(orc_fc) * nl);
    for (int x = 0; x < nl; x++) {
        H->leafnear[(size_t)x * nl + x] = 1;
        int q = 0;
        for (int y = 0; y < nl; y++)
            if (y != x) { fc[q].node = first + y; fc[q].dist = orc_dist(H, first + x, first + y); q++; }
        qsort(fc, (size_t)q, sizeof(orc_fc), orc_fc_cmp);
        for (int64_t j = 0; j < kb; j++) {
            int y = fc[j].node - first;
            H->leafnear[(size_t)x * nl + y] = H->leafnear[(size_t)y * nl + x] = 1;
        }
    }
    free(fc);
}

static int orc_admissible(const orc_h2 *H, int a, int b)
{
    if (a == b) return 0;
    if (H->adm == 1) return 1;
    if (H->adm == 2) {
        int L = H->L, first = (1 << L) - 1, nl = 1 << L;
        int64_t ca = (int64_t)1 << (L - H->level[a]), cb = (int64_t)1 << (L - H->level[b]);
        int64_t fa = (a + 1) * ca - 1 - first, fb = (b + 1) * cb - 1 - first;
        for (int64_t x = fa; x < fa + ca; x++)
            for (int64_t y = fb; y < fb + cb; y++)
                if (H->leafnear[(size_t)x * nl + y]) return 0;
        return 1;
    }
    return H->tau * orc_dist(H, a, b) > 2.0 * H->radius[a] + 2.0 * H->radius[b];
}

static void orc_interact(const orc_h2 *H, int a, int b, orc_pairs *far, orc_pairs *near)
{
    int la = H->left[a] < 0, lb = H->left[b] < 0;
    if (a == b) {
        if (la) { orc_push(near, a, a); return; }
        int l = H->left[a], r = H->right[a];
        orc_interact(H, l, l, far, near); orc_interact(H, l, r, far, near);
        orc_interact(H, r, l, far, near); orc_interact(H, r, r, far, near);
        return;
    }
    if (orc_admissible(H, a, b)) { orc_push(far, a, b); return; }
    if (la && lb) { orc_push(near, a, b); return; }
    if (la) {
        orc_interact(H, a, H->left[b], far, near); orc_interact(H, a, H->right[b], far, near);
    } else if (lb) {
        orc_interact(H, H->left[a], b, far, near); orc_interact(H, H->right[a], b, far, near);
    } else {
        orc_interact(H, H->left[a], H->left[b], far, near);
        orc_interact(H, H->left[a], H->right[b], far, near);
        orc_interact(H, H->right[a], H->left[b], far, near);
        orc_interact(H, H->right[a], H->right[b], far, near);
    }
}

static int orc_pair_cmp(const void *x, const void *y)
{
    const orc_pair *p = (const orc_pair *)x, *q = (const orc_pair *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    return (p->b > q->b) - (p->b < q->b);
}

static void orc_to_csr(int n, orc_pairs *P, int64_t **ptr, int **col)
{
    if (P->n > 1) qsort(P->v, (size_t)P->n, sizeof(orc_pair), orc_pair_cmp);  /* v is NULL when empty */
    *ptr = calloc((size_t)n + 1, sizeof(int64_t));
    *col = malloc(sizeof(int) * (P->n ? P->n : 1));
    for (int64_t e = 0; e < P->n; e++) { (*ptr)[P->v[e].a + 1]++; (*col)[e] = P->v[e].b; }
    for (int i = 0; i < n; i++) (*ptr)[i + 1] += (*ptr)[i];
}

static void orc_interactions(orc_h2 *H)
{
    orc_pairs far = {0}, near = {0};
    if (H->adm == 2) orc_budget_near(H);
    orc_interact(H, 0, 0, &far, &near);
    H->n_far = far.n; H->n_near = near.n;
    orc_to_csr(H->n_nodes, &far, &H->far_ptr, &H->far_col);
    orc_to_csr(H->n_nodes, &near, &H->near_ptr, &H->near_col);
    free(far.v); free(near.v);
}

/* ------------------------------------------------------------------------ */
/* Pivoted-QR interpolative decomposition of one block (Section 3.1: ID gives
 * the low-rank generators; the rank is adapted to the block accuracy).
 *
 * A is mr x nc, column-major (A[j*mr + i]); it is overwritten.  Householder QR
 * with column pivoting, where the pivot is the column of largest remaining
 * 2-norm, recomputed exactly at every step (lowest index on ties).
 * Reading of the adaptive rank rule: stop at the first step j where
 * |R_jj| <= tol * |R_11| (so k = j), or at the cap min(rmax, mr, nc); k = 0 if
 * R_11 = 0.  Then Tcoef = R11^{-1} R12 (k x (nc-k)) by back substitution.
 * Outputs: *k, piv[0..nc-1] (column order), Tcoef (k x (nc-k), row-major),
 * rdiag[0..k] = |R_jj| for j < k, and rdiag[k] = the first rejected |R_jj|
 * (0 when the cap or the full width ended the loop).  Returns 1 when the cap
 * decided the rank. */
static int orc_pqr_id(double *A, int64_t mr, int nc, double tol, int rmax,
                      int *k_out, int *piv, double *Tcoef, double *rdiag, int par)
{
    /* par: run the loops over columns on the OpenMP team (each column's
     * arithmetic is the same either way) */
    int cap = rmax;
    if (cap > nc) cap = nc;
    if ((int64_t)cap > mr) cap = (int)mr;
    for (int j = 0; j < nc; j++) piv[j] = j;
    double *nrm2 = malloc(sizeof(double) * (nc ? nc : 1));
    double r11 = 0.0;
    int k = 0, capped = 0;
    double *v = malloc(sizeof(double) * (mr ? mr : 1));
    if (rdiag) rdiag[0] = 0.0;
    for (int j = 0;; j++) {
        if (j >= nc || (int64_t)j >= mr) { k = j; if (rdiag) rdiag[j] = 0.0; break; }
        /* exact remaining column norms */
#pragma omp parallel for if (par) schedule(static)
        for (int c = j; c < nc; c++) {
            double s = 0.0;
            const double *col = A + (size_t)c * mr;
            for (int64_t i = j; i < mr; i++) s += col[i] * col[i];
            nrm2[c] = s;
        }
        int p = j;
        double best = -1.0;
        for (int c = j; c < nc; c++)
            if (nrm2[c] > best) { best = nrm2[c]; p = c; }
        double rjj = sqrt(best);
        if (j == 0) r11 = rjj;
        if (rjj == 0.0 || (j > 0 && rjj <= tol * r11)) { k = j; if (rdiag) rdiag[j] = rjj; break; }
        if (j == cap) { k = j; capped = 1; if (rdiag) rdiag[j] = rjj; break; }
        if (rdiag) rdiag[j] = rjj;
        /* swap columns j and p */
        if (p != j) {
            double *a = A + (size_t)j * mr, *b = A + (size_t)p * mr;
            for (int64_t i = 0; i < mr; i++) { double t = a[i]; a[i] = b[i]; b[i] = t; }
            int t = piv[j]; piv[j] = piv[p]; piv[p] = t;
        }
        /* Householder reflector for A[j:, j]: H = I - 2 v v^T / (v^T v) */
        double *a = A + (size_t)j * mr;
        double alpha = a[j] >= 0.0 ? -rjj : rjj;
        double vtv = 0.0;
        for (int64_t i = j; i < mr; i++) v[i] = a[i];
        v[j] -= alpha;
        for (int64_t i = j; i < mr; i++) vtv += v[i] * v[i];
        a[j] = alpha;
        for (int64_t i = j + 1; i < mr; i++) a[i] = 0.0;
        if (vtv > 0.0) {
#pragma omp parallel for if (par) schedule(static)
            for (int c = j + 1; c < nc; c++) {
                double *col = A + (size_t)c * mr;
                double s = 0.0;
                for (int64_t i = j; i < mr; i++) s += v[i] * col[i];
                double f = 2.0 * s / vtv;
                for (int64_t i = j; i < mr; i++) col[i] -= f * v[i];
            }
        }
    }
    /* Tcoef = R11^{-1} R12, R stored in the upper triangle of A */
    int nr = nc - k;
#pragma omp parallel for if (par) schedule(static)
    for (int c = 0; c < nr; c++) {
        for (int i = k - 1; i >= 0; i--) {
            double s = A[(size_t)(k + c) * mr + i];
            for (int t = i + 1; t < k; t++) s -= A[(size_t)t * mr + i] * Tcoef[(size_t)t * nr + c];
            Tcoef[(size_t)i * nr + c] = s / A[(size_t)i * mr + i];
        }
    }
    free(nrm2);
    free(v);
    *k_out = k;
    return capped;
}

/* ------------------------------------------------------------------------ */
/* Counter-based generator for the row sample: the SplitMix64 finalizer
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014), applied as key = mix(mix(mix(seed) ^ node) ^ point). */
static uint64_t orc_mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

typedef struct { uint64_t key; int64_t pos; } orc_hk;


static int orc_hk_cmp(const void *x, const void *y)
{
    const orc_hk *p = (const orc_hk *)x, *q = (const orc_hk *)y;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return (p->pos > q->pos) - (p->pos < q->pos);
}

static int orc_i64_cmp(const void *x, const void *y)
{
    int64_t p = *(const int64_t *)x, q = *(const int64_t *)y;
    return (p > q) - (p < q);
}

/* Far field F(a) = points of every far partner of a or of its ancestors
 * (the rows the basis of a must represent).  Row sample R(a), a reading of the
 * sampling module of Section 3.1: all of F(a) if |F(a)| <= S; otherwise the
 * points of the far clusters nearest to a (by centroid distance, ties by node
 * number, in tree order) up to S/2 points, plus the S - (that count) remaining
 * far points with the smallest SplitMix64 keys.  Returns tree positions,
 * ascending, in *rows (malloc'd); the count is returned. */
static int64_t orc_row_sample(const orc_h2 *H, int a, int64_t **rows)
{
    int nfc = 0;
    for (int x = a; x >= 0; x = H->parent[x]) nfc += (int)(H->far_ptr[x + 1] - H->far_ptr[x]);
    orc_fc *fc = malloc(sizeof(orc_fc) * (nfc ? nfc : 1));
    int q = 0;
    int64_t total = 0;
    for (int x = a; x >= 0; x = H->parent[x])
        for (int64_t e = H->far_ptr[x]; e < H->far_ptr[x + 1]; e++) {
            fc[q].node = H->far_col[e];
            fc[q].dist = orc_dist(H, a, H->far_col[e]);
            total += H->size[H->far_col[e]];
            q++;
        }
    int64_t cnt = total <= H->S ? total : H->S;
    int64_t *out = malloc(sizeof(int64_t) * (cnt ? cnt : 1));
    int64_t o = 0;
    if (total <= H->S) {
        for (int i = 0; i < nfc; i++)
            for (int64_t p = H->start[fc[i].node]; p < H->start[fc[i].node] + H->size[fc[i].node]; p++)
                out[o++] = p;
    } else {
        qsort(fc, (size_t)nfc, sizeof(orc_fc), orc_fc_cmp);
        int64_t half = H->S / 2;
        int i = 0;
        int64_t part = 0; /* points already taken from cluster fc[i] */
        while (o < half) {
            int b = fc[i].node;
            out[o++] = H->start[b] + part;
            part++;
            if (part == H->size[b]) { i++; part = 0; }
        }
        /* remaining far points: rest of cluster i, then clusters i+1.. */
        int64_t nrest = total - o;
        orc_hk *hk = malloc(sizeof(orc_hk) * (nrest ? nrest : 1));
        int64_t r = 0;
        uint64_t base = orc_mix64(orc_mix64(H->seed) ^ (uint64_t)a);
        for (int j = i; j < nfc; j++) {
            int b = fc[j].node;
            for (int64_t p = (j == i ? part : 0); p < H->size[b]; p++) {
                int64_t pos = H->start[b] + p;
                hk[r].pos = pos;
                hk[r].key = orc_mix64(base ^ (uint64_t)H->perm[pos]);
                r++;
            }
        }
        qsort(hk, (size_t)nrest, sizeof(orc_hk), orc_hk_cmp);
        for (int64_t j = 0; o < H->S; j++) out[o++] = hk[j].pos;
        free(hk);
    }
    qsort(out, (size_t)o, sizeof(int64_t), orc_i64_cmp);
    free(fc);
    *rows = out;
    return o;
}

/* ------------------------------------------------------------------------ */
/* Nested-basis compression, bottom-up by level (Section 3.1; the V
 * generators of Section 2.1 are nested).  Reading of the ID form: symmetric
 * skeletonization.  For node a with candidate columns C(a) (its own points if
 * a leaf, the skeletons [s_l, s_r] of its children otherwise) and sampled far
 * rows R(a), the ID A(:, C) ~= A(:, s) * P of A = K(X[R], X[C]) gives the
 * skeleton s_a and the k x |C| interpolation matrix: P_a for a leaf, the
 * transfer T_a for an internal node. */
static void orc_compress(orc_h2 *H)
{
    int n = H->n_nodes;
    H->rank = calloc((size_t)n, sizeof(int));
    H->cap_hit = calloc((size_t)n, sizeof(int));
    double **bas = calloc((size_t)n, sizeof(double *));
    int64_t **sk = calloc((size_t)n, sizeof(int64_t *));
    int *ncol = calloc((size_t)n, sizeof(int));
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    for (int lev = H->L; lev >= 0; lev--) {
        int first = (1 << lev) - 1, last = (2 << lev) - 1;
        /* a level with fewer nodes than threads runs its nodes one after the
         * other, each with the column loops of its ID on all threads */
        int inner = last - first < nthreads;
#pragma omp parallel for schedule(dynamic, 1) if (!inner)
        for (int a = first; a < last; a++) {
            int leaf = H->left[a] < 0;
            int nc = leaf ? (int)H->size[a] : H->rank[H->left[a]] + H->rank[H->right[a]];
            int64_t *cand = malloc(sizeof(int64_t) * (nc ? nc : 1));
            if (leaf) {
                for (int j = 0; j < nc; j++) cand[j] = H->perm[H->start[a] + j];
            } else {
                int kl = H->rank[H->left[a]];
                for (int j = 0; j < kl; j++) cand[j] = sk[H->left[a]][j];
                for (int j = kl; j < nc; j++) cand[j] = sk[H->right[a]][j - kl];
            }
            ncol[a] = nc;
            int64_t *rows = NULL;
            int64_t mr = orc_row_sample(H, a, &rows);
            int k = 0;
            double *P = NULL;
            if (mr > 0 && nc > 0) {
                double *A = malloc(sizeof(double) * (size_t)mr * nc);
#pragma omp parallel for if (inner) schedule(static)
                for (int j = 0; j < nc; j++)
                    for (int64_t i = 0; i < mr; i++)
                        A[(size_t)j * mr + i] = orc_kernel_idx(H, H->perm[rows[i]], cand[j]);
                int *piv = malloc(sizeof(int) * nc);
                double *Tc = malloc(sizeof(double) * (size_t)nc * nc + 1);
                H->cap_hit[a] = orc_pqr_id(A, mr, nc, H->tol, H->rmax, &k, piv, Tc, NULL, inner);
                P = calloc((size_t)k * nc + 1, sizeof(double));
                int nr = nc - k;
                for (int i = 0; i < k; i++) {
                    P[(size_t)i * nc + piv[i]] = 1.0;
                    for (int c = 0; c < nr; c++) P[(size_t)i * nc + piv[k + c]] = Tc[(size_t)i * nr + c];
                }
                sk[a] = malloc(sizeof(int64_t) * (k ? k : 1));
                for (int i = 0; i < k; i++) sk[a][i] = cand[piv[i]];
                free(A); free(piv); free(Tc);
            }
            H->rank[a] = k;
            bas[a] = P;
            free(rows);
            free(cand);
        }
    }
    /* pack bases and skeletons in node order */
    H->basis_off = malloc(sizeof(int64_t) * n);
    H->skel_ptr = calloc((size_t)n + 1, sizeof(int64_t));
    int64_t off = 0;
    for (int a = 0; a < n; a++) {
        H->basis_off[a] = off;
        off += (int64_t)H->rank[a] * ncol[a];
        H->skel_ptr[a + 1] = H->skel_ptr[a] + H->rank[a];
    }
    H->basis_len = off;
    H->skel_len = H->skel_ptr[n];
    H->basis = malloc(sizeof(double) * (off ? off : 1));
    H->skel = malloc(sizeof(int64_t) * (H->skel_len ? H->skel_len : 1));
    for (int a = 0; a < n; a++) {
        if (H->rank[a] > 0) {
            memcpy(H->basis + H->basis_off[a], bas[a], sizeof(double) * (size_t)H->rank[a] * ncol[a]);
            memcpy(H->skel + H->skel_ptr[a], sk[a], sizeof(int64_t) * H->rank[a]);
        }
        free(bas[a]);
        free(sk[a]);
    }
    free(bas); free(sk); free(ncol);
}

/* Coupling blocks B_ab = K(X[s_a], X[s_b]) for far pairs and full near blocks
 * D_ab = K(X[I_a], X[I_b]) in tree order (Section 3.1: D is stored without
 * approximation). */
static void orc_blocks(orc_h2 *H)
{
    int n = H->n_nodes;
    H->far_off = malloc(sizeof(int64_t) * (H->n_far ? H->n_far : 1));
    H->near_off = malloc(sizeof(int64_t) * (H->n_near ? H->n_near : 1));
    int64_t off = 0;
    for (int a = 0; a < n; a++)
        for (int64_t e = H->far_ptr[a]; e < H->far_ptr[a + 1]; e++) {
            H->far_off[e] = off;
            off += (int64_t)H->rank[a] * H->rank[H->far_col[e]];
        }
    H->B_len = off;
    off = 0;
    for (int a = 0; a < n; a++)
        for (int64_t e = H->near_ptr[a]; e < H->near_ptr[a + 1]; e++) {
            H->near_off[e] = off;
            off += H->size[a] * H->size[H->near_col[e]];
        }
    H->D_len = off;
    H->B = malloc(sizeof(double) * (H->B_len ? H->B_len : 1));
    H->D = malloc(sizeof(double) * (H->D_len ? H->D_len : 1));
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a < n; a++) {
        for (int64_t e = H->far_ptr[a]; e < H->far_ptr[a + 1]; e++) {
            int b = H->far_col[e];
            double *blk = H->B + H->far_off[e];
            for (int i = 0; i < H->rank[a]; i++)
                for (int j = 0; j < H->rank[b]; j++)
                    blk[(size_t)i * H->rank[b] + j] =
                        orc_kernel_idx(H, H->skel[H->skel_ptr[a] + i], H->skel[H->skel_ptr[b] + j]);
        }
        for (int64_t e = H->near_ptr[a]; e < H->near_ptr[a + 1]; e++) {
            int b = H->near_col[e];
            double *blk = H->D + H->near_off[e];
            for (int64_t i = 0; i < H->size[a]; i++)
                for (int64_t j = 0; j < H->size[b]; j++)
                    blk[i * H->size[b] + j] =
                        orc_kernel_idx(H, H->perm[H->start[a] + i], H->perm[H->start[b] + j]);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Public entry points (called from the Python test wrapper via ctypes). */

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_free(orc_h2 *H)
{
    if (!H) return;
    void *ptrs[] = {H->X, H->perm, H->start, H->size, H->parent, H->left, H->right, H->level,
                    H->centroid, H->radius, H->far_ptr, H->far_col, H->near_ptr, H->near_col,
                    H->rank, H->basis_off, H->basis, H->skel_ptr, H->skel, H->cap_hit,
                    H->far_off, H->B, H->near_off, H->D, H->split_c, H->leafnear};
    for (size_t i = 0; i < sizeof(ptrs) / sizeof(ptrs[0]); i++) free(ptrs[i]);
    free(H);
}

/* Build the compressed representation from points X (N x d, original order).
 * part: 0 widest-coordinate median, 1 two-means; adm: 0 distance (tau),
 * 1 HSS, 2 budget (budget in [0, 1]). */
orc_h2 *orc_build_ex(const double *X, int64_t N, int d, int kernel, double h, int m, double tol,
                     int rmax, int adm, double tau, int64_t S, uint64_t seed, int part, double budget)
{
    if (N < 1 || d < 1 || m < 2 || rmax < 0 || S < 1 || h <= 0.0 || tol < 0.0) return NULL;
    if (part < 0 || part > 1 || adm < 0 || adm > 2 || !(budget >= 0.0 && budget <= 1.0)) return NULL;
    for (int64_t i = 0; i < N * d; i++)
        if (!isfinite(X[i])) return NULL;
    orc_h2 *H = calloc(1, sizeof(orc_h2));
    H->N = N; H->d = d; H->kernel = kernel; H->h = h; H->m = m; H->tol = tol; H->rmax = rmax;
    H->adm = adm; H->tau = tau; H->S = S; H->seed = seed; H->part = part; H->budget = budget;
    H->X = malloc(sizeof(double) * (size_t)N * d);
    memcpy(H->X, X, sizeof(double) * (size_t)N * d);
    orc_build_tree(H);
    orc_geometry(H);
    orc_interactions(H);
    orc_compress(H);
    orc_blocks(H);
    return H;
}

orc_h2 *orc_build(const double *X, int64_t N, int d, int kernel, double h, int m, double tol,
                  int rmax, int adm, double tau, int64_t S, uint64_t seed)
{
    return orc_build_ex(X, N, d, kernel, h, m, tol, rmax, adm, tau, S, seed, 0, 0.0);
}

/* The two means of a two-means split of node a (2d values: c1 then c2);
 * returns 0 when a was not split that way. */
int orc_split_centers(const orc_h2 *H, int a, double *out)
{
    if (a < 0 || a >= H->n_nodes || H->part != 1 || H->left[a] < 0) return 0;
    memcpy(out, H->split_c + (size_t)a * 2 * H->d, sizeof(double) * 2 * H->d);
    return 1;
}

/* Sizes: out[0..] = N, d, L, n_nodes, n_far, n_near, basis_len, B_len, D_len, skel_len. */
void orc_sizes(const orc_h2 *H, int64_t *out)
{
    out[0] = H->N; out[1] = H->d; out[2] = H->L; out[3] = H->n_nodes; out[4] = H->n_far;
    out[5] = H->n_near; out[6] = H->basis_len; out[7] = H->B_len; out[8] = H->D_len;
    out[9] = H->skel_len;
}

/* Pointers to the representation's arrays (owned by H, valid until orc_free),
 * in this order: perm, start, size, parent, left, right, level, rank, cap_hit,
 * basis_off, basis, far_ptr, far_col, far_off, B, near_ptr, near_col, near_off,
 * D, skel_ptr, skel, centroid, radius. */
void orc_ptrs(const orc_h2 *H, void **out)
{
    void *p[] = {H->perm, H->start, H->size, H->parent, H->left, H->right, H->level, H->rank,
                 H->cap_hit, H->basis_off, H->basis, H->far_ptr, H->far_col, H->far_off, H->B,
                 H->near_ptr, H->near_col, H->near_off, H->D, H->skel_ptr, H->skel, H->centroid,
                 H->radius};
    for (size_t i = 0; i < sizeof(p) / sizeof(p[0]); i++) out[i] = p[i];
}

/* ------------------------------------------------------------------------ */
/* Evaluation Y = K~ W (Section 2.1, "Evaluation"), as plain loops:
 *   Wt = W[perm]                                   (tree order)
 *   up, levels L..1:  What_a = P_a Wt[I_a]  (leaf) | T_a [What_l; What_r]
 *   far reduction:    Yhat_a = sum_{b in Far(a)} B_ab What_b
 *   down, levels 1..L-1: Yhat_l += T_a(:, :k_l)^T Yhat_a, Yhat_r += T_a(:, k_l:)^T Yhat_a
 *   leaves:           Yt[I_a] = P_a^T Yhat_a + sum_{b in Near(a)} D_ab Wt[I_b]
 *   Y[perm] = Yt
 * W and Y are N x Q row-major in the original point order.  Optional dumps
 * (NULL to skip), node-major in node order, k_a x Q per node:
 *   what: skeleton weights after the up pass; yhat: skeleton potentials after
 *   the down pass; ynear, yfar: N x Q tree-order near / far parts. */

/* C[i][q] += sum_t A(i,t) * Bm[t][q]; A(i,t) = A[i*lda+t] (trans=0) or A[t*lda+i]. */
static void orc_gemm_acc(int64_t rows, int64_t K, int64_t Q, const double *A, int64_t lda,
                         int trans, const double *Bm, int64_t ldb, double *C, int64_t ldc)
{
    for (int64_t i = 0; i < rows; i++)
        for (int64_t t = 0; t < K; t++) {
            double a = trans ? A[t * lda + i] : A[i * lda + t];
            const double *b = Bm + t * ldb;
            double *c = C + i * ldc;
            for (int64_t q = 0; q < Q; q++) c[q] += a * b[q];
        }
}

int orc_eval(const orc_h2 *H, const double *W, int64_t Q, double *Y, double *what_dump,
             double *yhat_dump, double *ynear_dump, double *yfar_dump)
{
    if (Q < 0) return ORC_ERR;
    int n = H->n_nodes;
    int64_t N = H->N;
    int64_t *woff = malloc(sizeof(int64_t) * (n + 1));
    woff[0] = 0;
    for (int a = 0; a < n; a++) woff[a + 1] = woff[a] + (int64_t)H->rank[a] * Q;
    double *What = calloc((size_t)woff[n] + 1, sizeof(double));
    double *Yhat = calloc((size_t)woff[n] + 1, sizeof(double));
    double *Wt = malloc(sizeof(double) * (size_t)N * Q + 1);
    double *Yn = calloc((size_t)N * Q + 1, sizeof(double));
    double *Yf = calloc((size_t)N * Q + 1, sizeof(double));
    for (int64_t t = 0; t < N; t++) memcpy(Wt + t * Q, W + H->perm[t] * Q, sizeof(double) * Q);

    /* bottom-up (V) pass */
    for (int lev = H->L; lev >= 1; lev--) {
        int first = (1 << lev) - 1, last = (2 << lev) - 1;
#pragma omp parallel for schedule(dynamic, 1)
        for (int a = first; a < last; a++) {
            int k = H->rank[a];
            if (k == 0) continue;
            const double *P = H->basis + H->basis_off[a];
            if (H->left[a] < 0) {
                orc_gemm_acc(k, H->size[a], Q, P, H->size[a], 0, Wt + H->start[a] * Q, Q,
                             What + woff[a], Q);
            } else {
                int l = H->left[a], r = H->right[a], kl = H->rank[l], kr = H->rank[r];
                orc_gemm_acc(k, kl, Q, P, kl + kr, 0, What + woff[l], Q, What + woff[a], Q);
                orc_gemm_acc(k, kr, Q, P + kl, kl + kr, 0, What + woff[r], Q, What + woff[a], Q);
            }
        }
    }
    /* far-field reduction (B) */
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = 0; a < n; a++)
        for (int64_t e = H->far_ptr[a]; e < H->far_ptr[a + 1]; e++) {
            int b = H->far_col[e];
            orc_gemm_acc(H->rank[a], H->rank[b], Q, H->B + H->far_off[e], H->rank[b], 0,
                         What + woff[b], Q, Yhat + woff[a], Q);
        }
    /* top-down (U) pass */
    for (int lev = 1; lev < H->L; lev++) {
        int first = (1 << lev) - 1, last = (2 << lev) - 1;
#pragma omp parallel for schedule(dynamic, 1)
        for (int a = first; a < last; a++) {
            int k = H->rank[a];
            if (k == 0 || H->left[a] < 0) continue;
            int l = H->left[a], r = H->right[a], kl = H->rank[l], kr = H->rank[r];
            const double *T = H->basis + H->basis_off[a];
            orc_gemm_acc(kl, k, Q, T, kl + kr, 1, Yhat + woff[a], Q, Yhat + woff[l], Q);
            orc_gemm_acc(kr, k, Q, T + kl, kl + kr, 1, Yhat + woff[a], Q, Yhat + woff[r], Q);
        }
    }
    /* leaves: far part P^T Yhat and near part sum D Wt */
    int first = (1 << H->L) - 1, last = (2 << H->L) - 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int a = first; a < last; a++) {
        if (H->rank[a] > 0)
            orc_gemm_acc(H->size[a], H->rank[a], Q, H->basis + H->basis_off[a], H->size[a], 1,
                         Yhat + woff[a], Q, Yf + H->start[a] * Q, Q);
        for (int64_t e = H->near_ptr[a]; e < H->near_ptr[a + 1]; e++) {
            int b = H->near_col[e];
            orc_gemm_acc(H->size[a], H->size[b], Q, H->D + H->near_off[e], H->size[b], 0,
                         Wt + H->start[b] * Q, Q, Yn + H->start[a] * Q, Q);
        }
    }
    for (int64_t t = 0; t < N; t++) {
        double *y = Y + H->perm[t] * Q;
        for (int64_t q = 0; q < Q; q++) y[q] = Yn[t * Q + q] + Yf[t * Q + q];
    }
    if (what_dump) memcpy(what_dump, What, sizeof(double) * woff[n]);
    if (yhat_dump) memcpy(yhat_dump, Yhat, sizeof(double) * woff[n]);
    if (ynear_dump) memcpy(ynear_dump, Yn, sizeof(double) * N * Q);
    if (yfar_dump) memcpy(yfar_dump, Yf, sizeof(double) * N * Q);
    free(woff); free(What); free(Yhat); free(Wt); free(Yn); free(Yf);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Dense K~ (N x N, original order) straight from its block definition:
 *   K~[I_a, I_b] = D_ab for near leaf pairs,
 *   K~[I_a, I_b] = Pc_a^T B_ab Pc_b for far pairs, where the composite basis
 *   Pc_a (k_a x |I_a|) is P_a for a leaf and T_a * blockdiag(Pc_l, Pc_r)
 *   otherwise.  Small N only. */
int orc_dense_ktilde(const orc_h2 *H, double *Kt)
{
    int n = H->n_nodes;
    double **Pc = calloc((size_t)n, sizeof(double *));
    for (int a = n - 1; a >= 0; a--) {
        int k = H->rank[a];
        int64_t sz = H->size[a];
        Pc[a] = calloc((size_t)k * sz + 1, sizeof(double));
        if (k == 0) continue;
        const double *P = H->basis + H->basis_off[a];
        if (H->left[a] < 0) {
            memcpy(Pc[a], P, sizeof(double) * (size_t)k * sz);
        } else {
            int l = H->left[a], r = H->right[a], kl = H->rank[l], kr = H->rank[r];
            int64_t sl = H->size[l];
            for (int i = 0; i < k; i++) {
                for (int t = 0; t < kl; t++)
                    for (int64_t j = 0; j < sl; j++)
                        Pc[a][i * sz + j] += P[i * (kl + kr) + t] * Pc[l][t * sl + j];
                for (int t = 0; t < kr; t++)
                    for (int64_t j = 0; j < H->size[r]; j++)
                        Pc[a][i * sz + sl + j] += P[i * (kl + kr) + kl + t] * Pc[r][t * H->size[r] + j];
            }
        }
    }
    int64_t N = H->N;
    for (int a = 0; a < n; a++) {
        for (int64_t e = H->near_ptr[a]; e < H->near_ptr[a + 1]; e++) {
            int b = H->near_col[e];
            const double *Dm = H->D + H->near_off[e];
            for (int64_t i = 0; i < H->size[a]; i++)
                for (int64_t j = 0; j < H->size[b]; j++)
                    Kt[H->perm[H->start[a] + i] * N + H->perm[H->start[b] + j]] = Dm[i * H->size[b] + j];
        }
        for (int64_t e = H->far_ptr[a]; e < H->far_ptr[a + 1]; e++) {
            int b = H->far_col[e];
            int ka = H->rank[a], kb = H->rank[b];
            const double *Bm = H->B + H->far_off[e];
            int64_t sa = H->size[a], sb = H->size[b];
            /* tmp = B_ab Pc_b (ka x sb), then Pc_a^T tmp */
            double *tmp = calloc((size_t)ka * sb + 1, sizeof(double));
            for (int i = 0; i < ka; i++)
                for (int t = 0; t < kb; t++)
                    for (int64_t j = 0; j < sb; j++) tmp[i * sb + j] += Bm[i * kb + t] * Pc[b][t * sb + j];
            for (int64_t i = 0; i < sa; i++)
                for (int64_t j = 0; j < sb; j++) {
                    double s = 0.0;
                    for (int t = 0; t < ka; t++) s += Pc[a][t * sa + i] * tmp[t * sb + j];
                    Kt[H->perm[H->start[a] + i] * N + H->perm[H->start[b] + j]] = s;
                }
            free(tmp);
        }
    }
    for (int a = 0; a < n; a++) free(Pc[a]);
    free(Pc);
    return ORC_OK;
}

/* Exact kernel rows (K W)[rows[i], :] = sum_j K(x_rows[i], x_j) W[j, :] in the
 * original order: the direct definition, used for sampled-row accuracy. */
void orc_exact_rows(const orc_h2 *H, const int64_t *rows, int64_t nrows, const double *W,
                    int64_t Q, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nrows; i++) {
        double *o = out + i * Q;
        for (int64_t q = 0; q < Q; q++) o[q] = 0.0;
        for (int64_t j = 0; j < H->N; j++) {
            double kv = orc_kernel_idx(H, rows[i], j);
            for (int64_t q = 0; q < Q; q++) o[q] += kv * W[j * Q + q];
        }
    }
}

/* A point set with its kernel and nothing else (no tree, no compression),
 * for orc_exact_rows on workloads whose compression the caller does not
 * need.  Free with orc_free. */
orc_h2 *orc_points(const double *X, int64_t N, int d, int kernel, double h)
{
    if (N < 1 || d < 1 || h <= 0.0) return NULL;
    orc_h2 *H = calloc(1, sizeof(orc_h2));
    H->N = N; H->d = d; H->kernel = kernel; H->h = h;
    H->X = malloc(sizeof(double) * (size_t)N * d);
    memcpy(H->X, X, sizeof(double) * (size_t)N * d);
    return H;
}

/* Row sample R(a) of node a (tree positions, ascending) into out (room for
 * cap entries); returns the sample's size, or -1 if a is out of range or the
 * sample does not fit.  Exposed so that the tests can pin the sampling rule. */
int64_t orc_row_sample_public(const orc_h2 *H, int a, int64_t *out, int64_t cap)
{
    if (a < 0 || a >= H->n_nodes) return -1;
    int64_t *rows = NULL;
    int64_t n = orc_row_sample(H, a, &rows);
    if (n > cap) { free(rows); return -1; }
    memcpy(out, rows, sizeof(int64_t) * (size_t)n);
    free(rows);
    return n;
}

/* Standalone pivoted-QR ID of a column-major mr x nc block, for pinning. */
int orc_pqr_id_public(double *A, int64_t mr, int nc, double tol, int rmax, int *k, int *piv,
                      double *Tcoef, double *rdiag)
{
    return orc_pqr_id(A, mr, nc, tol, rmax, k, piv, Tcoef, rdiag, 0);
}

/* ------------------------------------------------------------------------ */
/* Compressed-representation file "HMC1", version 1, little-endian, written
 * field by field: a 128-byte header, then perm, the node table, the bases,
 * the far CSR with B, the near CSR with D, and the skeletons. */
static int orc_put(FILE *f, const void *p, size_t bytes)
{
    return bytes == 0 || fwrite(p, 1, bytes, f) == bytes ? 0 : -1;
}

int orc_write(const orc_h2 *H, const char *path)
{
    FILE *f = fopen(path, "wb");
    if (!f) return ORC_ERR;
    unsigned char hdr[128];
    memset(hdr, 0, sizeof(hdr));
    uint32_t version = 1, flags = H->adm == 1 ? 1u : 0u;
    int32_t n = H->n_nodes, L = H->L, kern = H->kernel, rmax = H->rmax, m = H->m;
    int64_t d = H->d;
    memcpy(hdr + 0, "HMC1", 4);
    memcpy(hdr + 4, &version, 4);
    memcpy(hdr + 8, &H->N, 8);
    memcpy(hdr + 16, &d, 8);
    memcpy(hdr + 24, &n, 4);
    memcpy(hdr + 28, &L, 4);
    memcpy(hdr + 32, &flags, 4);
    memcpy(hdr + 36, &kern, 4);
    memcpy(hdr + 40, &H->h, 8);
    memcpy(hdr + 48, &H->tol, 8);
    memcpy(hdr + 56, &H->tau, 8);
    memcpy(hdr + 64, &rmax, 4);
    memcpy(hdr + 68, &m, 4);
    memcpy(hdr + 72, &H->n_far, 8);
    memcpy(hdr + 80, &H->n_near, 8);
    memcpy(hdr + 88, &H->basis_len, 8);
    memcpy(hdr + 96, &H->B_len, 8);
    memcpy(hdr + 104, &H->D_len, 8);
    memcpy(hdr + 112, &H->skel_len, 8);
    int rc = orc_put(f, hdr, sizeof(hdr));
    rc |= orc_put(f, H->perm, sizeof(int64_t) * H->N);
    rc |= orc_put(f, H->start, sizeof(int64_t) * n);
    rc |= orc_put(f, H->size, sizeof(int64_t) * n);
    rc |= orc_put(f, H->parent, sizeof(int) * n);
    rc |= orc_put(f, H->left, sizeof(int) * n);
    rc |= orc_put(f, H->right, sizeof(int) * n);
    rc |= orc_put(f, H->level, sizeof(int) * n);
    rc |= orc_put(f, H->rank, sizeof(int) * n);
    rc |= orc_put(f, H->basis_off, sizeof(int64_t) * n);
    rc |= orc_put(f, H->basis, sizeof(double) * H->basis_len);
    rc |= orc_put(f, H->far_ptr, sizeof(int64_t) * (n + 1));
    rc |= orc_put(f, H->far_col, sizeof(int) * H->n_far);
    rc |= orc_put(f, H->far_off, sizeof(int64_t) * H->n_far);
    rc |= orc_put(f, H->B, sizeof(double) * H->B_len);
    rc |= orc_put(f, H->near_ptr, sizeof(int64_t) * (n + 1));
    rc |= orc_put(f, H->near_col, sizeof(int) * H->n_near);
    rc |= orc_put(f, H->near_off, sizeof(int64_t) * H->n_near);
    rc |= orc_put(f, H->D, sizeof(double) * H->D_len);
    rc |= orc_put(f, H->skel_ptr, sizeof(int64_t) * (n + 1));
    rc |= orc_put(f, H->skel, sizeof(int64_t) * H->skel_len);
    if (fclose(f) != 0) rc = -1;
    return rc ? ORC_ERR : ORC_OK;
}
