/*
 * Oracle: octree, interaction lists and a reference fast multipole method.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Follows Sec. 2.3 of the paper: expansions in spherical harmonics
 * Y_n^m = sqrt((n-|m|)!/(n+|m|)!) P_n^|m|(cos theta) e^{i m phi} (eq. FMM_coul,
 * multipole coefficients M_n^m = sum q rho^n Y_n^{-m}; eq. FMM_local, local
 * coefficients L_n^m with phi = sum L_n^m Y_n^m rho^n), truncated at degree p;
 * the smallest enclosing cube divided recursively into octants, a box being
 * divided only when it holds more than `leaf_size` ions (the adaptive rule
 * of the "Algorithm" subsection); an upward pass (multipoles at the leaves,
 * merged into parents), a downward pass (multipole-to-local conversion of
 * well-separated boxes from level 2 down, parent local expansions shifted to
 * children) and the remaining near interactions by direct summation.
 *
 * The three translation operators are the classical addition theorems for
 * this normalisation (Greengard & Rokhlin; Cheng, Greengard & Rokhlin 1999,
 * which the paper cites for the details), written with
 * A_n^m = (-1)^n / sqrt((n-m)!(n+m)!) and powers of i.
 *
 * Adaptive interaction lists (the paper defers these to Cheng et al.):
 *   V(B): same-level boxes whose parent touches B's parent but which do not
 *         touch B (multipole-to-local);
 *   near(T), T a leaf: every leaf L for which the ancestors of T and L at
 *         level min(level T, level L) touch (direct summation).  This puts
 *         the adaptive W and X interactions in the direct sum as well.
 * Two boxes "touch" when their closed cubes share at least one point.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define OR_MAXLEV 16

/* ---------------------------------------------------------------- keys */

/* Root cube and Morton keys.  lo/hi are the per-axis extremes, W the largest
 * extent, the cube is centred on the bounding box: o = (lo + hi)/2 - W/2.
 * Each coordinate is quantised to 16 bits, floor((x - o) * 2^16 / W) clamped
 * to [0, 2^16 - 1], and the three integers are bit-interleaved with x in
 * the most significant position of each triple (48-bit keys; 16 levels).  Built with
 * -ffp-contract=off so no multiply-add is fused. */
void or_root_cube(int n, const double *pos, double lo_out[3], double *W_out)
{
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        lo[d] = n > 0 ? pos[d] : 0.0;
        hi[d] = lo[d];
    }
    for (int i = 0; i < n; ++i)
        for (int d = 0; d < 3; ++d) {
            double v = pos[3 * i + d];
            if (v < lo[d]) lo[d] = v;
            if (v > hi[d]) hi[d] = v;
        }
    double W = 0.0;
    for (int d = 0; d < 3; ++d)
        if (hi[d] - lo[d] > W) W = hi[d] - lo[d];
    if (W == 0.0) W = 1e-9;
    for (int d = 0; d < 3; ++d) {
        double c = 0.5 * (lo[d] + hi[d]);
        lo_out[d] = c - 0.5 * W;
    }
    *W_out = W;
}

static uint64_t or_spread3(uint32_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < OR_MAXLEV; ++b)
        if (v & (1u << b)) r |= (uint64_t)1 << (3 * b);
    return r;
}

void or_morton_keys(int n, const double *pos, uint64_t *keys, double root_out[4])
{
    double o[3], W;
    or_root_cube(n, pos, o, &W);
    double S = 65536.0 / W;
    for (int i = 0; i < n; ++i) {
        uint32_t k[3];
        for (int d = 0; d < 3; ++d) {
            double f = floor((pos[3 * i + d] - o[d]) * S);
            if (f < 0.0) f = 0.0;
            if (f > 65535.0) f = 65535.0;
            k[d] = (uint32_t)f;
        }
        keys[i] = (or_spread3(k[0]) << 2) | (or_spread3(k[1]) << 1) | or_spread3(k[2]);
    }
    if (root_out) {
        root_out[0] = o[0];
        root_out[1] = o[1];
        root_out[2] = o[2];
        root_out[3] = W;
    }
}

/* ---------------------------------------------------------------- tree */

static const uint64_t *g_sort_keys;
static int or_cmp_key_id(const void *a, const void *b)
{
    int32_t i = *(const int32_t *)a, j = *(const int32_t *)b;
    uint64_t ki = g_sort_keys[i], kj = g_sort_keys[j];
    if (ki < kj) return -1;
    if (ki > kj) return 1;
    return (i > j) - (i < j);
}

typedef struct {
    int cap, n;
    int32_t *level, *parent, *ib, *ie, *ix, *iy, *iz;
} or_boxvec;

static int or_boxvec_push(or_boxvec *v, int level, int parent, int ib, int ie, int ix, int iy, int iz)
{
    if (v->n == v->cap) {
        int nc = v->cap ? 2 * v->cap : 64;
        int32_t **arrs[7] = {&v->level, &v->parent, &v->ib, &v->ie, &v->ix, &v->iy, &v->iz};
        for (int a = 0; a < 7; ++a) {
            int32_t *p = (int32_t *)realloc(*arrs[a], sizeof(int32_t) * (size_t)nc);
            if (!p) return -1;
            *arrs[a] = p;
        }
        v->cap = nc;
    }
    int k = v->n++;
    v->level[k] = level; v->parent[k] = parent; v->ib[k] = ib; v->ie[k] = ie;
    v->ix[k] = ix; v->iy[k] = iy; v->iz[k] = iz;
    return k;
}

/* Do boxes a and b touch (closed cubes intersect)?  Compare at the finer level. */
static int or_touch(const or_tree *t, int a, int b)
{
    int la = t->level[a], lb = t->level[b];
    if (la > lb) { int tmp = a; a = b; b = tmp; tmp = la; la = lb; lb = tmp; }
    int64_t s = (int64_t)1 << (lb - la);
    int64_t ca[3] = {t->ix[a], t->iy[a], t->iz[a]};
    int64_t cb[3] = {t->ix[b], t->iy[b], t->iz[b]};
    for (int d = 0; d < 3; ++d) {
        /* a covers [ca*s, (ca+1)*s], b covers [cb, cb+1] in level-lb units */
        if (cb[d] + 1 < ca[d] * s) return 0;
        if (cb[d] > (ca[d] + 1) * s) return 0;
    }
    return 1;
}

static int or_ancestor_at(const or_tree *t, int b, int level)
{
    while (t->level[b] > level) b = t->parent[b];
    return b;
}

void or_tree_free(or_tree *t)
{
    if (!t) return;
    free(t->key); free(t->perm);
    free(t->level); free(t->parent); free(t->child_first); free(t->nchild);
    free(t->ion_begin); free(t->ion_end); free(t->ix); free(t->iy); free(t->iz);
    free(t->is_leaf); free(t->v_off); free(t->v_src); free(t->near_off); free(t->near_src);
    free(t);
}

/* Build the octree and both interaction lists for n ions (pos: n x 3). */
or_tree *or_tree_build(int n, const double *pos, int leaf_size)
{
    if (n < 1 || leaf_size < 1) return NULL;
    or_tree *t = (or_tree *)calloc(1, sizeof(or_tree));
    t->n = n;
    t->key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    t->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double root[4];
    or_morton_keys(n, pos, t->key, root);
    t->lo[0] = root[0]; t->lo[1] = root[1]; t->lo[2] = root[2]; t->W = root[3];
    for (int i = 0; i < n; ++i) t->perm[i] = i;
    g_sort_keys = t->key;
    qsort(t->perm, (size_t)n, sizeof(int32_t), or_cmp_key_id);

    /* Breadth-first: a level's boxes are emitted parent by parent in octant
     * order, so each level ends up in ascending Morton-prefix order. */
    or_boxvec bv = {0};
    or_boxvec_push(&bv, 0, -1, 0, n, 0, 0, 0);
    int lev_begin = 0, lev_end = 1, nlev = 1;
    for (int l = 0; l < OR_MAXLEV && lev_begin < lev_end; ++l) {
        for (int b = lev_begin; b < lev_end; ++b) {
            int ib = bv.ib[b], ie = bv.ie[b];
            if (ie - ib <= leaf_size) continue;
            int shift = 3 * (OR_MAXLEV - 1 - l);
            int k = ib;
            for (int oct = 0; oct < 8; ++oct) {
                int k0 = k;
                while (k < ie && (int)((t->key[t->perm[k]] >> shift) & 7u) == oct) ++k;
                if (k > k0) {
                    int cx = 2 * bv.ix[b] + ((oct >> 2) & 1);
                    int cy = 2 * bv.iy[b] + ((oct >> 1) & 1);
                    int cz = 2 * bv.iz[b] + (oct & 1);
                    or_boxvec_push(&bv, l + 1, b, k0, k, cx, cy, cz);
                }
            }
        }
        lev_begin = lev_end;
        lev_end = bv.n;
        if (lev_end > lev_begin) nlev = l + 2;
    }
    int nb = bv.n;
    t->nbox = nb;
    t->nlevels = nlev;
    t->level = bv.level; t->parent = bv.parent; t->ion_begin = bv.ib; t->ion_end = bv.ie;
    t->ix = bv.ix; t->iy = bv.iy; t->iz = bv.iz;
    t->child_first = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    t->nchild = (int32_t *)calloc((size_t)nb, sizeof(int32_t));
    t->is_leaf = (uint8_t *)malloc((size_t)nb);
    for (int b = 0; b < nb; ++b) t->child_first[b] = -1;
    for (int b = 1; b < nb; ++b) {
        int pa = t->parent[b];
        if (t->child_first[pa] < 0) t->child_first[pa] = b;
        t->nchild[pa]++;
    }
    for (int b = 0; b < nb; ++b) t->is_leaf[b] = t->nchild[b] == 0;

    /* V lists, by their definition: O(boxes^2) per level. */
    t->v_off = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nb + 1));
    int vcap = 1024, vn = 0;
    t->v_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)vcap);
    for (int b = 0; b < nb; ++b) {
        t->v_off[b] = vn;
        if (t->level[b] < 2) continue;
        for (int c = 0; c < nb; ++c) {
            if (t->level[c] != t->level[b] || c == b) continue;
            if (!or_touch(t, t->parent[b], t->parent[c])) continue;
            if (or_touch(t, b, c)) continue;
            if (vn == vcap) { vcap *= 2; t->v_src = (int32_t *)realloc(t->v_src, sizeof(int32_t) * (size_t)vcap); }
            t->v_src[vn++] = c;
        }
    }
    t->v_off[nb] = vn;

    /* near lists of the leaves, by their definition: O(leaves^2). */
    t->near_off = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nb + 1));
    int ncap = 1024, nn = 0;
    t->near_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)ncap);
    for (int b = 0; b < nb; ++b) {
        t->near_off[b] = nn;
        if (!t->is_leaf[b]) continue;
        for (int c = 0; c < nb; ++c) {
            if (!t->is_leaf[c]) continue;
            int m = t->level[b] < t->level[c] ? t->level[b] : t->level[c];
            if (!or_touch(t, or_ancestor_at(t, b, m), or_ancestor_at(t, c, m))) continue;
            if (nn == ncap) { ncap *= 2; t->near_src = (int32_t *)realloc(t->near_src, sizeof(int32_t) * (size_t)ncap); }
            t->near_src[nn++] = c;
        }
    }
    t->near_off[nb] = nn;
    return t;
}

/* Sizes: nbox, nlevels, total V entries, total near entries. */
void or_tree_sizes(const or_tree *t, int64_t out[4])
{
    out[0] = t->nbox;
    out[1] = t->nlevels;
    out[2] = t->v_off[t->nbox];
    out[3] = t->near_off[t->nbox];
}

/* Copy the tree out.  Any pointer may be NULL. root: lower corner + side. */
void or_tree_export(const or_tree *t, uint64_t *key, int32_t *perm, int32_t *level, int32_t *parent,
                    int32_t *ion_begin, int32_t *ion_end, int32_t *coords /* nbox x 3 */, uint8_t *is_leaf,
                    int32_t *v_off, int32_t *v_src, int32_t *near_off, int32_t *near_src, double *root)
{
    int n = t->n, nb = t->nbox;
    if (key) memcpy(key, t->key, sizeof(uint64_t) * (size_t)n);
    if (perm) memcpy(perm, t->perm, sizeof(int32_t) * (size_t)n);
    if (level) memcpy(level, t->level, sizeof(int32_t) * (size_t)nb);
    if (parent) memcpy(parent, t->parent, sizeof(int32_t) * (size_t)nb);
    if (ion_begin) memcpy(ion_begin, t->ion_begin, sizeof(int32_t) * (size_t)nb);
    if (ion_end) memcpy(ion_end, t->ion_end, sizeof(int32_t) * (size_t)nb);
    if (coords)
        for (int b = 0; b < nb; ++b) {
            coords[3 * b] = t->ix[b]; coords[3 * b + 1] = t->iy[b]; coords[3 * b + 2] = t->iz[b];
        }
    if (is_leaf) memcpy(is_leaf, t->is_leaf, (size_t)nb);
    if (v_off) memcpy(v_off, t->v_off, sizeof(int32_t) * (size_t)(nb + 1));
    if (v_src) memcpy(v_src, t->v_src, sizeof(int32_t) * (size_t)t->v_off[nb]);
    if (near_off) memcpy(near_off, t->near_off, sizeof(int32_t) * (size_t)(nb + 1));
    if (near_src) memcpy(near_src, t->near_src, sizeof(int32_t) * (size_t)t->near_off[nb]);
    if (root) { root[0] = t->lo[0]; root[1] = t->lo[1]; root[2] = t->lo[2]; root[3] = t->W; }
}

/* Second, independent construction of the same interactions: a dual
 * traversal from (root, root).  Same-level pairs that do not touch go to
 * multipole-to-local; pairs at different levels that do not touch, and
 * touching leaf pairs, go to direct summation (expanded to leaf pairs);
 * a touching pair with a non-leaf side is refined on its non-leaf side(s).
 * Emits (target, source) pairs; the caller compares them as sets.
 * Returns the number of pairs written (counts only if the buffers are NULL). */
typedef struct {
    const or_tree *t;
    int64_t nv, nn;
    int32_t *vp, *np; /* pairs, 2 ints each */
} or_dual_ctx;

static void or_dual_emit_near(or_dual_ctx *cx, int a, int b)
{
    /* expand both sides to their leaves */
    const or_tree *t = cx->t;
    if (!t->is_leaf[a]) {
        for (int c = 0; c < t->nchild[a]; ++c) or_dual_emit_near(cx, t->child_first[a] + c, b);
        return;
    }
    if (!t->is_leaf[b]) {
        for (int c = 0; c < t->nchild[b]; ++c) or_dual_emit_near(cx, a, t->child_first[b] + c);
        return;
    }
    if (cx->np) { cx->np[2 * cx->nn] = a; cx->np[2 * cx->nn + 1] = b; }
    cx->nn++;
}

static void or_dual(or_dual_ctx *cx, int a, int b)
{
    const or_tree *t = cx->t;
    int touch = or_touch(t, a, b);
    if (!touch) {
        if (t->level[a] == t->level[b]) {
            if (cx->vp) { cx->vp[2 * cx->nv] = a; cx->vp[2 * cx->nv + 1] = b; }
            cx->nv++;
        } else {
            or_dual_emit_near(cx, a, b);
        }
        return;
    }
    int la = t->is_leaf[a], lb = t->is_leaf[b];
    if (la && lb) { or_dual_emit_near(cx, a, b); return; }
    if (!la && !lb) {
        for (int i = 0; i < t->nchild[a]; ++i)
            for (int j = 0; j < t->nchild[b]; ++j) or_dual(cx, t->child_first[a] + i, t->child_first[b] + j);
    } else if (!la) {
        for (int i = 0; i < t->nchild[a]; ++i) or_dual(cx, t->child_first[a] + i, b);
    } else {
        for (int j = 0; j < t->nchild[b]; ++j) or_dual(cx, a, t->child_first[b] + j);
    }
}

void or_dual_traversal(const or_tree *t, int64_t counts[2], int32_t *v_pairs, int32_t *near_pairs)
{
    or_dual_ctx cx = {t, 0, 0, v_pairs, near_pairs};
    or_dual(&cx, 0, 0);
    counts[0] = cx.nv;
    counts[1] = cx.nn;
}

/* ------------------------------------------------------- harmonics */

#define IDX(n, m) ((n) * (n) + (n) + (m))

static double complex or_ipow(int e)
{
    int r = ((e % 4) + 4) % 4;
    return r == 0 ? 1.0 : r == 1 ? I : r == 2 ? -1.0 : -I;
}

/* A_n^m = (-1)^n / sqrt((n-m)!(n+m)!) for n <= nmax, in A[IDX(n,m)]. */
static double *or_A_table(int nmax)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)(nmax + 1) * (size_t)(nmax + 1));
    for (int n = 0; n <= nmax; ++n)
        for (int m = -n; m <= n; ++m) {
            double f = 1.0;
            for (int k = 2; k <= n - m; ++k) f *= k;
            for (int k = 2; k <= n + m; ++k) f *= k;
            A[IDX(n, m)] = ((n & 1) ? -1.0 : 1.0) / sqrt(f);
        }
    return A;
}
#define or_A(n, m) A[IDX((n), (m))]

/* Y_n^m(theta, phi) for 0 <= n <= nmax, all m, in Y[IDX(n,m)]:
 * sqrt((n-|m|)!/(n+|m|)!) P_n^|m|(cos theta) e^{i m phi}, P without the
 * Condon-Shortley sign.  Recurrences: P_m^m = (2m-1)!! sin^m,
 * P_{m+1}^m = (2m+1) cos P_m^m, (n-m) P_n^m = (2n-1) cos P_{n-1}^m - (n+m-1) P_{n-2}^m. */
static void or_ylm(int nmax, double ct, double phi, double complex *Y)
{
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double *P = (double *)malloc(sizeof(double) * (size_t)(nmax + 1) * (size_t)(nmax + 1));
#define PI_(n, m) P[(n) * (nmax + 1) + (m)]
    double pmm = 1.0;
    for (int m = 0; m <= nmax; ++m) {
        if (m > 0) pmm *= (2.0 * m - 1.0) * st;
        PI_(m, m) = pmm;
        if (m + 1 <= nmax) PI_(m + 1, m) = (2.0 * m + 1.0) * ct * pmm;
        for (int n = m + 2; n <= nmax; ++n)
            PI_(n, m) = ((2.0 * n - 1.0) * ct * PI_(n - 1, m) - (n + m - 1.0) * PI_(n - 2, m)) / (double)(n - m);
    }
    for (int n = 0; n <= nmax; ++n)
        for (int m = 0; m <= n; ++m) {
            double ratio = 1.0; /* (n-m)!/(n+m)! */
            for (int k = n - m + 1; k <= n + m; ++k) ratio /= (double)k;
            double v = sqrt(ratio) * PI_(n, m);
            Y[IDX(n, m)] = v * cexp(I * (double)m * phi);
            Y[IDX(n, -m)] = v * cexp(-I * (double)m * phi);
        }
#undef PI_
    free(P);
}

static void or_sph(const double v[3], double *rho, double *ct, double *phi)
{
    double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    *rho = r;
    if (r == 0.0) { *ct = 1.0; *phi = 0.0; return; }
    *ct = v[2] / r;
    *phi = atan2(v[1], v[0]);
}

/* P2M (eq. FMM_coul): M_n^m = sum_i q_i rho_i^n Y_n^{-m}(theta_i, phi_i),
 * about `center`; M has (p+1)^2 complex entries. */
void or_p2m(int n, const double *pos, const double *q, const double center[3], int p, double complex *M)
{
    int K = (p + 1) * (p + 1);
    double complex *Y = (double complex *)malloc(sizeof(double complex) * (size_t)K);
    for (int k = 0; k < K; ++k) M[k] = 0.0;
    for (int i = 0; i < n; ++i) {
        double d[3] = {pos[3 * i] - center[0], pos[3 * i + 1] - center[1], pos[3 * i + 2] - center[2]};
        double rho, ct, ph;
        or_sph(d, &rho, &ct, &ph);
        or_ylm(p, ct, ph, Y);
        double rn = 1.0;
        for (int nn = 0; nn <= p; ++nn) {
            for (int m = -nn; m <= nn; ++m) M[IDX(nn, m)] += q[i] * rn * Y[IDX(nn, -m)];
            rn *= rho;
        }
    }
    free(Y);
}

/* Potential of a multipole expansion about c at x: sum M_n^m Y_n^m / rho^{n+1}. */
double or_eval_me(int p, const double complex *M, const double c[3], const double x[3])
{
    double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
    double rho, ct, ph;
    or_sph(d, &rho, &ct, &ph);
    int K = (p + 1) * (p + 1);
    double complex *Y = (double complex *)malloc(sizeof(double complex) * (size_t)K);
    or_ylm(p, ct, ph, Y);
    double complex s = 0.0;
    double rinv = 1.0 / rho, rp = rinv;
    for (int n = 0; n <= p; ++n) {
        for (int m = -n; m <= n; ++m) s += M[IDX(n, m)] * Y[IDX(n, m)] * rp;
        rp *= rinv;
    }
    free(Y);
    return creal(s);
}

/* M2M: expansion about c_old re-expanded about c_new; (rho, alpha, beta) is
 * c_old - c_new.  Out[j,k] = sum_{n<=j} sum_m M_old[j-n, k-m]
 *   i^{|k|-|m|-|k-m|} A_n^m A_{j-n}^{k-m} rho^n Y_n^{-m}(alpha, beta) / A_j^k. */
void or_m2m(int p, const double complex *M, const double c_old[3], const double c_new[3], double complex *Out)
{
    double d[3] = {c_old[0] - c_new[0], c_old[1] - c_new[1], c_old[2] - c_new[2]};
    double rho, ct, ph;
    or_sph(d, &rho, &ct, &ph);
    int K = (p + 1) * (p + 1);
    double complex *Y = (double complex *)malloc(sizeof(double complex) * (size_t)K);
    or_ylm(p, ct, ph, Y);
    double *A = or_A_table(p);
    for (int j = 0; j <= p; ++j)
        for (int k = -j; k <= j; ++k) {
            double complex s = 0.0;
            for (int n = 0; n <= j; ++n) {
                double rn = pow(rho, n);
                for (int m = -n; m <= n; ++m) {
                    if (abs(k - m) > j - n) continue;
                    s += M[IDX(j - n, k - m)] * or_ipow(abs(k) - abs(m) - abs(k - m)) * or_A(n, m) *
                         or_A(j - n, k - m) * rn * Y[IDX(n, -m)] / or_A(j, k);
                }
            }
            Out[IDX(j, k)] = s;
        }
    free(A);
    free(Y);
}

/* M2L (eq. FMM_local): multipole about c_src converted to a local expansion
 * about c_tgt; (rho, alpha, beta) is c_src - c_tgt.  L[j,k] = sum_{n,m} M[n,m]
 *   i^{|k-m|-|k|-|m|} A_n^m A_j^k Y_{j+n}^{m-k}(alpha,beta) / ((-1)^n A_{j+n}^{m-k} rho^{j+n+1}).
 * The result is ADDED to L. */
void or_m2l_add(int p, const double complex *M, const double c_src[3], const double c_tgt[3], double complex *L)
{
    double d[3] = {c_src[0] - c_tgt[0], c_src[1] - c_tgt[1], c_src[2] - c_tgt[2]};
    double rho, ct, ph;
    or_sph(d, &rho, &ct, &ph);
    int K2 = (2 * p + 1) * (2 * p + 1);
    double complex *Y = (double complex *)malloc(sizeof(double complex) * (size_t)K2);
    or_ylm(2 * p, ct, ph, Y);
    double *A = or_A_table(2 * p);
    for (int j = 0; j <= p; ++j)
        for (int k = -j; k <= j; ++k) {
            double complex s = 0.0;
            for (int n = 0; n <= p; ++n) {
                double sg = (n & 1) ? -1.0 : 1.0;
                double rp = pow(rho, j + n + 1);
                for (int m = -n; m <= n; ++m)
                    s += M[IDX(n, m)] * or_ipow(abs(k - m) - abs(k) - abs(m)) * or_A(n, m) * or_A(j, k) *
                         Y[IDX(j + n, m - k)] / (sg * or_A(j + n, m - k) * rp);
            }
            L[IDX(j, k)] += s;
        }
    free(A);
    free(Y);
}

/* L2L: local expansion about c_old shifted to c_new; (rho, alpha, beta) is
 * c_new - c_old.  Out[j,k] = sum_{n>=j} sum_m L[n,m]
 *   i^{|m|-|m-k|-|k|} A_{n-j}^{m-k} A_j^k Y_{n-j}^{m-k}(alpha,beta) rho^{n-j} / A_n^m.
 * Only degrees j <= jmax are produced. */
static void or_l2l_upto(int p, int jmax, const double complex *L, const double c_old[3], const double c_new[3],
                        double complex *Out)
{
    double d[3] = {c_new[0] - c_old[0], c_new[1] - c_old[1], c_new[2] - c_old[2]};
    double rho, ct, ph;
    or_sph(d, &rho, &ct, &ph);
    int K = (p + 1) * (p + 1);
    double complex *Y = (double complex *)malloc(sizeof(double complex) * (size_t)K);
    or_ylm(p, ct, ph, Y);
    double *A = or_A_table(p);
    for (int j = 0; j <= jmax; ++j)
        for (int k = -j; k <= j; ++k) {
            double complex s = 0.0;
            for (int n = j; n <= p; ++n) {
                double rn = pow(rho, n - j);
                for (int m = -n; m <= n; ++m) {
                    if (abs(m - k) > n - j) continue;
                    s += L[IDX(n, m)] * or_ipow(abs(m) - abs(m - k) - abs(k)) * or_A(n - j, m - k) * or_A(j, k) *
                         Y[IDX(n - j, m - k)] * rn / or_A(n, m);
                }
            }
            Out[IDX(j, k)] = s;
        }
    free(A);
    free(Y);
}

void or_l2l(int p, const double complex *L, const double c_old[3], const double c_new[3], double complex *Out)
{
    or_l2l_upto(p, p, L, c_old, c_new, Out);
}

/* Potential and gradient of the local expansion about c at x.  The
 * expansion is shifted exactly to x; its degree-0 term is the potential and
 * its degree-1 terms, with r Y_1^0 = z and r Y_1^{+-1} = (x +- i y)/sqrt(2),
 * give d/dz = L'_1^0, d/dx = sqrt(2) Re L'_1^1, d/dy = -sqrt(2) Im L'_1^1. */
void or_eval_le(int p, const double complex *L, const double c[3], const double x[3], double *phi, double grad[3])
{
    double complex Lp[4];
    or_l2l_upto(p, 1, L, c, x, Lp);
    if (phi) *phi = creal(Lp[IDX(0, 0)]);
    if (grad) {
        grad[0] = sqrt(2.0) * creal(Lp[IDX(1, 1)]);
        grad[1] = -sqrt(2.0) * cimag(Lp[IDX(1, 1)]);
        grad[2] = creal(Lp[IDX(1, 0)]);
    }
}

/* ------------------------------------------------------------- FMM */

static void or_box_center(const or_tree *t, int b, double c[3])
{
    double h = t->W / (double)((int64_t)1 << t->level[b]);
    c[0] = t->lo[0] + ((double)t->ix[b] + 0.5) * h;
    c[1] = t->lo[1] + ((double)t->iy[b] + 0.5) * h;
    c[2] = t->lo[2] + ((double)t->iz[b] + 0.5) * h;
}

/* Coulomb field sum_j (x_i - x_j)/|x_i - x_j|^3 (unit source weights) of the
 * targets listed in `targets` (ion ids; ns of them) through the FMM, written
 * to E (ns x 3; may be NULL), and the potential sum_j 1/|x_i - x_j| to phi
 * (ns; may be NULL): the local expansion's value (eq. FMM_local) plus the
 * near field.  need[b] marks the boxes whose local expansions are needed. */
static void or_fmm_field(const or_tree *t, const double *pos, int p, int ns, const int32_t *targets, double *E,
                         double *phi)
{
    int nb = t->nbox, K = (p + 1) * (p + 1);
    double complex *M = (double complex *)calloc((size_t)nb * (size_t)K, sizeof(double complex));
    double complex *L = (double complex *)calloc((size_t)nb * (size_t)K, sizeof(double complex));
    double complex *tmp = (double complex *)malloc(sizeof(double complex) * (size_t)K);
    uint8_t *need = (uint8_t *)calloc((size_t)nb, 1);
    int32_t *leaf_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)t->n); /* sorted slot -> leaf */
    int32_t *slot_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)t->n); /* id -> sorted slot */
    for (int k = 0; k < t->n; ++k) slot_of[t->perm[k]] = k;
    for (int b = 0; b < nb; ++b)
        if (t->is_leaf[b])
            for (int k = t->ion_begin[b]; k < t->ion_end[b]; ++k) leaf_of[k] = b;
    for (int a = 0; a < ns; ++a)
        for (int b = leaf_of[slot_of[targets[a]]]; b >= 0 && !need[b]; b = t->parent[b]) need[b] = 1;

    /* upward pass: P2M at the leaves, then M2M from the finest level up */
    for (int b = 0; b < nb; ++b) {
        if (!t->is_leaf[b]) continue;
        int cnt = t->ion_end[b] - t->ion_begin[b];
        double *ps = (double *)malloc(sizeof(double) * 3 * (size_t)cnt);
        double *qs = (double *)malloc(sizeof(double) * (size_t)cnt);
        for (int k = 0; k < cnt; ++k) {
            int id = t->perm[t->ion_begin[b] + k];
            ps[3 * k] = pos[3 * id]; ps[3 * k + 1] = pos[3 * id + 1]; ps[3 * k + 2] = pos[3 * id + 2];
            qs[k] = 1.0;
        }
        double c[3];
        or_box_center(t, b, c);
        or_p2m(cnt, ps, qs, c, p, M + (size_t)b * K);
        free(ps); free(qs);
    }
    for (int b = nb - 1; b >= 1; --b) {
        int pa = t->parent[b];
        double cb[3], cp[3];
        or_box_center(t, b, cb);
        or_box_center(t, pa, cp);
        or_m2m(p, M + (size_t)b * K, cb, cp, tmp);
        for (int k = 0; k < K; ++k) M[(size_t)pa * K + k] += tmp[k];
    }
    /* downward pass: M2L over the V lists, then L2L from the top */
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nb; ++b) {
        if (!need[b]) continue;
        double cb[3];
        or_box_center(t, b, cb);
        for (int e = t->v_off[b]; e < t->v_off[b + 1]; ++e) {
            int s = t->v_src[e];
            double cs[3];
            or_box_center(t, s, cs);
            or_m2l_add(p, M + (size_t)s * K, cs, cb, L + (size_t)b * K);
        }
    }
    for (int b = 1; b < nb; ++b) {
        if (!need[b]) continue;
        int pa = t->parent[b];
        double cb[3], cp[3];
        or_box_center(t, b, cb);
        or_box_center(t, pa, cp);
        or_l2l(p, L + (size_t)pa * K, cp, cb, tmp);
        for (int k = 0; k < K; ++k) L[(size_t)b * K + k] += tmp[k];
    }
    /* evaluation: far field from the leaf's local expansion, near field by
     * direct summation over the near list */
#pragma omp parallel for schedule(dynamic, 4)
    for (int a = 0; a < ns; ++a) {
        int id = targets[a];
        int leaf = leaf_of[slot_of[id]];
        double c[3], g[3], v;
        or_box_center(t, leaf, c);
        or_eval_le(p, L + (size_t)leaf * K, c, pos + 3 * id, &v, g);
        double ex = -g[0], ey = -g[1], ez = -g[2];
        for (int e = t->near_off[leaf]; e < t->near_off[leaf + 1]; ++e) {
            int s = t->near_src[e];
            for (int k = t->ion_begin[s]; k < t->ion_end[s]; ++k) {
                int j = t->perm[k];
                if (j == id) continue;
                double dx = pos[3 * id] - pos[3 * j];
                double dy = pos[3 * id + 1] - pos[3 * j + 1];
                double dz = pos[3 * id + 2] - pos[3 * j + 2];
                double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 == 0.0) continue;
                double r = sqrt(r2);
                double w = 1.0 / (r2 * r);
                ex += dx * w; ey += dy * w; ez += dz * w;
                v += 1.0 / r;
            }
        }
        if (E) { E[3 * a] = ex; E[3 * a + 1] = ey; E[3 * a + 2] = ez; }
        if (phi) phi[a] = v;
    }
    free(M); free(L); free(tmp); free(need); free(leaf_of); free(slot_of);
}

/* FMM Coulomb force on every ion (ion-id order): F = k_e q^2 E. */
int or_fmm_coulomb(int n, const double *pos, double q, int p, int leaf_size, double *F)
{
    if (n == 0) return 0;
    or_tree *t = or_tree_build(n, pos, leaf_size);
    if (!t) return -1;
    int32_t *ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int i = 0; i < n; ++i) ids[i] = i;
    or_fmm_field(t, pos, p, n, ids, F, NULL);
    double ke = 1.0 / (4.0 * OR_PI * OR_EPS0);
    for (int i = 0; i < 3 * n; ++i) F[i] *= ke * q * q;
    free(ids);
    or_tree_free(t);
    return 0;
}

/* FMM Coulomb force on the ions listed in idx only (F: ns x 3). */
int or_fmm_coulomb_sampled(int n, const double *pos, double q, int p, int leaf_size, int ns, const int32_t *idx,
                           double *F)
{
    or_tree *t = or_tree_build(n, pos, leaf_size);
    if (!t) return -1;
    or_fmm_field(t, pos, p, ns, idx, F, NULL);
    double ke = 1.0 / (4.0 * OR_PI * OR_EPS0);
    for (int i = 0; i < 3 * ns; ++i) F[i] *= ke * q * q;
    or_tree_free(t);
    return 0;
}

/* FMM Coulomb potential (volts) at the ions listed in idx (ns of them; all
 * n ions in id order when idx is NULL): phi^fmm of eq. (rms_pot). */
int or_fmm_potential(int n, const double *pos, double q, int p, int leaf_size, int ns, const int32_t *idx,
                     double *phi)
{
    if (n == 0) return 0;
    or_tree *t = or_tree_build(n, pos, leaf_size);
    if (!t) return -1;
    int32_t *ids = NULL;
    if (!idx) {
        ids = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
        for (int i = 0; i < n; ++i) ids[i] = i;
        ns = n;
    }
    or_fmm_field(t, pos, p, ns, idx ? idx : ids, NULL, phi);
    double ke = 1.0 / (4.0 * OR_PI * OR_EPS0);
    for (int i = 0; i < ns; ++i) phi[i] *= ke * q;
    free(ids);
    or_tree_free(t);
    return 0;
}
