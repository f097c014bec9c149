/*
 * canon_bvh.c -- canonical traversal cost of the BVH method (measurement model).
 *
 * Defines the algorithmic bytes per ray used for roofline accounting,
 * independently of the GPU renderer's own BVH: per environment, a binary BVH
 * built by a full-sweep surface-area heuristic (every centroid-sorted split on
 * each axis, traversal and intersection cost 1, leaves of at most 4
 * triangles), traversed nearest child first with the ray interval shrinking
 * to the closest hit found so far; stack entries whose entry distance lies
 * beyond the current closest hit are discarded without testing.  It counts
 * the ray-box tests (one per child box examined) and ray-triangle tests.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LEAF_MAX 4

typedef struct {
    float lo[3], hi[3];
} box_t;

typedef struct {
    box_t b[2];
    int32_t child[2]; /* >= 0 node, < 0: leaf ~(first << 4 | count) */
} node_t;

typedef struct {
    const float *tri;
    int32_t *idx;
    float *cen;
    node_t *nodes;
    int32_t n_nodes;
    float *sa_right;
    int32_t *scratch;
} build_t;

static int g_axis;
static const float *g_cen;

static int cmp_axis(const void *a, const void *b)
{
    const float ca = g_cen[3 * *(const int32_t *)a + g_axis], cb = g_cen[3 * *(const int32_t *)b + g_axis];
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    return *(const int32_t *)a - *(const int32_t *)b;
}

static void box_empty(box_t *b)
{
    for (int k = 0; k < 3; ++k) {
        b->lo[k] = INFINITY;
        b->hi[k] = -INFINITY;
    }
}

static void box_add_tri(box_t *b, const float *t)
{
    for (int v = 0; v < 3; ++v)
        for (int k = 0; k < 3; ++k) {
            b->lo[k] = fminf(b->lo[k], t[3 * v + k]);
            b->hi[k] = fmaxf(b->hi[k], t[3 * v + k]);
        }
}

static float half_area(const box_t *b)
{
    const float dx = b->hi[0] - b->lo[0], dy = b->hi[1] - b->lo[1], dz = b->hi[2] - b->lo[2];
    return dx * dy + dy * dz + dz * dx;
}

static box_t range_box(build_t *B, int32_t b, int32_t e)
{
    box_t r;
    box_empty(&r);
    for (int32_t i = b; i < e; ++i)
        box_add_tri(&r, B->tri + 9 * B->idx[i]);
    return r;
}

/* returns the child ref of the subtree over idx[b, e) */
static int32_t build(build_t *B, int32_t b, int32_t e)
{
    const int32_t n = e - b;
    if (n <= LEAF_MAX)
        return ~((b << 4) | n);
    int best_axis = -1, best_k = -1;
    double best_cost = INFINITY;
    for (int axis = 0; axis < 3; ++axis) {
        g_axis = axis;
        g_cen = B->cen;
        qsort(B->idx + b, n, sizeof(int32_t), cmp_axis);
        box_t acc;
        box_empty(&acc);
        for (int32_t i = n - 1; i >= 1; --i) {
            box_add_tri(&acc, B->tri + 9 * B->idx[b + i]);
            B->sa_right[i] = half_area(&acc);
        }
        box_empty(&acc);
        for (int32_t i = 0; i < n - 1; ++i) {
            box_add_tri(&acc, B->tri + 9 * B->idx[b + i]);
            const double c = (double)half_area(&acc) * (i + 1) + (double)B->sa_right[i + 1] * (n - i - 1);
            if (c < best_cost) {
                best_cost = c;
                best_axis = axis;
                best_k = i + 1;
            }
        }
    }
    g_axis = best_axis;
    g_cen = B->cen;
    qsort(B->idx + b, n, sizeof(int32_t), cmp_axis);
    const int32_t id = B->n_nodes++;
    const int32_t m = b + best_k;
    B->nodes[id].b[0] = range_box(B, b, m);
    B->nodes[id].b[1] = range_box(B, m, e);
    const int32_t l = build(B, b, m);
    const int32_t r = build(B, m, e);
    B->nodes[id].child[0] = l;
    B->nodes[id].child[1] = r;
    return id;
}

static int slab(const box_t *b, const double *o, const double *inv, double tn, double tf, double *tenter)
{
    double t0 = tn, t1 = tf;
    for (int k = 0; k < 3; ++k) {
        double a = (b->lo[k] - o[k]) * inv[k], c = (b->hi[k] - o[k]) * inv[k];
        if (isnan(a)) a = -INFINITY;
        if (isnan(c)) c = INFINITY;
        if (a > c) { const double s = a; a = c; c = s; }
        if (a > t0) t0 = a;
        if (c < t1) t1 = c;
    }
    *tenter = t0;
    return t0 <= t1;
}

static int tri_hit(const float *t, const double *o, const double *d, double tn, double tf, double *th)
{
    const double e1[3] = {t[3] - t[0], t[4] - t[1], t[5] - t[2]};
    const double e2[3] = {t[6] - t[0], t[7] - t[1], t[8] - t[2]};
    const double p[3] = {d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]};
    const double det = e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2];
    if (det == 0.0) return 0;
    const double inv = 1.0 / det;
    const double s[3] = {o[0] - t[0], o[1] - t[1], o[2] - t[2]};
    const double u = (s[0] * p[0] + s[1] * p[1] + s[2] * p[2]) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    const double q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
    const double v = (d[0] * q[0] + d[1] * q[1] + d[2] * q[2]) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    const double tt = (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]) * inv;
    if (tt < tn || tt > tf) return 0;
    *th = tt;
    return 1;
}

/* One environment: n_tris world triangles, n_rays rays; accumulates counts. */
__attribute__((visibility("default"))) int canon_counts(int64_t n_tris, const float *tri, int64_t n_rays,
                                                        const float *o, const float *d, const float *tn,
                                                        const float *tf, double *box_tests, double *tri_tests,
                                                        int32_t *max_depth)
{
    if (n_tris <= 0)
        return 0;
    build_t B;
    B.tri = tri;
    B.idx = (int32_t *)malloc(sizeof(int32_t) * n_tris);
    B.cen = (float *)malloc(sizeof(float) * 3 * n_tris);
    B.nodes = (node_t *)malloc(sizeof(node_t) * (n_tris + 1));
    B.sa_right = (float *)malloc(sizeof(float) * (n_tris + 1));
    B.n_nodes = 0;
    for (int64_t i = 0; i < n_tris; ++i) {
        B.idx[i] = (int32_t)i;
        box_t b;
        box_empty(&b);
        box_add_tri(&b, tri + 9 * i);
        for (int k = 0; k < 3; ++k)
            B.cen[3 * i + k] = 0.5f * (b.lo[k] + b.hi[k]);
    }
    const int32_t root = build(&B, 0, (int32_t)n_tris);
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (B.n_nodes + 4));
    double *stack_t = (double *)malloc(sizeof(double) * (B.n_nodes + 4));
    double nbox = 0, ntri = 0;
    int32_t depth_max = 0;
    for (int64_t r = 0; r < n_rays; ++r) {
        const double O[3] = {o[3 * r], o[3 * r + 1], o[3 * r + 2]};
        const double D[3] = {d[3 * r], d[3 * r + 1], d[3 * r + 2]};
        const double inv[3] = {1.0 / D[0], 1.0 / D[1], 1.0 / D[2]};
        double best = tf[r];
        const double near = tn[r];
        int sp = 0;
        stack[sp] = root;
        stack_t[sp] = near;
        ++sp;
        while (sp > 0) {
            --sp;
            const int32_t ref = stack[sp];
            if (stack_t[sp] > best)
                continue;
            if (ref < 0) {
                const int32_t code = ~ref, first = code >> 4, cnt = code & 15;
                for (int32_t k = 0; k < cnt; ++k) {
                    double th;
                    ntri += 1;
                    if (tri_hit(tri + 9 * B.idx[first + k], O, D, near, best, &th))
                        best = th;
                }
                continue;
            }
            const node_t *nd = &B.nodes[ref];
            double t0, t1;
            const int h0 = slab(&nd->b[0], O, inv, near, best, &t0);
            const int h1 = slab(&nd->b[1], O, inv, near, best, &t1);
            nbox += 2;
            if (h0 && h1) {
                const int first0 = t0 <= t1;
                stack[sp] = first0 ? nd->child[1] : nd->child[0];
                stack_t[sp] = first0 ? t1 : t0;
                ++sp;
                stack[sp] = first0 ? nd->child[0] : nd->child[1];
                stack_t[sp] = first0 ? t0 : t1;
                ++sp;
            } else if (h0 || h1) {
                stack[sp] = h0 ? nd->child[0] : nd->child[1];
                stack_t[sp] = h0 ? t0 : t1;
                ++sp;
            }
            if (sp > depth_max)
                depth_max = sp;
        }
    }
    *box_tests += nbox;
    *tri_tests += ntri;
    if (depth_max > *max_depth)
        *max_depth = depth_max;
    free(stack);
    free(stack_t);
    free(B.idx);
    free(B.cen);
    free(B.nodes);
    free(B.sa_right);
    return 0;
}
