/*
 * evo_bvh.c -- oracle: a plain median-split bounding volume hierarchy used
 * only to make the oracle fast enough on large scenes.  It must return the
 * same answers as brute force: boxes are padded generously and tested in
 * FP64, so a box never culls a triangle that the FP32 triangle test hits,
 * and the closest hit keeps the (t, primitive) lexicographic rule.
 * TEST INFRASTRUCTURE ONLY (see evo.h).
 */
#include "evo_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double key;
    uint32_t prim;
} sort_item;

static int cmp_item(const void *a, const void *b)
{
    const sort_item *x = (const sort_item *)a, *y = (const sort_item *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return x->prim < y->prim ? -1 : (x->prim > y->prim ? 1 : 0);
}

typedef struct {
    evo_instant *I;
    uint32_t cap;
    sort_item *scratch;
} builder;

static uint32_t new_node(builder *b)
{
    if (b->I->n_nodes == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 64;
        b->I->bvh = (evo_node *)realloc(b->I->bvh, sizeof(evo_node) * b->cap);
    }
    return b->I->n_nodes++;
}

static void build_rec(builder *b, uint32_t node, uint32_t first, uint32_t count)
{
    evo_instant *I = b->I;
    evo_node *n = &I->bvh[node];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = first; i < first + count; ++i) {
        const float *v = I->tri + 9 * (size_t)I->bvh_idx[i];
        for (int c = 0; c < 3; ++c) {
            double cen = 0.0;
            for (int k = 0; k < 3; ++k) {
                double x = v[3 * k + c];
                if (x < lo[c]) lo[c] = x;
                if (x > hi[c]) hi[c] = x;
                cen += x;
            }
            cen /= 3.0;
            if (cen < clo[c]) clo[c] = cen;
            if (cen > chi[c]) chi[c] = cen;
        }
    }
    /* Padding far above FP32 rounding of the triangle test. */
    for (int c = 0; c < 3; ++c) {
        double mag = fabs(lo[c]) > fabs(hi[c]) ? fabs(lo[c]) : fabs(hi[c]);
        double pad = 1e-4 * (1.0 + mag);
        n->lo[c] = lo[c] - pad;
        n->hi[c] = hi[c] + pad;
    }
    n->left = n->right = -1;
    n->first = first;
    n->count = count;
    if (count <= 4) return;

    int axis = 0;
    double ext = chi[0] - clo[0];
    for (int c = 1; c < 3; ++c)
        if (chi[c] - clo[c] > ext) { ext = chi[c] - clo[c]; axis = c; }
    for (uint32_t i = 0; i < count; ++i) {
        uint32_t p = I->bvh_idx[first + i];
        const float *v = I->tri + 9 * (size_t)p;
        b->scratch[i].key = ((double)v[axis] + (double)v[3 + axis]) + (double)v[6 + axis];
        b->scratch[i].prim = p;
    }
    qsort(b->scratch, count, sizeof(sort_item), cmp_item);
    for (uint32_t i = 0; i < count; ++i) I->bvh_idx[first + i] = b->scratch[i].prim;

    uint32_t half = count / 2;
    uint32_t l = new_node(b);
    uint32_t r = new_node(b);
    n = &I->bvh[node]; /* realloc may have moved it */
    n->left = (int32_t)l;
    n->right = (int32_t)r;
    n->count = 0;
    build_rec(b, l, first, half);
    build_rec(b, r, first + half, count - half);
}

void evo__bvh_build(evo_instant *I)
{
    builder b;
    b.I = I;
    b.cap = 0;
    I->bvh = NULL;
    I->n_nodes = 0;
    I->bvh_idx = (uint32_t *)malloc(sizeof(uint32_t) * I->n_tri);
    for (uint32_t i = 0; i < I->n_tri; ++i) I->bvh_idx[i] = i;
    b.scratch = (sort_item *)malloc(sizeof(sort_item) * I->n_tri);
    uint32_t root = new_node(&b);
    build_rec(&b, root, 0, I->n_tri);
    free(b.scratch);
}

/* FP64 slab test of the ray segment [tmin, tmax] against a padded box. */
static int box_hit(const evo_node *n, const evo_ray *r, double tmin, double tmax)
{
    double t0 = tmin, t1 = tmax;
    for (int c = 0; c < 3; ++c) {
        double o = r->o[c], d = r->d[c];
        if (d == 0.0) {
            if (o < n->lo[c] || o > n->hi[c]) return 0;
            continue;
        }
        double ta = (n->lo[c] - o) / d;
        double tb = (n->hi[c] - o) / d;
        if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
        if (t0 > t1) return 0;
    }
    return 1;
}

int evo__bvh_closest(const evo_instant *I, const evo_ray *r, float tmin, float tmax,
                     uint32_t skip, float *t_out, uint32_t *prim_out)
{
    float best_t = tmax;
    uint32_t best_p = EVO_NO_PRIM;
    uint32_t stack[128];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const evo_node *n = &I->bvh[stack[--sp]];
        if (!box_hit(n, r, (double)tmin, (double)best_t)) continue;
        if (n->left < 0) {
            for (uint32_t i = n->first; i < n->first + n->count; ++i) {
                uint32_t p = I->bvh_idx[i];
                if (p == skip) continue;
                float t;
                if (!evo__tri_test(r, I->tri + 9 * (size_t)p, &t)) continue;
                if (!(t > tmin) || !(t < tmax)) continue;
                if (t < best_t || (t == best_t && p < best_p)) {
                    best_t = t;
                    best_p = p;
                }
            }
        } else {
            stack[sp++] = (uint32_t)n->left;
            stack[sp++] = (uint32_t)n->right;
        }
    }
    *t_out = best_t;
    *prim_out = best_p;
    return best_p != EVO_NO_PRIM;
}

int evo__bvh_any(const evo_instant *I, const evo_ray *r, float tmin, float tmax, uint32_t skip)
{
    uint32_t stack[128];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const evo_node *n = &I->bvh[stack[--sp]];
        if (!box_hit(n, r, (double)tmin, (double)tmax)) continue;
        if (n->left < 0) {
            for (uint32_t i = n->first; i < n->first + n->count; ++i) {
                uint32_t p = I->bvh_idx[i];
                if (p == skip) continue;
                float t;
                if (!evo__tri_test(r, I->tri + 9 * (size_t)p, &t)) continue;
                if (t > tmin && t < tmax) return 1;
            }
        } else {
            stack[sp++] = (uint32_t)n->left;
            stack[sp++] = (uint32_t)n->right;
        }
    }
    return 0;
}
