/*
 * evo_scene.c -- oracle: animated scene at an instant, pinhole camera,
 * watertight ray/triangle test, brute-force and plain-BVH ray queries.
 * TEST INFRASTRUCTURE ONLY (see evo.h).
 *
 * The renderer in the paper is pbrt-v4's unidirectional path tracer over
 * an animated scene (Sec. 3.3, Sec. 4).  The paper does not fix the camera
 * model, the intersection routine or the acceleration structure, so this
 * oracle takes the simplest definitions:
 *   - instance transform at time t: entry-wise linear interpolation of 3x4
 *     key matrices in FP64, vertices transformed in FP64 and rounded once
 *     to FP32;
 *   - pinhole camera with a box pixel filter, or a thin lens (a point on
 *     the aperture disk, the ray through the pinhole ray's point on the
 *     plane in focus);
 *   - watertight ray/triangle test (Woop, Benthin, Wald, JCGT 2013) in FP32;
 *   - closest hit = lexicographic minimum of (t, primitive index) over all
 *     triangles other than the ray's origin primitive with tmin < t < tmax,
 *     so the answer does not depend on any acceleration structure.
 */
#include "evo_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Scene description copy. */

static void *dup_bytes(const void *src, size_t n)
{
    if (n == 0) return NULL;
    void *p = malloc(n);
    memcpy(p, src, n);
    return p;
}

float evo_luminance(float r, float g, float b)
{
    return (0.2126f * r + 0.7152f * g) + 0.0722f * b;
}

float evo__emission_y(const evo_scene_desc *d, uint32_t m)
{
    if (!d->albedo_rgb) return d->emission[m];
    const float *e = d->emission_rgb + 3 * (size_t)m;
    return evo_luminance(e[0], e[1], e[2]);
}

evo_scene *evo_scene_new(const evo_scene_desc *d)
{
    evo_scene *s = (evo_scene *)calloc(1, sizeof(*s));
    s->d = *d;
    s->d.albedo = dup_bytes(d->albedo, sizeof(float) * d->n_mat);
    s->d.emission = dup_bytes(d->emission, sizeof(float) * d->n_mat);
    s->d.xyz = dup_bytes(d->xyz, sizeof(float) * 3 * d->n_vert);
    s->d.tri_idx = dup_bytes(d->tri_idx, sizeof(uint32_t) * 3 * d->n_tri);
    s->d.tri_mat = dup_bytes(d->tri_mat, sizeof(uint32_t) * d->n_tri);
    s->d.mesh_tri_off = dup_bytes(d->mesh_tri_off, sizeof(uint32_t) * (d->n_mesh + 1));
    s->d.inst_mesh = dup_bytes(d->inst_mesh, sizeof(uint32_t) * d->n_inst);
    s->d.inst_key_off = dup_bytes(d->inst_key_off, sizeof(uint32_t) * (d->n_inst + 1));
    uint32_t nk = d->n_inst ? d->inst_key_off[d->n_inst] : 0;
    s->d.key_t = dup_bytes(d->key_t, sizeof(double) * nk);
    s->d.key_xform = dup_bytes(d->key_xform, sizeof(double) * 12 * nk);
    s->d.pl_pos = dup_bytes(d->pl_pos, sizeof(float) * 3 * d->n_plight);
    s->d.pl_intensity = dup_bytes(d->pl_intensity, sizeof(float) * d->n_plight);
    s->d.cam_t = dup_bytes(d->cam_t, sizeof(double) * d->cam_nkeys);
    s->d.cam_elu = dup_bytes(d->cam_elu, sizeof(double) * 9 * d->cam_nkeys);
    s->d.env = dup_bytes(d->env, sizeof(float) * 6 * (size_t)d->env_res * d->env_res);
    s->d.albedo_rgb = d->albedo_rgb ? dup_bytes(d->albedo_rgb, sizeof(float) * 3 * d->n_mat) : NULL;
    s->d.emission_rgb = d->albedo_rgb ? dup_bytes(d->emission_rgb, sizeof(float) * 3 * d->n_mat) : NULL;
    s->d.pl_rgb = d->albedo_rgb && d->pl_rgb ? dup_bytes(d->pl_rgb, sizeof(float) * 3 * d->n_plight) : NULL;
    return s;
}

void evo_scene_free(evo_scene *s)
{
    if (!s) return;
    free((void *)s->d.albedo); free((void *)s->d.emission); free((void *)s->d.xyz);
    free((void *)s->d.tri_idx); free((void *)s->d.tri_mat); free((void *)s->d.mesh_tri_off);
    free((void *)s->d.inst_mesh); free((void *)s->d.inst_key_off); free((void *)s->d.key_t);
    free((void *)s->d.key_xform); free((void *)s->d.pl_pos); free((void *)s->d.pl_intensity);
    free((void *)s->d.cam_t); free((void *)s->d.cam_elu); free((void *)s->d.env);
    free((void *)s->d.albedo_rgb); free((void *)s->d.emission_rgb); free((void *)s->d.pl_rgb);
    free(s);
}

/* ---------------------------------------------------------------------- */
/* Keyframe interpolation: before the first key the first value, after the
 * last key the last value, otherwise v_k + w (v_{k+1} - v_k) with
 * w = (t - t_k) / (t_{k+1} - t_k), entry by entry, in FP64. */
static void interp_keys(const double *kt, const double *kv, uint32_t nkeys, uint32_t width,
                        double t, double *out)
{
    if (nkeys == 1 || t <= kt[0]) {
        memcpy(out, kv, sizeof(double) * width);
        return;
    }
    if (t >= kt[nkeys - 1]) {
        memcpy(out, kv + (size_t)(nkeys - 1) * width, sizeof(double) * width);
        return;
    }
    uint32_t k = 0;
    while (!(t < kt[k + 1])) ++k;
    double w = (t - kt[k]) / (kt[k + 1] - kt[k]);
    const double *a = kv + (size_t)k * width;
    const double *b = a + width;
    for (uint32_t e = 0; e < width; ++e) out[e] = a[e] + w * (b[e] - a[e]);
}

/* Unit geometric normal n = cross(v1 - v0, v2 - v0) / |.| and area |.|/2 in
 * FP32; a degenerate triangle gets a zero normal. */
static void tri_normal(const float *v, float n[3], float *area)
{
    float e1x = v[3] - v[0], e1y = v[4] - v[1], e1z = v[5] - v[2];
    float e2x = v[6] - v[0], e2y = v[7] - v[1], e2z = v[8] - v[2];
    float gx = e1y * e2z - e1z * e2y;
    float gy = e1z * e2x - e1x * e2z;
    float gz = e1x * e2y - e1y * e2x;
    float len = sqrtf((gx * gx + gy * gy) + gz * gz);
    if (len == 0.0f) {
        n[0] = n[1] = n[2] = 0.0f;
    } else {
        n[0] = gx / len; n[1] = gy / len; n[2] = gz / len;
    }
    *area = 0.5f * len;
}

static void build_instant(const evo_scene *s, double t, evo_instant *I, int use_bvh)
{
    const evo_scene_desc *d = &s->d;
    uint32_t nt = 0;
    for (uint32_t i = 0; i < d->n_inst; ++i) {
        uint32_t m = d->inst_mesh[i];
        nt += d->mesh_tri_off[m + 1] - d->mesh_tri_off[m];
    }
    I->n_tri = nt;
    I->tri = (float *)malloc(sizeof(float) * 9 * (nt ? nt : 1));
    I->nrm = (float *)malloc(sizeof(float) * 3 * (nt ? nt : 1));
    I->area = (float *)malloc(sizeof(float) * (nt ? nt : 1));
    I->mat = (uint32_t *)malloc(sizeof(uint32_t) * (nt ? nt : 1));
    uint32_t prim = 0;
    for (uint32_t i = 0; i < d->n_inst; ++i) {
        uint32_t m = d->inst_mesh[i];
        uint32_t k0 = d->inst_key_off[i], nk = d->inst_key_off[i + 1] - k0;
        double M[12];
        interp_keys(d->key_t + k0, d->key_xform + (size_t)12 * k0, nk, 12, t, M);
        for (uint32_t tr = d->mesh_tri_off[m]; tr < d->mesh_tri_off[m + 1]; ++tr) {
            for (int c = 0; c < 3; ++c) {
                const float *p = d->xyz + 3 * (size_t)d->tri_idx[3 * (size_t)tr + c];
                double x = p[0], y = p[1], z = p[2];
                for (int r = 0; r < 3; ++r) {
                    const double *row = M + 4 * r;
                    double w = ((row[0] * x + row[1] * y) + row[2] * z) + row[3];
                    I->tri[9 * (size_t)prim + 3 * c + r] = (float)w;
                }
            }
            I->mat[prim] = d->tri_mat[tr];
            tri_normal(I->tri + 9 * (size_t)prim, I->nrm + 3 * (size_t)prim, &I->area[prim]);
            ++prim;
        }
    }

    /* Emitter table: triangles with Le > 0, in primitive order.  Power
     * w_j = A_j * Le_j (FP32), prefix sums and total S in FP64 in that
     * order, cdf_j = (float)(prefix_j / S), last entry exactly 1.  With RGB
     * radiance Le_j is the luminance of the emission. */
    I->n_emit = 0;
    for (uint32_t p = 0; p < nt; ++p)
        if (evo__emission_y(d, I->mat[p]) > 0.0f) ++I->n_emit;
    I->emit_prim = (uint32_t *)malloc(sizeof(uint32_t) * (I->n_emit ? I->n_emit : 1));
    I->emit_cdf = (float *)malloc(sizeof(float) * (I->n_emit ? I->n_emit : 1));
    double *pref = (double *)malloc(sizeof(double) * (I->n_emit ? I->n_emit : 1));
    double S = 0.0;
    uint32_t j = 0;
    for (uint32_t p = 0; p < nt; ++p) {
        float le = evo__emission_y(d, I->mat[p]);
        if (le > 0.0f) {
            float w = I->area[p] * le;
            S += (double)w;
            pref[j] = S;
            I->emit_prim[j] = p;
            ++j;
        }
    }
    for (j = 0; j < I->n_emit; ++j) I->emit_cdf[j] = (float)(pref[j] / S);
    if (I->n_emit) I->emit_cdf[I->n_emit - 1] = 1.0f;
    I->emit_S = (float)S;
    free(pref);

    /* Camera basis in FP64, rounded once to FP32. */
    double cam[9];
    interp_keys(d->cam_t, d->cam_elu, d->cam_nkeys, 9, t, cam);
    double f[3] = {cam[3] - cam[0], cam[4] - cam[1], cam[5] - cam[2]};
    double fl = sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
    f[0] = f[0] / fl; f[1] = f[1] / fl; f[2] = f[2] / fl;
    const double *up = cam + 6;
    double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2],
                   f[0] * up[1] - f[1] * up[0]};
    double rl = sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
    r[0] = r[0] / rl; r[1] = r[1] / rl; r[2] = r[2] / rl;
    double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2],
                   r[0] * f[1] - r[1] * f[0]};
    double th = tan(d->vfov_deg * (3.14159265358979323846 / 360.0));
    for (int c = 0; c < 3; ++c) {
        I->eye[c] = (float)cam[c];
        I->fwd[c] = (float)f[c];
        I->right[c] = (float)r[c];
        I->up[c] = (float)u[c];
    }
    I->sx = (float)(th * ((double)d->width / (double)d->height));
    I->sy = (float)th;

    I->bvh = NULL;
    I->n_nodes = 0;
    if (use_bvh && nt > 0) evo__bvh_build(I);
}

static void free_instant(evo_instant *I)
{
    free(I->tri); free(I->nrm); free(I->area); free(I->mat);
    free(I->emit_prim); free(I->emit_cdf); free(I->bvh); free(I->bvh_idx);
}

evo_frame *evo_frame_new(const evo_scene *s, double t0, double t1, int use_bvh)
{
    evo_frame *f = (evo_frame *)calloc(1, sizeof(*f));
    f->scene = s;
    f->time[0] = t0;
    f->time[1] = t1;
    f->use_bvh = use_bvh;
    build_instant(s, t0, &f->inst[0], use_bvh);
    build_instant(s, t1, &f->inst[1], use_bvh);
    return f;
}

void evo_frame_free(evo_frame *f)
{
    if (!f) return;
    free_instant(&f->inst[0]);
    free_instant(&f->inst[1]);
    free(f);
}

uint32_t evo_frame_num_tris(const evo_frame *f) { return f->inst[0].n_tri; }

void evo_frame_world_tris(const evo_frame *f, int instant, float *xyz9, uint32_t *mat)
{
    const evo_instant *I = &f->inst[instant];
    memcpy(xyz9, I->tri, sizeof(float) * 9 * I->n_tri);
    memcpy(mat, I->mat, sizeof(uint32_t) * I->n_tri);
}

void evo_frame_camera(const evo_frame *f, int instant, float *eye3, float *fwd3,
                      float *right3, float *up3, float *sxy2)
{
    const evo_instant *I = &f->inst[instant];
    memcpy(eye3, I->eye, sizeof(float) * 3);
    memcpy(fwd3, I->fwd, sizeof(float) * 3);
    memcpy(right3, I->right, sizeof(float) * 3);
    memcpy(up3, I->up, sizeof(float) * 3);
    sxy2[0] = I->sx;
    sxy2[1] = I->sy;
}

/* ---------------------------------------------------------------------- */
/* Watertight ray/triangle test (Woop, Benthin, Wald 2013).  The axis of the
 * largest |d| component becomes z (ties go to the lower axis index), the
 * other two follow cyclically and are swapped when d_z < 0 to keep the
 * winding.  Vertices are translated to the ray origin and sheared so the
 * ray is the +z axis; the 2D edge functions U, V, W decide the hit (all of
 * one sign), recomputed in FP64 when any is exactly zero. */
void evo__ray_setup(evo_ray *r, const float o[3], const float d[3])
{
    for (int c = 0; c < 3; ++c) { r->o[c] = o[c]; r->d[c] = d[c]; }
    float ax = fabsf(d[0]), ay = fabsf(d[1]), az = fabsf(d[2]);
    int kz = 0;
    float m = ax;
    if (ay > m) { kz = 1; m = ay; }
    if (az > m) { kz = 2; }
    int kx = kz + 1 == 3 ? 0 : kz + 1;
    int ky = kx + 1 == 3 ? 0 : kx + 1;
    if (d[kz] < 0.0f) { int tmp = kx; kx = ky; ky = tmp; }
    r->kx = kx; r->ky = ky; r->kz = kz;
    r->Sx = d[kx] / d[kz];
    r->Sy = d[ky] / d[kz];
    r->Sz = 1.0f / d[kz];
}

int evo__tri_test(const evo_ray *r, const float *v, float *t_out)
{
    const int kx = r->kx, ky = r->ky, kz = r->kz;
    float A[3], B[3], C[3];
    for (int c = 0; c < 3; ++c) {
        A[c] = v[c] - r->o[c];
        B[c] = v[3 + c] - r->o[c];
        C[c] = v[6 + c] - r->o[c];
    }
    float Ax = A[kx] - r->Sx * A[kz];
    float Ay = A[ky] - r->Sy * A[kz];
    float Bx = B[kx] - r->Sx * B[kz];
    float By = B[ky] - r->Sy * B[kz];
    float Cx = C[kx] - r->Sx * C[kz];
    float Cy = C[ky] - r->Sy * C[kz];
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if (U == 0.0f || V == 0.0f || W == 0.0f) {
        U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
        V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
        W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
    }
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return 0;
    float det = (U + V) + W;
    if (det == 0.0f) return 0;
    float Az = r->Sz * A[kz];
    float Bz = r->Sz * B[kz];
    float Cz = r->Sz * C[kz];
    float T = (U * Az + V * Bz) + W * Cz;
    *t_out = T / det;
    return 1;
}

/* ---------------------------------------------------------------------- */
/* Ray queries.  Brute force tests every triangle; the BVH path must give
 * the same answer (checked by the tests). */

static int closest_brute(const evo_instant *I, const evo_ray *r, float tmin, float tmax,
                         uint32_t skip, float *bt, uint32_t *bp)
{
    float best_t = tmax;
    uint32_t best_p = EVO_NO_PRIM;
    for (uint32_t p = 0; p < I->n_tri; ++p) {
        if (p == skip) continue;
        float t;
        if (!evo__tri_test(r, I->tri + 9 * (size_t)p, &t)) continue;
        if (!(t > tmin) || !(t < tmax)) continue;
        if (t < best_t || (t == best_t && p < best_p)) {
            best_t = t;
            best_p = p;
        }
    }
    *bt = best_t;
    *bp = best_p;
    return best_p != EVO_NO_PRIM;
}

static int any_brute(const evo_instant *I, const evo_ray *r, float tmin, float tmax,
                     uint32_t skip)
{
    for (uint32_t p = 0; p < I->n_tri; ++p) {
        if (p == skip) continue;
        float t;
        if (!evo__tri_test(r, I->tri + 9 * (size_t)p, &t)) continue;
        if (t > tmin && t < tmax) return 1;
    }
    return 0;
}

int evo__closest(const evo_frame *f, int instant, const evo_ray *r, float tmin, float tmax,
                 uint32_t skip, int brute, float *t_out, uint32_t *prim_out)
{
    const evo_instant *I = &f->inst[instant];
    if (brute || !I->bvh) return closest_brute(I, r, tmin, tmax, skip, t_out, prim_out);
    return evo__bvh_closest(I, r, tmin, tmax, skip, t_out, prim_out);
}

int evo__any(const evo_frame *f, int instant, const evo_ray *r, float tmin, float tmax,
             uint32_t skip, int brute)
{
    const evo_instant *I = &f->inst[instant];
    if (brute || !I->bvh) return any_brute(I, r, tmin, tmax, skip);
    return evo__bvh_any(I, r, tmin, tmax, skip);
}

int evo_closest_hit(const evo_frame *f, int instant, const float o[3], const float d[3],
                    float tmin, float tmax, uint32_t skip, int brute,
                    float *t_out, uint32_t *prim_out)
{
    evo_ray r;
    evo__ray_setup(&r, o, d);
    return evo__closest(f, instant, &r, tmin, tmax, skip, brute, t_out, prim_out);
}

int evo_any_hit(const evo_frame *f, int instant, const float o[3], const float d[3],
                float tmin, float tmax, uint32_t skip, int brute)
{
    evo_ray r;
    evo__ray_setup(&r, o, d);
    return evo__any(f, instant, &r, tmin, tmax, skip, brute);
}

void evo_ray_queries(const evo_frame *f, int instant, uint32_t n, const float *o, const float *d,
                     const float *tmin, const float *tmax, const uint32_t *skip, int any, int brute,
                     float *t_out, uint32_t *prim_out)
{
    for (uint32_t i = 0; i < n; ++i) {
        if (any) {
            prim_out[i] = (uint32_t)evo_any_hit(f, instant, o + 3 * (size_t)i, d + 3 * (size_t)i, tmin[i], tmax[i],
                                                skip[i], brute);
        } else {
            evo_closest_hit(f, instant, o + 3 * (size_t)i, d + 3 * (size_t)i, tmin[i], tmax[i], skip[i], brute,
                            &t_out[i], &prim_out[i]);
        }
    }
}
