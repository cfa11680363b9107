/* evo_internal.h -- oracle internals.  TEST INFRASTRUCTURE ONLY. */
#ifndef EVO_INTERNAL_H
#define EVO_INTERNAL_H

#include "evo.h"

struct evo_scene {
    evo_scene_desc d; /* deep copy */
};

typedef struct {
    double lo[3], hi[3];
    int32_t left, right; /* child nodes, -1 for a leaf */
    uint32_t first, count; /* leaf range into bvh_idx */
} evo_node;

typedef struct {
    uint32_t n_tri;
    float *tri;       /* [n_tri][9] world-space vertices, FP32 */
    float *nrm;       /* [n_tri][3] unit geometric normal      */
    float *area;      /* [n_tri]                               */
    uint32_t *mat;    /* [n_tri]                               */
    uint32_t n_emit;
    uint32_t *emit_prim;
    float *emit_cdf;
    float emit_S;     /* sum of A_j * Le_j over emitters       */
    float eye[3], fwd[3], right[3], up[3], sx, sy;
    evo_node *bvh;
    uint32_t *bvh_idx;
    uint32_t n_nodes;
} evo_instant;

struct evo_frame {
    const evo_scene *scene;
    double time[2];
    int use_bvh;
    evo_instant inst[2];
};

typedef struct {
    float o[3], d[3];
    int kx, ky, kz;
    float Sx, Sy, Sz;
} evo_ray;

/* Emitted radiance of material m used for emitter selection: Le, or the
 * luminance of the RGB emission. */
float evo__emission_y(const evo_scene_desc *d, uint32_t m);
void evo__ray_setup(evo_ray *r, const float o[3], const float d[3]);
int evo__tri_test(const evo_ray *r, const float *v, float *t_out);
int evo__closest(const evo_frame *f, int instant, const evo_ray *r, float tmin, float tmax,
                 uint32_t skip, int brute, float *t_out, uint32_t *prim_out);
int evo__any(const evo_frame *f, int instant, const evo_ray *r, float tmin, float tmax,
             uint32_t skip, int brute);
void evo__bvh_build(evo_instant *I);
int evo__bvh_closest(const evo_instant *I, const evo_ray *r, float tmin, float tmax,
                     uint32_t skip, float *t_out, uint32_t *prim_out);
int evo__bvh_any(const evo_instant *I, const evo_ray *r, float tmin, float tmax, uint32_t skip);
void evo__stats_decide(const double *x0, uint32_t m0, const double *x1, uint32_t m1,
                       const evo_params *p, double *mean, double *var, double *t_out,
                       double *df_out, double *p_out, int *stop_out, double *norm_margin);

#endif
