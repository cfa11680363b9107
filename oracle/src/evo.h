/*
 * evo.h -- CPU oracle for the adaptive event-camera path tracer.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the plain, slow, independent
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or constant generator with the GPU
 * library; both sides implement the same written definitions separately.
 *
 * What it computes (paper: "Monte Carlo Path Tracing and Statistical Event
 * Detection for Event Camera Simulation", arXiv 2408.07996):
 *   - per-path Monte Carlo radiance at a pixel and a time instant (the
 *     tracePaths subroutine of Algorithm 1 and Sec. 3.3), as a plain
 *     unidirectional path tracer with next-event estimation;
 *   - log-luminance samples and their mean/variance (Eq. 3-4, calcMeanVar
 *     of Algorithm 1) in FP64 by the two-pass formula;
 *   - the one-tailed t-test of Eq. 7 and Sec. 3.2 on the lower tail, with the
 *     p-value from the Student t CDF (regularized incomplete beta, Lentz
 *     continued fraction), and the event rule of Algorithm 1 / Eq. 1.
 *
 * Precision: path radiance in FP32 (the renderer's radiance type), every
 * statistic and the test in FP64.
 */
#ifndef EVO_H
#define EVO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EVO_NO_PRIM 0xffffffffu

enum { EVO_MODE_ADAPTIVE_1T = 0, EVO_MODE_FIXED = 1, EVO_MODE_ADAPTIVE_2T = 2, EVO_MODE_MEAN_ONLY = 3 };
enum { EVO_DF_STUDENT = 0, EVO_DF_WELCH = 1 };
enum { EVO_REF_LOCKSTEP = 0, EVO_REF_FULL = 1 };

/* Flat scene description.  All arrays are read during evo_scene_new and
 * deep-copied.  Vertex indices in tri_idx are global (into xyz). */
typedef struct {
    uint32_t n_mat;
    const float *albedo;      /* [n_mat]  Lambertian albedo a in [0,1)        */
    const float *emission;    /* [n_mat]  emitted radiance Le >= 0 (one-sided) */
    uint32_t n_vert;
    const float *xyz;         /* [n_vert][3] object-space vertices             */
    uint32_t n_tri;
    const uint32_t *tri_idx;  /* [n_tri][3]                                    */
    const uint32_t *tri_mat;  /* [n_tri]                                       */
    uint32_t n_mesh;
    const uint32_t *mesh_tri_off; /* [n_mesh+1] triangle range of each mesh    */
    uint32_t n_inst;
    const uint32_t *inst_mesh;    /* [n_inst]                                  */
    const uint32_t *inst_key_off; /* [n_inst+1] key range of each instance     */
    const double *key_t;          /* [total keys]                              */
    const double *key_xform;      /* [total keys][12] row-major 3x4            */
    uint32_t n_plight;
    const float *pl_pos;          /* [n_plight][3]                             */
    const float *pl_intensity;    /* [n_plight]                                */
    uint32_t width, height;
    double vfov_deg;
    uint32_t cam_nkeys;
    const double *cam_t;          /* [cam_nkeys]                               */
    const double *cam_elu;        /* [cam_nkeys][9] eye, look-at, up           */
    /* Environment seen by rays that leave the scene: a grey cube map of
     * env_res x env_res texels per face (0: black background), faces +x,
     * -x, +y, -y, +z, -z, texel (i, j) at env[(face * N + j) * N + i]. */
    uint32_t env_res;
    const float *env;
    /* Thin lens (0: pinhole): aperture radius and the distance of the plane
     * in focus along the viewing direction. */
    float lens_radius, focus_dist;
    /* RGB radiance (NULL: grey): per material albedo_rgb[n_mat][3] in
     * [0, 1) and emission_rgb[n_mat][3] >= 0, per point light
     * pl_rgb[n_plight][3] (NULL with RGB materials: the grey intensity in
     * every channel).  albedo / emission are then ignored. */
    const float *albedo_rgb, *emission_rgb, *pl_rgb;
} evo_scene_desc;

/* Luminance of linear RGB with the Rec. 709 primaries (ITU-R BT.709):
 * Y = 0.2126 R + 0.7152 G + 0.0722 B, FP32 in that order. */
float evo_luminance(float r, float g, float b);

typedef struct {
    uint64_t seed;
    uint32_t spp_init, spp_batch, spp_max;
    uint32_t max_depth, rr_start_depth, minibatch;
    double log_eps;
    float C, alpha;
    uint8_t nee, jitter, mode, df_mode, ref_mode;
    uint8_t mis;              /* 1: next-event estimation and BSDF sampling of
                                 emitters combined by the power heuristic    */
    uint32_t key_base;        /* frame index of instant 0 in the keys */
    float normality_alpha;    /* > 0: a pixel stops early only if neither
                                 instant's log-luminance samples reject
                                 normality (Jarque-Bera) at this level      */
} evo_params;

typedef struct {
    int8_t polarity;
    uint8_t decided_early;   /* 1 when the t-test stopped sampling        */
    uint8_t near_crit;       /* 1 when any executed decision was within
                                the exemption band of its critical value  */
    uint8_t pad;
    uint32_t n_paths;        /* paths traced per instant (reference holds
                                n_paths_ref in REF_FULL mode)             */
    uint32_t n_paths_ref;
    uint32_t rounds;
    double mean[2], var[2];  /* logL mean and unbiased variance           */
    double mean_radiance[2]; /* mean of the mini-batch radiance Y         */
    double t_last;
    double crit_margin;      /* min |t - critical value| over decisions   */
} evo_pixel_out;

typedef struct evo_scene evo_scene;
typedef struct evo_frame evo_frame;

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void evo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
float evo_u01(uint32_t x);

/* Student t distribution, FP64. */
double evo_ibeta(double a, double b, double x);
double evo_t_cdf(double t, double df);
double evo_t_ppf(double p, double df);

evo_scene *evo_scene_new(const evo_scene_desc *d);
void evo_scene_free(evo_scene *s);

/* Scene state at the two instants of one event frame. use_bvh=0 makes every
 * ray query brute force over all triangles. */
evo_frame *evo_frame_new(const evo_scene *s, double t0, double t1, int use_bvh);
void evo_frame_free(evo_frame *f);
uint32_t evo_frame_num_tris(const evo_frame *f);
void evo_frame_world_tris(const evo_frame *f, int instant, float *xyz9, uint32_t *mat);
void evo_frame_camera(const evo_frame *f, int instant, float *eye3, float *fwd3,
                      float *right3, float *up3, float *sxy2);

int evo_closest_hit(const evo_frame *f, int instant, const float o[3], const float d[3],
                    float tmin, float tmax, uint32_t skip, int brute,
                    float *t_out, uint32_t *prim_out);
int evo_any_hit(const evo_frame *f, int instant, const float o[3], const float d[3],
                float tmin, float tmax, uint32_t skip, int brute);
/* The two queries above for n rays (o, d: [n][3]; tmin, tmax, skip: [n]):
 * any = 0 stores the closest (t, primitive), any = 1 stores 1 or 0 in
 * prim_out (t_out unused). */
void evo_ray_queries(const evo_frame *f, int instant, uint32_t n, const float *o, const float *d,
                     const float *tmin, const float *tmax, const uint32_t *skip, int any, int brute,
                     float *t_out, uint32_t *prim_out);

float evo_path_radiance(const evo_frame *f, const evo_params *p, uint32_t pixel,
                        int instant, uint32_t sample);

/* The camera ray of one path sample (origin on the lens, unit direction). */
void evo_camera_ray(const evo_frame *f, const evo_params *p, uint32_t pixel, int instant,
                    uint32_t sample, float o[3], float d[3]);

/* Environment radiance in direction d (need not be unit length). */
float evo_env_radiance(const evo_frame *f, const float d[3]);

/* Record of one path for the derivatives of its radiance L with respect to
 * material albedos and emitted radiances, with every sampling decision
 * (light pick, Russian roulette, directions) held fixed: vertex k with
 * material vmat[k] and albedo a > 0 multiplies every term added after
 * vlb[k] (the radiance accumulated before its light samples), so
 * dL/da_j = sum over k with vmat[k] = j of (L - vlb[k]) / a_j; term k of
 * value tval[k] is proportional to the emitted radiance of material
 * tmat[k], so dL/dLe_e = sum over k with tmat[k] = e of tval[k] / Le_e. */
#define EVO_REC_MAX 64
typedef struct {
    uint32_t n_vert, n_term;
    uint32_t vmat[EVO_REC_MAX];
    float vlb[EVO_REC_MAX];
    uint32_t tmat[2 * EVO_REC_MAX];
    float tval[2 * EVO_REC_MAX];
} evo_path_rec;

float evo_path_radiance_rec(const evo_frame *f, const evo_params *p, uint32_t pixel,
                            int instant, uint32_t sample, evo_path_rec *rec);

/* Smoothed event loss of one pair at a fixed count of spp paths per pixel
 * and instant: Delta = mean_k ln(Y_k(t1) + eps) - mean_k ln(Y_k(t0) + eps)
 * over mini-batch means Y_k, loss = sum over the pixels of
 * softplus((|Delta| - C) / tau).  Its gradient with respect to every
 * material's albedo and emitted radiance by path replay (the derivative of
 * each path's radiance with its sampling decisions held fixed), all in
 * FP64.  pixels = NULL means every pixel.  Outputs may be NULL. */
int evo_event_loss(const evo_frame *f, const evo_params *p, double C, double tau, uint32_t spp,
                   const uint32_t *pixels, uint32_t n_pixels, int n_threads, double *loss,
                   double *grad_albedo, double *grad_emission, double *loss_px, double *delta_px);

/* Vector-Jacobian product through the per-pixel differences Delta above:
 * for weights g (one per listed pixel, the derivative dL/dDelta of an outer
 * function L) value = sum_p g_p Delta_p and its gradient with respect to
 * every material's albedo and emitted radiance, by the same path replay.
 * Outputs may be NULL. */
int evo_delta_vjp(const evo_frame *f, const evo_params *p, uint32_t spp, const double *g, const uint32_t *pixels,
                  uint32_t n_pixels, int n_threads, double *value, double *grad_albedo, double *grad_emission,
                  double *delta_px);

/* Sequential event video (Algorithm 1 over n_frames frames): pairs[k - 1]
 * is the frame of instants (t_{k-1}, t_k); frame 0 at spp_max is the first
 * reference of every pixel, frame k is sampled adaptively against the
 * pixel's reference and replaces it where it produces an event; frame k is
 * keyed key_base + k.  out: [(n_frames - 1) * n_pixels], frame-major. */
int evo_render_video(const evo_frame *const *pairs, uint32_t n_frames, const evo_params *p,
                     const uint32_t *pixels, uint32_t n_pixels, int n_threads, evo_pixel_out *out);

/* Decision on given logL sample sets (m0 samples at the reference instant,
 * m1 at the second): t of Eq. 7, its lower-tail p-value, the degrees of
 * freedom, the stop flag of `mode`, and (margin_out may be NULL) the
 * exemption margin of this test as a checkpoint before the last count. */
int evo_decide(const double *x0, uint32_t m0, const double *x1, uint32_t m1,
               float C, float alpha, int df_mode, int mode,
               double *t_out, double *p_out, double *df_out, int *stop_out, double *margin_out);

/* Jarque-Bera statistic of m samples: m/6 (g1^2 + g2^2 / 4), skewness g1
 * and excess kurtosis g2 from the population central moments; 0 when the
 * samples have no spread. */
double evo_jarque_bera(const double *x, uint32_t m);

/* Exemption margin of one executed decision (|t - critical value| for the
 * boundaries of `mode`; |t| for the event rule at the last count). */
double evo_crit_margin(int mode, double t, double df, float alpha, int final_check);

int evo_paths_batch(const evo_frame *f, const evo_params *p, uint32_t n, const uint32_t *pixel,
                    const uint8_t *instant, const uint32_t *sample, float *out, int n_threads);

int evo_render(const evo_frame *f, const evo_params *p, const uint32_t *pixels,
               uint32_t n_pixels, int n_threads, evo_pixel_out *out);

#ifdef __cplusplus
}
#endif
#endif
