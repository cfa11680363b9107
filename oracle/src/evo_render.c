/*
 * evo_render.c -- oracle: the per-path radiance estimator (tracePaths of
 * Algorithm 1) and the per-pixel adaptive sampling loop of Algorithm 1 for
 * one pair of instants.
 * TEST INFRASTRUCTURE ONLY (see evo.h).
 *
 * Readings of the paper taken here (the paper leaves these open):
 *   - grey (scalar) radiance, so luminance Y = radiance; or, as an option,
 *     linear RGB (Rec. 709 primaries) with the throughput carried per
 *     channel and each contribution reduced to its luminance
 *     Y = 0.2126 R + 0.7152 G + 0.0722 B when it is added to the path
 *     (luminance is linear, so the path's Y is the sum); emitters are then
 *     picked in proportion to A_j Y(Le_j) and Russian roulette survives
 *     with min(1, largest throughput channel); the environment stays grey;
 *   - next-event estimation to area emitters chosen with probability
 *     proportional to A_j * Le_j, without multiple importance sampling;
 *   - cosine-weighted Lambertian sampling and Russian roulette with
 *     survival probability min(1, beta) from a configurable depth;
 *   - the log of Eq. 3 is taken of the mean radiance of a mini-batch of
 *     paths plus a small epsilon, x_k = ln(Y_k + eps), so that zero-radiance
 *     paths do not produce -inf;
 *   - both instants are sampled in lock step (same count n) by default, or
 *     the first instant at the full count ("REF_FULL", Algorithm 1's first
 *     frame rendered at N_spp);
 *   - the first test runs at the initial count and then after every batch,
 *     with the batch clamped so the count never exceeds the maximum;
 *   - after sampling stops the event rule |mu_b - mu_a| > C (strict) gives
 *     polarity sign(mu_b - mu_a), at most one event per pixel per pair.
 */
#include "evo_internal.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define RAY_TMIN 1e-4f          /* self-intersection offset, scene units  */
#define SHADOW_SCALE 0.9999f    /* shadow segment stops short of the light */
#define INV_PI_F 0.318309886183790671538f
#define TWO_PI_D 6.283185307179586476925

/* Four random words of (pixel, sample, frame q = key_base + instant, vertex,
 * block): Philox counter (pixel, sample, (q mod 256) << 24 | vertex << 8 |
 * block, q >> 8). */
static void rng4(const evo_params *p, uint32_t pixel, uint32_t sample, int instant,
                 uint32_t vertex, uint32_t block, uint32_t out[4])
{
    const uint32_t q = p->key_base + (uint32_t)instant;
    uint32_t ctr[4] = {pixel, sample, ((q & 0xffu) << 24) | (vertex << 8) | block, q >> 8};
    uint32_t key[2] = {(uint32_t)(p->seed & 0xffffffffu), (uint32_t)(p->seed >> 32)};
    evo_philox4x32_10(ctr, key, out);
}

static float dot3(const float *a, const float *b)
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

/* Environment radiance: nearest texel of the cube map face of the major
 * axis of d (ties: x before y before z), in the usual cube-map face
 * coordinates (sc, tc) / |major|, mapped from [-1, 1] to [0, N) and
 * truncated; plain FP32 operations. */
float evo_env_radiance(const evo_frame *f, const float d[3])
{
    const evo_scene_desc *sd = &f->scene->d;
    const uint32_t N = sd->env_res;
    if (N == 0) return 0.0f;
    const float ax = fabsf(d[0]), ay = fabsf(d[1]), az = fabsf(d[2]);
    uint32_t face;
    float ma, sc, tc;
    if (ax >= ay && ax >= az) {
        ma = ax;
        face = d[0] >= 0.0f ? 0u : 1u;
        sc = d[0] >= 0.0f ? -d[2] : d[2];
        tc = -d[1];
    } else if (ay >= az) {
        ma = ay;
        face = d[1] >= 0.0f ? 2u : 3u;
        sc = d[0];
        tc = d[1] >= 0.0f ? d[2] : -d[2];
    } else {
        ma = az;
        face = d[2] >= 0.0f ? 4u : 5u;
        sc = d[2] >= 0.0f ? d[0] : -d[0];
        tc = -d[1];
    }
    if (!(ma > 0.0f)) return 0.0f;
    const float s = ((sc / ma) + 1.0f) * 0.5f;
    const float t = ((tc / ma) + 1.0f) * 0.5f;
    uint32_t i = (uint32_t)(s * (float)N), j = (uint32_t)(t * (float)N);
    if (i >= N) i = N - 1;
    if (j >= N) j = N - 1;
    return sd->env[((size_t)face * N + j) * N + i];
}

/* Camera ray of a path sample: pixel (x + u, y + v) with (u, v) from the
 * vertex-0 block (or the centre), pinhole direction f + a r + b u'; with a
 * thin lens the origin is the aperture point eye + rl cos(phi) r + rl
 * sin(phi) u', rl = R sqrt(u2), phi = 2 pi u3 (words 2 and 3 of the same
 * block), and the ray aims at eye + F (f + a r + b u'), the pinhole ray's
 * point on the plane in focus (its forward component is F). */
void evo_camera_ray(const evo_frame *f, const evo_params *p, uint32_t pixel, int instant,
                    uint32_t sample, float o[3], float d[3])
{
    const evo_scene_desc *sd = &f->scene->d;
    const evo_instant *I = &f->inst[instant];
    const uint32_t W = sd->width, H = sd->height;
    const uint32_t px = pixel % W, py = pixel / W;
    uint32_t r[4] = {0, 0, 0, 0};
    const int lens = sd->lens_radius > 0.0f;
    if (p->jitter || lens) rng4(p, pixel, sample, instant, 0, 0, r);
    float j0 = 0.5f, j1 = 0.5f;
    if (p->jitter) {
        j0 = evo_u01(r[0]);
        j1 = evo_u01(r[1]);
    }
    float fx = (float)px + j0, fy = (float)py + j1;
    float nx = (2.0f * fx) / (float)W - 1.0f;
    float ny = 1.0f - (2.0f * fy) / (float)H;
    float a = nx * I->sx, b = ny * I->sy;
    for (int c = 0; c < 3; ++c) {
        d[c] = (I->fwd[c] + a * I->right[c]) + b * I->up[c];
        o[c] = I->eye[c];
    }
    if (lens) {
        const float rl = sd->lens_radius * sqrtf(evo_u01(r[2]));
        const double ph = TWO_PI_D * (double)evo_u01(r[3]);
        const float lu = rl * (float)cos(ph), lv = rl * (float)sin(ph);
        for (int c = 0; c < 3; ++c) {
            const float focus = I->eye[c] + sd->focus_dist * d[c];
            o[c] = (I->eye[c] + lu * I->right[c]) + lv * I->up[c];
            d[c] = focus - o[c];
        }
    }
    float len = sqrtf((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    for (int c = 0; c < 3; ++c) d[c] = d[c] / len;
}

/* Radiance carried by one camera path, FP32.  Vertex d = 1..max_depth is
 * the d-th surface hit.  Random numbers come from Philox keyed by (pixel,
 * sample, instant, vertex, block): vertex 0 block 0 gives the pixel jitter;
 * vertex d block 0 gives (light pick, two light-point numbers, roulette);
 * vertex d block 1 gives the two direction numbers. */
static float path_radiance(const evo_frame *f, const evo_params *p, uint32_t pixel, int instant,
                           uint32_t sample, evo_path_rec *rec)
{
    const evo_scene_desc *sd = &f->scene->d;
    const evo_instant *I = &f->inst[instant];
    const int brute = !f->use_bvh;

    float d[3], o[3];
    evo_camera_ray(f, p, pixel, instant, sample, o, d);

    /* RGB radiance: the throughput per channel (b3), every contribution
     * reduced to its luminance when it is added to L. */
    const int rgb = sd->albedo_rgb != NULL;
    float L = 0.0f, beta = 1.0f;
    float b3[3] = {1.0f, 1.0f, 1.0f};
    float pb_prev = 0.0f; /* solid-angle pdf of the direction sampled at the
                             previous vertex (cosine: cos / pi) */
    uint32_t skip = EVO_NO_PRIM;
    if (rec) {
        rec->n_vert = 0;
        rec->n_term = 0;
    }
    for (uint32_t depth = 1; depth <= p->max_depth; ++depth) {
        evo_ray ray;
        evo__ray_setup(&ray, o, d);
        float t;
        uint32_t prim;
        if (!evo__closest(f, instant, &ray, RAY_TMIN, INFINITY, skip, brute, &t, &prim)) {
            /* Leaves the scene: the environment's radiance (found by this
             * direction only; light samples do not sample it). */
            if (sd->env_res) {
                const float Lenv = evo_env_radiance(f, d);
                if (rgb) L = L + evo_luminance(b3[0] * Lenv, b3[1] * Lenv, b3[2] * Lenv);
                else L = L + beta * Lenv;
            }
            break;
        }
        float P[3];
        for (int c = 0; c < 3; ++c) P[c] = o[c] + t * d[c];
        const float *n = I->nrm + 3 * (size_t)prim;
        const uint32_t m = I->mat[prim];
        const float *alb3 = rgb ? sd->albedo_rgb + 3 * (size_t)m : NULL;
        const float *Le3 = rgb ? sd->emission_rgb + 3 * (size_t)m : NULL;
        /* Grey: albedo and emission; RGB: the largest albedo channel (the
         * surface reflects when it is > 0) and the luminance of the
         * emission. */
        const float alb = rgb ? fmaxf(alb3[0], fmaxf(alb3[1], alb3[2])) : sd->albedo[m];
        const float Le = rgb ? evo_luminance(Le3[0], Le3[1], Le3[2]) : sd->emission[m];
        const float cosi = dot3(n, d);
        float ns[3];
        for (int c = 0; c < 3; ++c) ns[c] = cosi < 0.0f ? n[c] : -n[c];

        /* Emission of a front-facing emitter: at the first vertex, or at
         * every vertex without next-event estimation.  With MIS, a later
         * vertex reached by BSDF sampling adds it too, weighted by the power
         * heuristic against the pdf with which next-event estimation would
         * have sampled this point, in solid angle at the previous vertex:
         * p_light = P_j / A_j * r^2 / cos_y = Le r^2 / (S cos_y). */
        if (Le > 0.0f && cosi < 0.0f && (depth == 1 || !p->nee || p->mis)) {
            float term = rgb ? evo_luminance(b3[0] * Le3[0], b3[1] * Le3[1], b3[2] * Le3[2]) : beta * Le;
            if (depth > 1 && p->nee) {
                const float pl = (Le * (t * t)) / (I->emit_S * (-cosi));
                const float ratio = pl / pb_prev;
                term = term * (1.0f / (1.0f + ratio * ratio));
            }
            L = L + term;
            if (rec) {
                rec->tmat[rec->n_term] = m;
                rec->tval[rec->n_term++] = term;
            }
        }
        if (!(alb > 0.0f)) break;
        /* Every term added from here on carries the factor a of this
         * vertex (the BRDF of its light samples, the throughput of its
         * continuation). */
        if (rec) {
            rec->vmat[rec->n_vert] = m;
            rec->vlb[rec->n_vert++] = L;
        }

        uint32_t r0[4];
        rng4(p, pixel, sample, instant, depth, 0, r0);
        const float fr = alb * INV_PI_F; /* Lambertian BRDF a / pi */
        float fr3[3] = {0.0f, 0.0f, 0.0f};
        if (rgb)
            for (int c = 0; c < 3; ++c) fr3[c] = alb3[c] * INV_PI_F;

        if (p->nee) {
            float Dd = 0.0f;
            if (I->n_emit > 0) {
                const float ul = evo_u01(r0[0]);
                uint32_t j = 0;
                while (j + 1 < I->n_emit && !(ul < I->emit_cdf[j])) ++j;
                const uint32_t q = I->emit_prim[j];
                const float *v = I->tri + 9 * (size_t)q;
                const float *nq = I->nrm + 3 * (size_t)q;
                /* Uniform point on the triangle (Osada et al. 2002). */
                const float su = sqrtf(evo_u01(r0[1]));
                const float u2 = evo_u01(r0[2]);
                const float w0 = 1.0f - su, w1 = su * (1.0f - u2), w2 = su * u2;
                float wv[3];
                for (int c = 0; c < 3; ++c) {
                    float y = (w0 * v[c] + w1 * v[3 + c]) + w2 * v[6 + c];
                    wv[c] = y - P[c];
                }
                const float r2 = dot3(wv, wv);
                if (r2 > 0.0f) {
                    const float rl = sqrtf(r2);
                    float wi[3] = {wv[0] / rl, wv[1] / rl, wv[2] / rl};
                    const float cx = dot3(ns, wi);
                    const float cy = -dot3(nq, wi);
                    if (cx > 0.0f && cy > 0.0f) {
                        evo_ray sr;
                        evo__ray_setup(&sr, P, wi);
                        if (!evo__any(f, instant, &sr, RAY_TMIN, rl * SHADOW_SCALE, prim, brute)) {
                            /* beta * (a/pi) * Le_j * cx * cy / r^2 / (P_j / A_j)
                             * with P_j = A_j Le_j / S, i.e. the emitter terms
                             * collapse to S. */
                            float cval;
                            if (rgb) {
                                /* Per channel the grey estimate times
                                 * Le_j,c / Y(Le_j): the emitter was picked
                                 * in proportion to A_j Y(Le_j). */
                                const float *Lq = sd->emission_rgb + 3 * (size_t)I->mat[q];
                                const float Yq = evo_luminance(Lq[0], Lq[1], Lq[2]);
                                float c3[3];
                                for (int c = 0; c < 3; ++c)
                                    c3[c] = (((((b3[c] * fr3[c]) * (Lq[c] / Yq)) * cx) * cy) * I->emit_S) / r2;
                                cval = evo_luminance(c3[0], c3[1], c3[2]);
                            } else {
                                cval = ((((beta * fr) * cx) * cy) * I->emit_S) / r2;
                            }
                            if (p->mis && depth < p->max_depth) {
                                /* Power heuristic against the cosine-sampling
                                 * pdf of the same direction; the last vertex
                                 * samples no direction, so its light sample
                                 * keeps the full weight. */
                                const float Lej = evo__emission_y(sd, I->mat[q]);
                                const float pl = (Lej * r2) / (I->emit_S * cy);
                                const float ratio = (cx * INV_PI_F) / pl;
                                cval = cval * (1.0f / (1.0f + ratio * ratio));
                            }
                            Dd = Dd + cval;
                            if (rec) {
                                rec->tmat[rec->n_term] = f->inst[instant].mat[q];
                                rec->tval[rec->n_term++] = cval;
                            }
                        }
                    }
                }
            }
            for (uint32_t k = 0; k < sd->n_plight; ++k) {
                const float *lp = sd->pl_pos + 3 * (size_t)k;
                float wv[3] = {lp[0] - P[0], lp[1] - P[1], lp[2] - P[2]};
                const float r2 = dot3(wv, wv);
                if (!(r2 > 0.0f)) continue;
                const float rl = sqrtf(r2);
                float wi[3] = {wv[0] / rl, wv[1] / rl, wv[2] / rl};
                const float cx = dot3(ns, wi);
                if (!(cx > 0.0f)) continue;
                evo_ray sr;
                evo__ray_setup(&sr, P, wi);
                if (evo__any(f, instant, &sr, RAY_TMIN, rl * SHADOW_SCALE, prim, brute)) continue;
                float cval;
                if (rgb) {
                    float c3[3];
                    for (int c = 0; c < 3; ++c) {
                        const float Ik = sd->pl_rgb ? sd->pl_rgb[3 * (size_t)k + c] : sd->pl_intensity[k];
                        c3[c] = (((b3[c] * fr3[c]) * Ik) * cx) / r2;
                    }
                    cval = evo_luminance(c3[0], c3[1], c3[2]);
                } else {
                    cval = (((beta * fr) * sd->pl_intensity[k]) * cx) / r2;
                }
                Dd = Dd + cval;
            }
            L = L + Dd;
        }
        if (depth == p->max_depth) break;
        if (depth >= p->rr_start_depth) {
            /* RGB: survival min(1, largest throughput channel). */
            const float q = fminf(1.0f, rgb ? fmaxf(b3[0], fmaxf(b3[1], b3[2])) : beta);
            if (evo_u01(r0[3]) >= q) break;
            beta = beta / q;
            if (rgb)
                for (int c = 0; c < 3; ++c) b3[c] = b3[c] / q;
        }

        /* Cosine-weighted direction about ns; sin/cos are the correctly
         * rounded FP32 values, obtained from FP64 evaluation. */
        uint32_t r1[4];
        rng4(p, pixel, sample, instant, depth, 1, r1);
        const float e0 = evo_u01(r1[0]), e1 = evo_u01(r1[1]);
        const float rr = sqrtf(e0);
        const double ph = TWO_PI_D * (double)e1;
        const float cph = (float)cos(ph), sph = (float)sin(ph);
        const float lx = rr * cph, ly = rr * sph, lz = sqrtf(fmaxf(0.0f, 1.0f - e0));
        pb_prev = lz * INV_PI_F;
        /* Orthonormal basis of Duff et al. 2017. */
        const float sg = copysignf(1.0f, ns[2]);
        const float aa = -1.0f / (sg + ns[2]);
        const float bb = (ns[0] * ns[1]) * aa;
        const float T[3] = {1.0f + ((sg * ns[0]) * ns[0]) * aa, sg * bb, (-sg) * ns[0]};
        const float B[3] = {bb, sg + (ns[1] * ns[1]) * aa, -ns[1]};
        for (int c = 0; c < 3; ++c) {
            d[c] = (T[c] * lx + B[c] * ly) + ns[c] * lz;
            o[c] = P[c];
        }
        beta = beta * alb;
        if (rgb)
            for (int c = 0; c < 3; ++c) b3[c] = b3[c] * alb3[c];
        skip = prim;
    }
    return L;
}

float evo_path_radiance(const evo_frame *f, const evo_params *p, uint32_t pixel,
                        int instant, uint32_t sample)
{
    return path_radiance(f, p, pixel, instant, sample, NULL);
}

float evo_path_radiance_rec(const evo_frame *f, const evo_params *p, uint32_t pixel,
                            int instant, uint32_t sample, evo_path_rec *rec)
{
    if (p->max_depth > EVO_REC_MAX) return NAN;
    return path_radiance(f, p, pixel, instant, sample, rec);
}

/* Mean of a power-of-two mini-batch by a pairwise sum tree, FP32. */
static float pair_sum(const float *v, uint32_t n)
{
    if (n == 1) return v[0];
    return pair_sum(v, n / 2) + pair_sum(v + n / 2, n / 2);
}

static float minibatch_mean(const float *v, uint32_t mb)
{
    return pair_sum(v, mb) * (1.0f / (float)mb);
}

typedef struct {
    float *L[2];
    double *x[2];
    double *y[2];
} pixel_scratch;

/* Algorithm 1 for one pixel and one pair of instants.  ref_n > 0: the
 * first instant's samples are already in ws->x[0] / ws->y[0], ref_n paths
 * of them (a carried reference), and are not sampled further. */
static void render_pixel(const evo_frame *f, const evo_params *p, uint32_t pixel,
                         pixel_scratch *ws, evo_pixel_out *o, uint32_t ref_n)
{
    const uint32_t mb = p->minibatch;
    const int full_ref = ref_n > 0 || p->ref_mode == EVO_REF_FULL;
    const int fixed = p->mode == EVO_MODE_FIXED;
    uint32_t n_prev[2] = {ref_n, 0};
    uint32_t n1 = fixed ? p->spp_max : p->spp_init;
    double margin = INFINITY, norm_margin = INFINITY;
    double mean[2] = {0, 0}, var[2] = {0, 0}, t = 0.0, df = 0.0, pl = 0.0;
    int stop = 0;
    uint32_t rounds = 0;
    memset(o, 0, sizeof(*o));

    for (;;) {
        uint32_t target[2] = {ref_n > 0 ? ref_n : (full_ref ? p->spp_max : n1), n1};
        for (int i = 0; i < 2; ++i) {
            for (uint32_t s = n_prev[i]; s < target[i]; ++s)
                ws->L[i][s] = evo_path_radiance(f, p, pixel, i, s);
            for (uint32_t k = n_prev[i] / mb; k < target[i] / mb; ++k) {
                float Y = minibatch_mean(ws->L[i] + (size_t)k * mb, mb);
                ws->y[i][k] = (double)Y;
                ws->x[i][k] = log((double)Y + p->log_eps);
            }
            n_prev[i] = target[i];
        }
        ++rounds;
        const uint32_t m0 = target[0] / mb, m1 = target[1] / mb;
        evo__stats_decide(ws->x[0], m0, ws->x[1], m1, p, mean, var, &t, &df, &pl, &stop, &norm_margin);
        const int final_check = n1 >= p->spp_max;
        const double mg = evo_crit_margin(p->mode, t, df, p->alpha, final_check);
        if (mg < margin) margin = mg;
        if (final_check) {
            /* Final event rule |gap| > C, i.e. t > 0. */
            stop = 0;
            break;
        }
        if (stop) break;
        n1 = n1 + p->spp_batch < p->spp_max ? n1 + p->spp_batch : p->spp_max;
    }

    const double gap = mean[1] - mean[0];
    o->polarity = fabs(gap) > (double)p->C ? (gap > 0.0 ? 1 : -1) : 0;
    o->decided_early = (uint8_t)stop;
    /* Exempt: a t within 1e-4 of a critical value, or a normality
     * statistic within 1e-6 (relative) of its critical value. */
    o->near_crit = (margin < 1e-4 || norm_margin < 1e-6) ? 1 : 0;
    o->n_paths = n_prev[1];
    o->n_paths_ref = n_prev[0];
    o->rounds = rounds;
    for (int i = 0; i < 2; ++i) {
        o->mean[i] = mean[i];
        o->var[i] = var[i];
        const uint32_t m = n_prev[i] / mb;
        double s = 0.0;
        for (uint32_t k = 0; k < m; ++k) s += ws->y[i][k];
        o->mean_radiance[i] = s / (double)m;
    }
    o->t_last = t;
    o->crit_margin = margin;
}

typedef struct {
    const evo_frame *f;
    const evo_params *p;
    const uint32_t *pixels;
    uint32_t n_pixels;
    evo_pixel_out *out;
    uint32_t next; /* shared work counter */
} render_job;

static void *render_worker(void *arg)
{
    render_job *job = (render_job *)arg;
    const evo_params *p = job->p;
    pixel_scratch ws;
    const uint32_t mmax = p->spp_max / p->minibatch;
    for (int i = 0; i < 2; ++i) {
        ws.L[i] = (float *)malloc(sizeof(float) * p->spp_max);
        ws.x[i] = (double *)malloc(sizeof(double) * mmax);
        ws.y[i] = (double *)malloc(sizeof(double) * mmax);
    }
    for (;;) {
        uint32_t k = __atomic_fetch_add(&job->next, 1u, __ATOMIC_RELAXED);
        if (k >= job->n_pixels) break;
        render_pixel(job->f, p, job->pixels[k], &ws, &job->out[k], 0u);
    }
    for (int i = 0; i < 2; ++i) { free(ws.L[i]); free(ws.x[i]); free(ws.y[i]); }
    return NULL;
}

int evo_render(const evo_frame *f, const evo_params *p, const uint32_t *pixels,
               uint32_t n_pixels, int n_threads, evo_pixel_out *out)
{
    const uint32_t mb = p->minibatch;
    if (mb == 0 || (mb & (mb - 1)) != 0) return -1;
    if (p->spp_init % mb || p->spp_batch % mb || p->spp_max % mb) return -1;
    if (p->spp_init < 2 * mb || p->spp_init > p->spp_max || p->spp_batch == 0) return -1;
    const uint32_t npx = f->scene->d.width * f->scene->d.height;
    for (uint32_t k = 0; k < n_pixels; ++k)
        if (pixels[k] >= npx) return -1;
    if (n_threads <= 0) n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads < 1) n_threads = 1;
    render_job job = {f, p, pixels, n_pixels, out, 0u};
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, render_worker, &job);
    for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
    free(th);
    return 0;
}

/* Sequential event video (Algorithm 1 over frames t_0 ... t_{n-1}): frame 0
 * at the full count is every pixel's first reference; frame k >= 1 is
 * sampled adaptively against the pixel's reference (the first instant held
 * at the full count, as in REF_FULL) and, where it produces an event,
 * becomes the pixel's reference.  Frame k is keyed key_base + k.
 * pairs[k - 1] holds the instants (t_{k-1}, t_k).  out is frame-major:
 * out[(k - 1) * n_pixels + i]. */
typedef struct {
    const evo_frame *const *pairs;
    uint32_t n_frames;
    const evo_params *p;
    const uint32_t *pixels;
    uint32_t n_pixels;
    evo_pixel_out *out;
    uint32_t next;
} video_job;

static void *video_worker(void *arg)
{
    video_job *job = (video_job *)arg;
    const evo_params *p = job->p;
    pixel_scratch ws;
    const uint32_t mmax = p->spp_max / p->minibatch;
    for (int i = 0; i < 2; ++i) {
        ws.L[i] = (float *)malloc(sizeof(float) * p->spp_max);
        ws.x[i] = (double *)malloc(sizeof(double) * mmax);
        ws.y[i] = (double *)malloc(sizeof(double) * mmax);
    }
    for (;;) {
        uint32_t i = __atomic_fetch_add(&job->next, 1u, __ATOMIC_RELAXED);
        if (i >= job->n_pixels) break;
        /* Paths in the pixel's reference: 0 before frame 0 is rendered (the
         * first pair renders it at the full count). */
        uint32_t ref_n = 0;
        for (uint32_t k = 1; k < job->n_frames; ++k) {
            evo_params pk = *p;
            pk.ref_mode = EVO_REF_FULL;
            pk.key_base = p->key_base + k - 1;
            evo_pixel_out *o = &job->out[(size_t)(k - 1) * job->n_pixels + i];
            render_pixel(job->pairs[k - 1], &pk, job->pixels[i], &ws, o, ref_n);
            ref_n = o->n_paths_ref;
            if (o->polarity != 0) {
                /* The frame's samples up to its stop become the reference
                 * (a two-tailed test can fire before spp_max). */
                const uint32_t m = o->n_paths / p->minibatch;
                memcpy(ws.x[0], ws.x[1], sizeof(double) * m);
                memcpy(ws.y[0], ws.y[1], sizeof(double) * m);
                ref_n = o->n_paths;
            }
        }
    }
    for (int i = 0; i < 2; ++i) { free(ws.L[i]); free(ws.x[i]); free(ws.y[i]); }
    return NULL;
}

int evo_render_video(const evo_frame *const *pairs, uint32_t n_frames, const evo_params *p,
                     const uint32_t *pixels, uint32_t n_pixels, int n_threads, evo_pixel_out *out)
{
    const uint32_t mb = p->minibatch;
    if (n_frames < 2) return -1;
    if (mb == 0 || (mb & (mb - 1)) != 0) return -1;
    if (p->spp_init % mb || p->spp_batch % mb || p->spp_max % mb) return -1;
    if (p->spp_init < 2 * mb || p->spp_init > p->spp_max || p->spp_batch == 0) return -1;
    const uint32_t npx = pairs[0]->scene->d.width * pairs[0]->scene->d.height;
    for (uint32_t k = 0; k < n_pixels; ++k)
        if (pixels[k] >= npx) return -1;
    if (n_threads <= 0) n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads < 1) n_threads = 1;
    video_job job = {pairs, n_frames, p, pixels, n_pixels, out, 0u};
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, video_worker, &job);
    for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
    free(th);
    return 0;
}
