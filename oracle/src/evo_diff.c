/*
 * evo_diff.c -- oracle: a smoothed event loss of one pair of instants and
 * its gradient with respect to material albedos and emitted radiances.
 * TEST INFRASTRUCTURE ONLY (see evo.h).
 *
 * The loss follows the event statistic of the paper (Eq. 3 and 7, the
 * difference of the mean log-luminance of the two instants against the
 * threshold C of Eq. 1), smoothed so that it has a gradient:
 *   x_{i,k} = ln(Y_{i,k} + eps), Y_{i,k} the mean of mini-batch k of the
 *             paths at instant i (FP32, as the renderer computes it),
 *   mu_i    = (1/m) sum_k x_{i,k}   (FP64, k ascending),
 *   Delta   = mu_1 - mu_0,
 *   loss    = sum over pixels of softplus((|Delta| - C) / tau).
 * Gradient by the chain rule, with each path's radiance differentiated by
 * replaying it from its random-number keys with every sampling decision
 * held fixed (evo_path_rec in evo.h):
 *   dloss/dtheta = sum_px sigmoid(z)/tau * sign(Delta) * (dmu_1 - dmu_0),
 *   dmu_i        = (1/m) sum_k (1/(Y_{i,k} + eps)) (1/mb) sum_{s in k} dL_s.
 * Gradients are reported for materials with albedo > 0 (albedo) and with
 * emission > 0 (emission); the sampler never produces the other terms.
 *
 * The same replay gives the gradient of any outer function of the
 * per-pixel differences: with caller weights g_p = dL/dDelta_p the
 * "loss" is sum_p g_p Delta_p and sigmoid(z)/tau * sign(Delta) above is
 * replaced by g_p (evo_delta_vjp).
 */
#include "evo_internal.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

static double softplus(double z) { return z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z)); }

static double sigmoid(double z)
{
    if (z >= 0.0) return 1.0 / (1.0 + exp(-z));
    const double e = exp(z);
    return e / (1.0 + e);
}

/* Mean of a power-of-two mini-batch (FP32 pairwise tree), the same
 * summation order as the adaptive loop. */
static float mb_mean(const float *v, uint32_t mb)
{
    if (mb == 1) return v[0];
    if (mb == 2) return (v[0] + v[1]) * 0.5f;
    if (mb == 4) return ((v[0] + v[1]) + (v[2] + v[3])) * 0.25f;
    return (((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]))) * 0.125f;
}

typedef struct {
    const evo_frame *f;
    const evo_params *p;
    double C, tau;
    const double *upstream;    /* per listed pixel dL/dDelta, or NULL: the smoothed loss */
    uint32_t spp;
    const uint32_t *pixels;
    uint32_t n_pixels;
    uint32_t next;
    pthread_mutex_t lock;
    double loss;
    double *ga, *ge;           /* shared sums, under lock */
    double *loss_px, *delta_px;
} diff_job;

static void *diff_worker(void *arg)
{
    diff_job *j = (diff_job *)arg;
    const evo_scene_desc *sd = &j->f->scene->d;
    const uint32_t nm = sd->n_mat, spp = j->spp, mb = j->p->minibatch, m = spp / mb;
    double *ga = (double *)calloc(2 * (size_t)nm, sizeof(double));
    double *ge = ga + nm;
    float *L = (float *)malloc(sizeof(float) * 2 * (size_t)spp);
    float *Y = (float *)malloc(sizeof(float) * 2 * (size_t)m);
    evo_path_rec rec;
    double loss = 0.0;
    for (;;) {
        const uint32_t k = __atomic_fetch_add(&j->next, 1u, __ATOMIC_RELAXED);
        if (k >= j->n_pixels) break;
        const uint32_t pixel = j->pixels ? j->pixels[k] : k;
        double mu[2];
        for (int i = 0; i < 2; ++i) {
            for (uint32_t s = 0; s < spp; ++s) L[i * spp + s] = evo_path_radiance(j->f, j->p, pixel, i, s);
            double sum = 0.0;
            for (uint32_t b = 0; b < m; ++b) {
                const float y = mb_mean(L + i * spp + b * mb, mb);
                Y[i * m + b] = y;
                sum += log((double)y + j->p->log_eps);
            }
            mu[i] = sum / (double)m;
        }
        const double delta = mu[1] - mu[0];
        double g;
        if (j->upstream) {
            g = j->upstream[k];
            loss += g * delta;
            if (j->loss_px) j->loss_px[k] = g * delta;
        } else {
            const double z = (fabs(delta) - j->C) / j->tau;
            loss += softplus(z);
            if (j->loss_px) j->loss_px[k] = softplus(z);
            const double sgn = delta > 0.0 ? 1.0 : (delta < 0.0 ? -1.0 : 0.0);
            g = sigmoid(z) / j->tau * sgn;
        }
        if (j->delta_px) j->delta_px[k] = delta;
        if (g == 0.0) continue;
        for (int i = 0; i < 2; ++i) {
            for (uint32_t s = 0; s < spp; ++s) {
                const double w = (i ? g : -g) / (double)m / (double)mb /
                                 ((double)Y[i * m + s / mb] + j->p->log_eps);
                const float Lp = evo_path_radiance_rec(j->f, j->p, pixel, i, s, &rec);
                for (uint32_t v = 0; v < rec.n_vert; ++v) {
                    const uint32_t mat = rec.vmat[v];
                    ga[mat] += w * ((double)Lp - (double)rec.vlb[v]) / (double)sd->albedo[mat];
                }
                for (uint32_t t = 0; t < rec.n_term; ++t) {
                    const uint32_t mat = rec.tmat[t];
                    ge[mat] += w * (double)rec.tval[t] / (double)sd->emission[mat];
                }
            }
        }
    }
    pthread_mutex_lock(&j->lock);
    j->loss += loss;
    for (uint32_t q = 0; q < nm; ++q) {
        j->ga[q] += ga[q];
        j->ge[q] += ge[q];
    }
    pthread_mutex_unlock(&j->lock);
    free(ga);
    free(L);
    free(Y);
    return NULL;
}

static int loss_grad(const evo_frame *f, const evo_params *p, double C, double tau, const double *upstream,
                     uint32_t spp, const uint32_t *pixels, uint32_t n_pixels, int n_threads, double *loss,
                     double *grad_albedo, double *grad_emission, double *loss_px, double *delta_px)
{
    const evo_scene_desc *sd = &f->scene->d;
    const uint32_t mb = p->minibatch;
    if (mb != 1 && mb != 2 && mb != 4 && mb != 8) return -1;
    if (spp == 0 || spp % mb != 0 || p->max_depth > EVO_REC_MAX) return -1;
    if (!upstream && !(tau > 0.0)) return -1;
    if (p->mis) return -1; /* the gradient follows the estimator without MIS */
    if (f->scene->d.albedo_rgb) return -1; /* ... and with grey radiance */
    if (!pixels) n_pixels = sd->width * sd->height;
    if (n_threads <= 0) n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads < 1) n_threads = 1;
    diff_job job;
    memset(&job, 0, sizeof(job));
    job.f = f;
    job.p = p;
    job.C = C;
    job.tau = tau;
    job.upstream = upstream;
    job.spp = spp;
    job.pixels = pixels;
    job.n_pixels = n_pixels;
    job.ga = (double *)calloc(2 * (size_t)sd->n_mat, sizeof(double));
    job.ge = job.ga + sd->n_mat;
    job.loss_px = loss_px;
    job.delta_px = delta_px;
    pthread_mutex_init(&job.lock, NULL);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, diff_worker, &job);
    for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
    free(th);
    pthread_mutex_destroy(&job.lock);
    if (loss) *loss = job.loss;
    if (grad_albedo) memcpy(grad_albedo, job.ga, sizeof(double) * sd->n_mat);
    if (grad_emission) memcpy(grad_emission, job.ge, sizeof(double) * sd->n_mat);
    free(job.ga);
    return 0;
}

int evo_event_loss(const evo_frame *f, const evo_params *p, double C, double tau, uint32_t spp,
                   const uint32_t *pixels, uint32_t n_pixels, int n_threads, double *loss,
                   double *grad_albedo, double *grad_emission, double *loss_px, double *delta_px)
{
    return loss_grad(f, p, C, tau, NULL, spp, pixels, n_pixels, n_threads, loss, grad_albedo, grad_emission,
                     loss_px, delta_px);
}

int evo_delta_vjp(const evo_frame *f, const evo_params *p, uint32_t spp, const double *g, const uint32_t *pixels,
                  uint32_t n_pixels, int n_threads, double *value, double *grad_albedo, double *grad_emission,
                  double *delta_px)
{
    if (!g) return -1;
    return loss_grad(f, p, 0.0, 1.0, g, spp, pixels, n_pixels, n_threads, value, grad_albedo, grad_emission,
                     NULL, delta_px);
}
