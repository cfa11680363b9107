/*
 * evo_batch.c -- oracle: many independent path samples over a thread pool
 * (for per-path comparisons).  TEST INFRASTRUCTURE ONLY (see evo.h).
 */
#include "evo_internal.h"

#include <pthread.h>
#include <stdlib.h>
#include <unistd.h>

typedef struct {
    const evo_frame *f;
    const evo_params *p;
    uint32_t n;
    const uint32_t *pixel;
    const uint8_t *instant;
    const uint32_t *sample;
    float *out;
    uint32_t next;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *j = (batch_job *)arg;
    for (;;) {
        uint32_t k = __atomic_fetch_add(&j->next, 1u, __ATOMIC_RELAXED);
        if (k >= j->n) break;
        j->out[k] = evo_path_radiance(j->f, j->p, j->pixel[k], j->instant[k], j->sample[k]);
    }
    return NULL;
}

int evo_paths_batch(const evo_frame *f, const evo_params *p, uint32_t n, const uint32_t *pixel,
                    const uint8_t *instant, const uint32_t *sample, float *out, int n_threads)
{
    if (n_threads <= 0) n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads < 1) n_threads = 1;
    batch_job job = {f, p, n, pixel, instant, sample, out, 0u};
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)n_threads);
    for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, batch_worker, &job);
    for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
    free(th);
    return 0;
}
