/*
 * evrt.h -- C ABI of the MI355X (gfx950) adaptive event-camera path tracer.
 *
 * Implements the method of "Monte Carlo Path Tracing and Statistical Event
 * Detection for Event Camera Simulation" (arXiv 2408.07996) for one pair of
 * time instants per call: every pixel is path traced at instants t0 and t1,
 * the log-luminance of 4-path mini-batches is accumulated per pixel and
 * instant (Eq. 3-4), and a pixel keeps being sampled only until the
 * one-tailed t-test of Eq. 7 (Sec. 3.2, Sec. 3.3, Algorithm 1) decides that
 * |mean logL(t1) - mean logL(t0)| is significantly below the event
 * threshold C, or the maximum sample count is reached; then the event rule
 * of Algorithm 1 (|gap| > C, polarity = sign(gap)) is applied.
 *
 * Conventions (all entry points):
 *   - Every function returns an int status: EVRT_OK (0) or a negative
 *     EVRT_E_* code.  No C++ exception crosses this boundary.  On failure
 *     evrt_last_error() describes the cause.
 *   - Argument errors are detected on the host before any device work is
 *     enqueued.  HIP runtime failures are reported as EVRT_E_DEVICE.
 *   - Host arrays passed to scene functions are deep-copied; the caller
 *     keeps ownership and may free them when the call returns.
 *   - Output pointers of render calls are caller-allocated DEVICE memory on
 *     the context's device, row-major pixels (pixel = y * width + x, y = 0
 *     at the top of the image).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Render calls enqueue their kernels on it and return after the work
 *     they enqueued has completed (they read per-round active counts).
 *   - A context belongs to one device and must not be used from two host
 *     threads at once.
 */
#ifndef EVRT_H
#define EVRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EVRT_ABI_VERSION 7

enum {
    EVRT_OK = 0,
    EVRT_E_INVALID = -1,     /* bad argument or inconsistent scene            */
    EVRT_E_NOMEM = -2,       /* host or device allocation failed              */
    EVRT_E_DEVICE = -3,      /* HIP runtime error or no device in the context */
    EVRT_E_STATE = -4,       /* call out of order (e.g. render before commit) */
    EVRT_E_UNSUPPORTED = -5  /* valid request that the library does not serve */
};

/* Sampling modes (Sec. 3.2 and its ablation). */
enum {
    EVRT_MODE_ADAPTIVE_1T = 0, /* stop when p_lower(t) < alpha: no event         */
    EVRT_MODE_FIXED = 1,       /* trace spp_max everywhere (the baseline, Sec. 4) */
    EVRT_MODE_ADAPTIVE_2T = 2, /* stop on either tail at alpha/2                  */
    EVRT_MODE_MEAN_ONLY = 3    /* stop once |gap| <= C                            */
};
/* Degrees of freedom of the t-test (the paper states none, Sec. 3.2):
 * STUDENT = pooled m0 + m1 - 2 (m0, m1 = mini-batches per instant; with
 * equal counts Eq. 7 is then the pooled two-sample t statistic), compared
 * with critical values of the schedule's counts.  WELCH = Welch-Satterthwaite
 * for the variance estimate (s0^2 + s1^2) / m1 of Eq. 7,
 * df = (s0^2 + s1^2)^2 / (s0^4 / (m0 - 1) + s1^4 / (m1 - 1)) (the pooled
 * value when both variances are 0), real-valued and per pixel: each pixel
 * compares its own lower-tail probability, from an FP64 Student t
 * distribution function evaluated on the device, with alpha. */
enum { EVRT_DF_STUDENT = 0, EVRT_DF_WELCH = 1 };
/* LOCKSTEP: both instants hold the same sample count.  REF_FULL: the first
 * instant is rendered at spp_max and only the second one is adaptive (the
 * first frame of Algorithm 1 is rendered at the full count). */
enum { EVRT_REF_LOCKSTEP = 0, EVRT_REF_FULL = 1 };

typedef struct evrt_ctx evrt_ctx;

/* Returns EVRT_ABI_VERSION. */
int evrt_abi_version(void);

/* Creates a context on HIP device `hip_device` (>= 0).  hip_device = -1
 * creates a host-only context: scene calls and argument validation work,
 * anything that needs the device returns EVRT_E_DEVICE.  *out receives the
 * context (NULL on failure). */
int evrt_create(int hip_device, evrt_ctx **out);
void evrt_destroy(evrt_ctx *ctx);

/* Message of the last failure on ctx (or of the last evrt_create failure on
 * this thread when ctx is NULL).  Valid until the next call on ctx. */
const char *evrt_last_error(const evrt_ctx *ctx);

/* ---- Scene --------------------------------------------------------------
 * Grey Lambertian materials: albedo in [0, 1), emitted radiance >= 0.  An
 * emitter radiates from its front side only (front = the side toward which
 * cross(v1 - v0, v2 - v0) points); reflection is two-sided. */
int evrt_scene_set_materials(evrt_ctx *ctx, const float *albedo, const float *emission,
                             uint32_t n_mat);

/* RGB radiance (the paper's renderer is spectral; grey radiance is the
 * default): n_mat Lambertian materials with albedo_rgb[n_mat][3] in [0, 1)
 * and emission_rgb[n_mat][3] >= 0 per channel, linear Rec. 709 primaries.
 * A path's throughput is carried per channel and every contribution it
 * gathers is reduced to its luminance Y = 0.2126 R + 0.7152 G + 0.0722 B
 * (FP32 in that order) when it is added, so the per-path radiance, and all
 * statistics of the event decision (Sec. 3.2, Eq. 7: log-luminance), stay
 * scalar.  Emitters are picked in proportion to area times the luminance
 * of their emission; Russian roulette survives with min(1, largest
 * throughput channel); the environment map stays grey (its radiance in
 * every channel); grey point lights shine with their intensity in every
 * channel.  Replaces evrt_scene_set_materials (and is replaced by it).
 * The event-loss gradient refuses RGB scenes (EVRT_E_UNSUPPORTED).
 * Errors: EVRT_E_INVALID for n_mat = 0, NULL arrays, an albedo channel
 * outside [0, 1) or a negative or non-finite emission channel. */
int evrt_scene_set_materials_rgb(evrt_ctx *ctx, const float *albedo_rgb, const float *emission_rgb,
                                 uint32_t n_mat);

/* Mesh `mesh_id` (ids must end up dense 0..n-1): nv object-space vertices
 * (xyz[nv][3]) and nt triangles (tri_idx[nt][3] into this mesh's vertices,
 * tri_mat[nt] material ids).  Replaces a mesh with the same id. */
int evrt_scene_set_mesh(evrt_ctx *ctx, uint32_t mesh_id, const float *xyz, uint32_t nv,
                        const uint32_t *tri_idx, const uint32_t *tri_mat, uint32_t nt);

/* Instance `inst_id` of mesh `mesh_id` (ids dense 0..n-1) with n_keys
 * keyframes: strictly increasing times key_t[n_keys] and row-major 3x4
 * object-to-world matrices xform3x4[n_keys][12].  At time t the matrix is
 * the first key before the first key time, the last key after the last key
 * time, and otherwise the entry-wise FP64 interpolation
 * M_k + w (M_{k+1} - M_k), w = (t - t_k) / (t_{k+1} - t_k).  World vertices
 * are computed in FP64 as ((m0 x + m1 y) + m2 z) + m3 and rounded to FP32.
 * World triangles are numbered instance by instance, mesh triangle order
 * within an instance; that number breaks ties between equal hit distances. */
int evrt_scene_set_instance(evrt_ctx *ctx, uint32_t inst_id, uint32_t mesh_id, uint32_t n_keys,
                            const double *key_t, const double *xform3x4);

/* Point lights (n may be 0): positions pos_xyz[n][3], intensities
 * intensity[n].  Reached through next-event estimation only. */
int evrt_scene_set_point_lights(evrt_ctx *ctx, const float *pos_xyz, const float *intensity,
                                uint32_t n);

/* Point lights with RGB intensities intensity_rgb[n][3] (scenes with RGB
 * materials only: the commit refuses them otherwise with EVRT_E_INVALID).
 * Replaces evrt_scene_set_point_lights (and is replaced by it). */
int evrt_scene_set_point_lights_rgb(evrt_ctx *ctx, const float *pos_xyz, const float *intensity_rgb,
                                    uint32_t n);

/* Pinhole camera: image width x height, vertical field of view vfov_deg,
 * keyframed (eye, look-at, up) eye_look_up[n_keys][9], interpolated like
 * instance matrices.  The ray through pixel (x, y) with sub-pixel offset
 * (u, v) has direction f + (2 (x + u) / W - 1) s_x r + (1 - 2 (y + v) / H) s_y u'
 * (normalized), with s_y = tan(vfov / 2), s_x = s_y W / H, f, r, u' the
 * forward, right and up unit vectors of the camera. */
int evrt_scene_set_camera(evrt_ctx *ctx, uint32_t width, uint32_t height, double vfov_deg,
                          uint32_t n_keys, const double *key_t, const double *eye_look_up);

/* Environment seen by rays that leave the scene (the background of the
 * paper's failure case, Sec. 5, is an environment map): a grey cube map of
 * face_res x face_res texels per face, texels[6][face_res][face_res] (host,
 * deep-copied), faces +x, -x, +y, -y, +z, -z, row j then column i.  The
 * radiance in direction d is the texel nearest to d: the face of the major
 * axis of d (ties x, then y, then z), face coordinates (sc, tc) = (-dz, -dy)
 * on +x, (dz, -dy) on -x, (dx, dz) on +y, (dx, -dz) on -y, (dx, -dy) on +z,
 * (-dx, -dy) on -z, i = floor(N (sc / |major| + 1) / 2), likewise j from
 * tc, clamped to N - 1 (FP32 operations in that order).  A path that leaves
 * the scene adds throughput times that radiance; light samples do not
 * sample the environment.  face_res = 0 (default): black background.
 * Errors: EVRT_E_INVALID for NULL texels or a negative or non-finite
 * radiance; EVRT_E_UNSUPPORTED above 4096 texels per face edge. */
int evrt_scene_set_environment(evrt_ctx *ctx, const float *texels, uint32_t face_res);

/* Thin-lens camera (the depth of field of the paper's failure case,
 * Sec. 5): a camera ray starts at the aperture point eye + rl cos(phi) r +
 * rl sin(phi) u', rl = aperture_radius sqrt(u2), phi = 2 pi u3 (the third
 * and fourth numbers of the pixel's jitter block), and aims at eye +
 * focus_distance (f + a r + b u'), the pinhole ray's point on the plane in
 * focus.  aperture_radius = 0 (default) is the pinhole camera.  Errors:
 * EVRT_E_INVALID for a negative or non-finite radius or a non-positive
 * focus distance. */
int evrt_scene_set_lens(evrt_ctx *ctx, float aperture_radius, float focus_distance);

/* Clears the pending scene description (materials, meshes, instances,
 * lights, camera, environment, lens).  The committed scene stays current until the next
 * successful evrt_scene_commit. */
int evrt_scene_reset(evrt_ctx *ctx);

/* Validates the scene (dense ids, indices in range, finite values) and
 * makes it current.  Geometry and BVHs for an instant are built on first
 * use and cached. */
int evrt_scene_commit(evrt_ctx *ctx);

/* ---- Rendering ---------------------------------------------------------- */
typedef struct {
    uint64_t seed;           /* Philox key (low word, high word)                   */
    uint32_t max_depth;      /* surface vertices per path (>= 1), default 4        */
    uint32_t rr_start_depth; /* first vertex with Russian roulette, default 2      */
    uint32_t minibatch;      /* paths per log-luminance sample: 1, 2, 4 or 8 (4)   */
    double log_eps;          /* x = ln(Y + log_eps), default 1e-4                  */
    uint8_t nee;             /* next-event estimation on (1, default) or off (0)   */
    uint8_t jitter;          /* random sub-pixel offset (1, default) or centre (0) */
    uint8_t mode;            /* EVRT_MODE_*                                        */
    uint8_t df_mode;         /* EVRT_DF_*                                          */
    uint8_t ref_mode;        /* EVRT_REF_*                                         */
    uint8_t profile;         /* 1: time traversal launches with HIP events         */
    uint8_t count_work;      /* 1: count BVH node visits and triangle tests        */
    uint8_t lds_nodes;       /* top 4-wide BVH nodes staged in LDS, 0..32 (0)      */
    uint8_t mis;             /* 1: multiple importance sampling of area emitters:
                                each light sample (at vertices that also sample
                                a direction) and each BSDF-sampled hit of a
                                front-facing emitter after the first vertex
                                count with power-heuristic weights (pbrt's
                                PathIntegrator, Sec. 3.3, combines the two);
                                0 (default): light samples only.  Not
                                supported by evrt_event_loss_grad             */
    uint32_t ray_batch;      /* paths in flight per round, split over two
                                pieces on two streams (0: 64 M)                   */
    uint32_t key_base;       /* frame index of instant t0 in the random-number
                                keys; t1 is key_base + 1 (default 0)              */
    uint32_t trace_blocks_per_cu; /* traversal blocks per CU (0: occupancy max)    */
    uint32_t replay_retrace; /* evrt_event_loss_grad: 1 = the replay traces its
                                rays again; 0 (default) = it reads the closest
                                hits and shadow visibility the forward pass
                                logged, when the log fits (see
                                evrt_event_loss_grad)                        */
    float normality_alpha;   /* > 0: normality pre-test (Sec. 5 suggests testing
                                normality first when counts are small): an
                                early stop also needs each instant's
                                log-luminance samples to pass the Jarque-Bera
                                test, exp(-JB/2) >= normality_alpha, JB =
                                m/6 (g1^2 + g2^2/4) from the population
                                skewness g1 and excess kurtosis g2; 0 (default):
                                off.  Not supported by evrt_render_event_batch */
} evrt_render_opts;

/* Fills *opts with the defaults listed above (seed 0). */
void evrt_default_opts(evrt_render_opts *opts);

/* Per-pixel outputs, caller-owned device arrays with width*height entries
 * (two per pixel, [pixel][instant], where marked x2).  Optional arrays may
 * be NULL. */
typedef struct {
    int8_t *polarity;        /* -1, 0, +1                                  */
    uint32_t *n_paths;       /* paths traced per instant (second instant)  */
    double *mean;            /* x2: mean logL per instant                  */
    double *var;             /* x2: unbiased variance of logL per instant  */
    double *t_last;          /* optional: t of the last decision           */
    double *mean_radiance;   /* optional x2: mean of the mini-batch radiance */
    uint8_t *flags;          /* optional: bit 0 = stopped by the test      */
} evrt_frame_out;

/* Renders one event frame for the instants (t0, t1) with threshold C >= 0,
 * significance 0 < alpha < 1 and the schedule spp_init, spp_init +
 * spp_batch, ... (clamped to spp_max) paths per instant: Algorithm 1 for
 * one pair of instants, per pixel.  Each path is the tracePaths estimator
 * of Algorithm 1 (a path tracer as in Sec. 3.3); the mini-batch
 * log-luminance samples give per-instant means and variances (Eq. 3-4);
 * after every batch the t value of Eq. 7 is tested (Sec. 3.2: one-tailed,
 * lower tail, by default) and a pixel whose gap is significantly below C
 * stops with polarity 0; at spp_max the event rule of Algorithm 1 gives
 * polarity sign(gap) when |gap| > C.  The first test runs at spp_init and
 * later ones after every spp_batch (the schedule of Sec. 3.3).
 * spp_init, spp_batch and spp_max must be multiples of opts->minibatch,
 * spp_init at least two mini-batches and at most spp_max.  opts NULL =
 * defaults.  FIXED mode traces spp_max paths everywhere and applies only
 * the event rule (the comparison renderer of Sec. 4).
 * Errors: EVRT_E_INVALID for a NULL required output, C < 0 or non-finite,
 * alpha outside (0, 1), a schedule that breaks the rules above or bad
 * options; EVRT_E_STATE before a scene commit; EVRT_E_UNSUPPORTED for
 * spp_max above 2^24 or an image too large for one piece;
 * EVRT_E_NOMEM / EVRT_E_DEVICE from the device.  All argument errors are
 * reported before any device work. */
int evrt_render_event_frame(evrt_ctx *ctx, double t0, double t1, float C, float alpha,
                            uint32_t spp_init, uint32_t spp_batch, uint32_t spp_max,
                            const evrt_render_opts *opts, const evrt_frame_out *out,
                            void *stream);

/* Sequential event video (Algorithm 1 over a sequence of frames): frame 0
 * at times[0] is rendered at spp_max and becomes every pixel's reference;
 * each frame k = 1 .. n_frames - 1 is sampled adaptively against the
 * pixel's reference (the test of REF_FULL mode: Eq. 7 with N = the current
 * frame's count, df = m_ref + m - 2 or Welch), and where it fires an event
 * it replaces the reference with the frame's statistics at the count where
 * the frame stopped.  Under the one-tailed and mean-only rules events
 * happen only at spp_max; the two-tailed rule can fire early (upper tail),
 * so a reference may hold fewer samples and the tests then take each
 * pixel's own reference count into its degrees of freedom.  Frame k is keyed opts->key_base + k; opts->ref_mode is not
 * used.  Any scene motion is allowed.  Outputs as for one frame,
 * frame-major with n_frames - 1 entries per pixel: entry (k - 1) * width *
 * height + pixel holds frame k against its reference (x2 arrays: reference
 * first, then frame k). */
int evrt_render_event_video(evrt_ctx *ctx, uint32_t n_frames, const double *times, float C, float alpha,
                            uint32_t spp_init, uint32_t spp_batch, uint32_t spp_max,
                            const evrt_render_opts *opts, const evrt_frame_out *out, void *stream);

/* Renders n_pairs consecutive event frames at once: pair k is (times[k],
 * times[k+1]) (host array of n_pairs + 1 finite times) and is computed as
 * evrt_render_event_frame(times[k], times[k+1]) with opts->key_base + k
 * would compute it, bit for bit.  The frame shared by pairs k - 1 and k is
 * sampled once, up to the larger count the two pairs need (its samples are
 * the same random-number stream in both), and all pairs advance through the
 * schedule together.  Geometry and camera may move: when instances move
 * across the batch, every frame's geometry and BVH is built (in parallel on
 * the host) and kept on the device, and each round traces each frame's
 * items with its own geometry; lock-step sampling only (ref_mode LOCKSTEP);
 * at most 2047 pairs and 2^21 pixels.  Outputs as for one frame, pair-major:
 * entry k * width * height + pixel (x2 arrays: two per entry).  With the
 * environment variable EVRT_LOG_ROUNDS set to anything but "0" when the
 * library first reads it, each round prints one progress line to stderr
 * (items traced, sample range, undecided entries, seconds since the call
 * began). */
int evrt_render_event_batch(evrt_ctx *ctx, uint32_t n_pairs, const double *times, float C, float alpha,
                            uint32_t spp_init, uint32_t spp_batch, uint32_t spp_max,
                            const evrt_render_opts *opts, const evrt_frame_out *out, void *stream);

/* Counters of the last render call on ctx. */
typedef struct {
    uint64_t camera_rays, extension_rays, shadow_rays; /* rays traced        */
    uint64_t node_visits, tri_tests;  /* closest-hit traversal (4-wide node
                                         visits, triangle tests), when
                                         count_work was set (else 0)         */
    uint64_t node_visits_shadow, tri_tests_shadow; /* any-hit traversal      */
    uint64_t paths;                   /* camera paths traced (a round traces
                                         every checkpoint it covers for each
                                         active pixel, so paths past a
                                         pixel's stop are counted)           */
    uint32_t rounds;                  /* scheduling rounds (each covers one
                                         or more decision checkpoints)       */
    uint32_t pieces;                  /* wavefront pieces launched           */
    uint32_t n_closest_launches, n_shadow_launches;
    double ms_wall;                   /* host wall time of the call          */
    double ms_closest, ms_shadow;     /* summed duration of traversal
                                         launches, from events recorded by
                                         the dispatches (when profile was
                                         set, else 0)                        */
    double ms_build;                  /* geometry/BVH build done in the call */
    uint32_t active_after_round[64];  /* active pixels after rounds 0..63    */
} evrt_frame_stats;

int evrt_get_frame_stats(const evrt_ctx *ctx, evrt_frame_stats *out);

/* ---- Test and measurement hooks ----------------------------------------- */

/* Traces n caller rays against the scene at time t with the renderer's
 * traversal kernels.  rays: device float[n][8] = (ox, oy, oz, tmin, dx, dy,
 * dz, tmax); skip: device uint32[n] primitive to ignore (0xffffffff: none)
 * or NULL.  any_hit = 0: t_out[i] = closest distance and prim_out[i] = its
 * primitive, (tmax, 0xffffffff) when nothing is hit; any_hit = 1: prim_out[i]
 * = 1 if anything is hit in (tmin, tmax) else 0, t_out unused (may be NULL).
 * Results are exact (the lexicographic minimum over all triangles) for ray
 * origins within the scene's coordinate range (the largest |coordinate| of
 * its vertices, camera eye and point lights at time t): the BVH's box
 * padding, a fixed fraction of that range, covers the rounding of the box
 * test for such rays only; an origin far outside it may miss hits. */
int evrt_trace_rays(evrt_ctx *ctx, double t, uint32_t n, const float *rays,
                    const uint32_t *skip, int any_hit, float *t_out, uint32_t *prim_out,
                    void *stream);

/* ---- Entry point that allocates nothing ---------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * ray queries as evrt_trace_rays (same arguments, same kernels, identical
 * results), except that:
 *   - n <= EVRT_NOALLOC_MAX_RAYS; larger n returns EVRT_E_INVALID before
 *     any device work;
 *   - the call allocates nothing: the rays are staged in a static device
 *     array of the library (44 bytes per ray, 44 MiB + 256 bytes), which
 *     every GPU the library runs on holds until the process ends;
 *   - nothing is built: the scene at time t must already be resident on the
 *     device (an earlier evrt_trace_rays or render call at t, or, when no
 *     instance moves, at any time); otherwise EVRT_E_STATE;
 *   - the call only enqueues its two kernels on `stream` and returns; the
 *     outputs are valid once the stream has reached them.
 * Every call on one GPU uses that GPU's one array: calls that overlap on the
 * same GPU (different streams or host threads, any contexts) race and must
 * be serialized by the caller. */
#define EVRT_NOALLOC_MAX_RAYS (1u << 20)
int evrt_trace_rays_noalloc(evrt_ctx *ctx, double t, uint32_t n, const float *rays,
                            const uint32_t *skip, int any_hit, float *t_out, uint32_t *prim_out,
                            void *stream);

/* Radiance of every path sample s in [0, spp) of the listed pixels at both
 * instants (the tracePaths estimator of Algorithm 1), written to device
 * L_out[n_pixels][2][spp].  pixels: device uint32[n_pixels]. */
int evrt_render_paths(evrt_ctx *ctx, double t0, double t1, uint32_t n_pixels,
                      const uint32_t *pixels, uint32_t spp, const evrt_render_opts *opts,
                      float *L_out, void *stream);

/* Runs the accumulator and decision kernels on caller log-luminance
 * samples (Eq. 3-4 statistics, the Eq. 7 test of Sec. 3.2, the event rule
 * of Algorithm 1): x0, x1 device double[n_pixels][m] (m >= 2), pixel-major.
 * Writes t_out[n] (Eq. 7 with N = m), stop_out[n] (1 when the rule of
 * `mode` stops sampling at this count) and polarity_out[n] (event rule
 * |gap| > C).  df_mode: EVRT_DF_STUDENT (2m - 2) or EVRT_DF_WELCH.  p_out
 * (optional, NULL ok): device double[n], the lower-tail probability
 * P(T <= t) at each pixel's degrees of freedom from the device's FP64 t
 * distribution function.  All outputs are caller-owned device arrays.
 * Errors: EVRT_E_INVALID for m < 2, C < 0, alpha outside (0, 1), an unknown
 * mode or df_mode, or a NULL required array (n_pixels = 0 does nothing). */
int evrt_decide_stats(evrt_ctx *ctx, const double *x0, const double *x1, uint32_t n_pixels,
                      uint32_t m, float C, float alpha, uint8_t mode, uint8_t df_mode, double *t_out,
                      uint8_t *stop_out, int8_t *polarity_out, double *p_out, void *stream);

/* ---- Differentiation: a smoothed event loss and its gradient ---------
 *
 * For the pair (t0, t1) every pixel is sampled with spp paths per instant
 * (fixed count; spp a multiple of opts->minibatch).  With Y_{i,k} the mean
 * radiance of mini-batch k at instant i and m = spp / minibatch:
 *   mu_i  = (1/m) sum_k ln(Y_{i,k} + log_eps)    (the log-luminance of
 *           Eq. 3, averaged as in Eq. 4),
 *   Delta = mu_1 - mu_0                          (the change that Eq. 1
 *           compares with the threshold C),
 *   loss  = sum over pixels of softplus((|Delta| - C) / tau), tau > 0,
 * a smooth stand-in for the count of events.  The gradient with respect to
 * every material's albedo and emitted radiance is computed by replaying
 * each path from its random-number keys and differentiating its radiance
 * with every sampling decision held fixed: light pick, Russian roulette and
 * scattering directions.  The replay re-shades every vertex; its ray
 * queries come from a log of the forward pass (closest hit, 8 bytes per
 * path and vertex; shadow visibility, 4 bytes, with at most 31 point
 * lights, count_work 0 and lds_nodes 0) unless opts->replay_retrace is 1 or
 * the log would exceed 16 GiB or half of the free device memory, in which
 * case they are traced again.  This estimates the gradient of the expected loss terms
 * without bias; it is reported for materials with albedo > 0 (albedo) and
 * emission > 0 (emission), zero elsewhere.
 *
 * out (caller-owned device memory, double precision):
 *   loss            [1]
 *   grad            [2 * n_mat]: d loss / d albedo[j] at j, then
 *                   d loss / d emission[j] at n_mat + j
 *   loss_px, delta  [width * height] per-pixel loss term and Delta, or NULL
 *   replay_mismatch [1] number of paths whose replayed radiance differs in
 *                   any bit from the forward pass (0 expected), or NULL
 * Errors: EVRT_E_INVALID for tau <= 0, C < 0, non-finite arguments, spp not
 * a positive multiple of the mini-batch, NULL loss or grad;
 * EVRT_E_UNSUPPORTED for more than 2048 materials or 2^31 paths.  The
 * library keeps per-path radiances and weights (12 bytes per path) and the
 * ray log in its own buffers between calls. */
typedef struct {
    double *loss;
    double *grad;
    double *loss_px;
    double *delta;
    uint32_t *replay_mismatch;
} evrt_diff_out;

int evrt_event_loss_grad(evrt_ctx *ctx, double t0, double t1, float C, float tau, uint32_t spp,
                         const evrt_render_opts *opts, const evrt_diff_out *out, void *stream);

/* The per-pixel log-luminance difference Delta of evrt_event_loss_grad
 * (Eq. 3 and 7: mu_1 - mu_0 at spp paths per pixel and instant) and a
 * vector-Jacobian product through it, for an outer function L of the
 * differences whose derivative the caller gives: grad_delta, device
 * double[width * height], g_p = dL/dDelta_p.  Writes
 *   out->loss            [1] sum_p g_p Delta_p
 *   out->grad            [2 * n_mat] its derivative with respect to every
 *                        albedo, then every emission (same replay, same
 *                        reporting rule as evrt_event_loss_grad)
 *   out->loss_px, delta  g_p Delta_p and Delta per pixel, or NULL
 *   out->replay_mismatch as in evrt_event_loss_grad, or NULL.
 * grad_delta = NULL computes Delta only (out->delta required; no replay;
 * nothing else written), the forward half of an autograd step.
 * Errors as evrt_event_loss_grad (without C and tau); NULL loss or grad with
 * grad_delta set, or NULL delta without it: EVRT_E_INVALID. */
int evrt_delta_vjp(evrt_ctx *ctx, double t0, double t1, uint32_t spp, const evrt_render_opts *opts,
                   const double *grad_delta, const evrt_diff_out *out, void *stream);

/* Host-side build of the scene at time t (world triangles and the 4-wide
 * BVH, no device work) with a structural check of the BVH: every primitive
 * in exactly one leaf, every vertex inside the padded boxes of all its
 * ancestors, every node reachable once, unused child slots empty, depth
 * within the traversal stack.  Works on host-only contexts.  Returns
 * EVRT_E_INVALID (message in evrt_last_error) when a check fails.
 * n_nodes counts 4-wide inner nodes (0 when the root is a leaf), depth
 * their levels, sah_cost is the SAH cost of the binary tree the 4-wide
 * tree is collapsed from, in root-box traversals. */
typedef struct {
    uint32_t n_tri, n_nodes, n_lds, depth, n_emit;
    float box_pad;
    double sah_cost;
} evrt_scene_info;

int evrt_scene_info_at(evrt_ctx *ctx, double t, evrt_scene_info *out);

/* Host-side Student t quantile used for the critical values: the value q
 * with P(T_df <= q) = p, for integer df >= 1.  Returns NaN on bad input. */
double evrt_t_quantile(double p, uint32_t df);

#ifdef __cplusplus
}
#endif
#endif /* EVRT_H */
