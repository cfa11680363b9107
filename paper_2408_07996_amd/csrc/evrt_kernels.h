// evrt_kernels.h -- launch interface between the host scheduler and the
// gfx950 kernels (internal to the library).
#pragma once

#include "evrt_types.h"

namespace evrt {

// Layout of the uint32 device counter array: two counts (one per instant
// region) per bounce.
constexpr int kCntMaxDepth = 64;                           // max_depth limit
constexpr int kCntRay0 = 0;                                // [0, 130): rays to trace per bounce
constexpr int kCntShadow0 = kCntRay0 + 2 * (kCntMaxDepth + 1);  // [130, 260): shadow entries
constexpr int kCntActive = kCntShadow0 + 2 * (kCntMaxDepth + 1); // [260, 262): compaction counts
constexpr int kCntItems = kCntActive + 2;                  // 262: items of a frame-batch round
constexpr int kCntSize = 320;

// Decision constants of one round.  A round covers one or more checkpoints
// of the mini-batch schedule: checkpoint j ends at sample count ck_end[j]
// at the second instant and is tested with crit_lo[j] / crit_hi[j].
constexpr uint32_t kMaxChecks = 32;
// With df_per_pixel set the tests do not use the critical values: each
// pixel's degrees of freedom (Welch, or pooled over the pixel's own counts)
// give the lower-tail probability of its t, compared with alpha.
struct Decide {
    double C;
    double alpha;
    double crit_lo[kMaxChecks], crit_hi[kMaxChecks];  // t critical values (lower, upper tail)
    uint32_t ck_end[kMaxChecks];
    uint32_t n_checks;
    uint32_t mode;             // EVRT_MODE_*
    uint32_t df_mode;          // EVRT_DF_* (with df_per_pixel)
    uint32_t df_per_pixel;
    double normality_alpha;    // > 0: early stops need both instants' samples
                               // to pass the Jarque-Bera test at this level
    uint32_t final_round;      // 1 when the last checkpoint is spp_max: event rule only
    uint32_t minibatch;
    uint32_t cnt_slot;         // which of the two compaction counters this round uses
};

// Adjoint replay of the event-loss gradient: the forward pieces are traced
// again with the same keys; shading adds w dL/d(albedo) and w dL/d(Le) of
// every vertex to FP64 accumulators (per block in LDS, then g[0, n_mat) for
// albedo and g[n_mat, 2 n_mat) for emission).  W[(pixel * 2 + instant) * m
// + mini-batch] are the mini-batch weights, Lfwd[(pixel * 2 + instant) *
// spp + sample] the forward path radiances; sw / semat carry the weight and
// the emitter material of each shadow entry (its area-light slot) to the
// shadow kernel.
struct Adjoint {
    const double *W;
    const float *Lfwd;
    double *g;
    double *sw;
    uint32_t *semat;
    uint32_t n_mat, m, mb, spp;
};

// Caller output arrays (device).
struct Outputs {
    int8_t *polarity;
    uint32_t *n_paths;
    double *mean, *var, *t_last, *mean_radiance;
    uint8_t *flags;
};

// The first active list holds every pixel: in pixel order, or with rows
// (device, rows[k] = image row at list row k, npx / width entries) row by
// row in that order.
void launch_init_frame(hipStream_t s, uint32_t npx, uint32_t *wf_n, double *wf_mean, double *wf_m2,
                       double *wf_ysum, uint32_t *act, uint32_t *cnt, unsigned long long *stat,
                       uint32_t width = 1, const uint32_t *rows = nullptr);
void launch_raygen(hipStream_t s, const Piece &pc, const DevScene &sc, const RenderParams &rp,
                   const RayQueue &q, uint32_t *cnt);
// Traversal and shading kernels take the per-region counts cnt_in[0..1],
// the region size and the number of regions; grids must be multiples of 8.
// ev_start / ev_stop (may be null) are recorded by the dispatch itself, so
// they time the kernel's execution and not its wait in the queue.
void launch_trace_closest(hipStream_t s, uint32_t blocks, bool count, const DevScene &sc,
                          const RayQueue &q, const uint32_t *cnt_in, uint32_t region, uint32_t n_split,
                          uint32_t inst_base, float2 *hit, int stat_kind, unsigned long long *stat,
                          hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// Ray log of a gradient: vis_log (per-vertex slice indexed by radiance
// index) is written by the forward pass (adj null: the tracing kernel also
// stores each entry's mask of unoccluded slots) and read by the replay (adj
// set: no tracing, the masks decide).  With vis_log: n_slots <= 32, count
// false and no LDS treelet.  hit_log (per-vertex slice indexed by path id)
// likewise: the forward shade writes each ray's hit, the replay shade reads
// it in place of `hit`.
void launch_trace_shadow(hipStream_t s, uint32_t blocks, bool count, const DevScene &sc,
                         const ShadowQueue &sq, uint32_t n_slots, const uint32_t *cnt_in, uint32_t region,
                         uint32_t n_split, uint32_t inst_base, float *rad, unsigned long long *stat,
                         hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr,
                         const Adjoint *adj = nullptr, uint32_t *vis_log = nullptr);
void launch_shade(hipStream_t s, uint32_t blocks, const Piece &pc, const DevScene &sc,
                  const RenderParams &rp, const RayQueue &qin, const uint32_t *cnt_in,
                  const float2 *hit, const RayQueue &qout, uint32_t *cnt_out, const ShadowQueue &sq,
                  uint32_t *cnt_sh, uint32_t depth, uint32_t threads, const Adjoint *adj = nullptr,
                  float2 *hit_log = nullptr);
void launch_accumulate(hipStream_t s, const Piece &pc, const RenderParams &rp, uint32_t *wf_n,
                       double *wf_mean, double *wf_m2, double *wf_ysum);
// Welford updates and the decision at every checkpoint of the round, for
// pieces that hold the round's whole sample range of their pixels.
void launch_accumulate_decide(hipStream_t s, const Piece &pc, const RenderParams &rp, const Decide &dc,
                              uint32_t *act_out, uint32_t *cnt, uint32_t *wf_n, double *wf_mean,
                              double *wf_m2, double *wf_ysum, const Outputs &out);
void launch_decide_compact(hipStream_t s, const RenderParams &rp, const Decide &dc, const uint32_t *act_in,
                           uint32_t nA, uint32_t *act_out, uint32_t *cnt, const uint32_t *wf_n,
                           const double *wf_mean, const double *wf_m2, const double *wf_ysum,
                           const Outputs &out);
void launch_hook_rays(hipStream_t s, uint32_t n, const float *rays, const uint32_t *skip,
                      const RayQueue &q, float *tminmax, uint32_t *cnt);
void launch_hook_trace(hipStream_t s, uint32_t blocks, bool any, const DevScene &sc, const RayQueue &q,
                       const float *tminmax, uint32_t n, float *t_out, uint32_t *p_out);
// p_out (may be null): lower-tail probability of each t at the pixel's
// degrees of freedom (dc.df_mode), from the device CDF.
void launch_hook_decide(hipStream_t s, const double *x0, const double *x1, uint32_t n, uint32_t m,
                        const Decide &dc, double *t_out, uint8_t *stop_out, int8_t *pol_out, double *p_out);

// Event loss and its gradient: zeroing, per-pixel statistics and weights,
// path-replay adjoint (g = [albedo gradients | emission gradients]).
void launch_diff_zero(hipStream_t s, double *loss, double *g, uint32_t n_g, uint32_t *mismatch);
// Per pixel: Delta, the loss term and the weight of every mini-batch;
// upstream (null: the smoothed event loss) holds the caller's dL/dDelta.
void launch_diff_stats(hipStream_t s, uint32_t npx, uint32_t spp, uint32_t mb, double log_eps, double C,
                       double tau, const double *upstream, const float *L, double *W, double *loss,
                       double *loss_px, double *delta_px);
void launch_diff_compare(hipStream_t s, uint64_t n, const float *a, const float *b, uint32_t *mismatch);

// Sequential video: current-frame slots cleared / references replaced at
// events.
void launch_video_frame_init(hipStream_t s, uint32_t npx, uint32_t *wf_n, double *wf_mean, double *wf_m2,
                             double *wf_ysum, uint32_t *act, uint32_t *cnt, uint32_t width = 1,
                             const uint32_t *rows = nullptr);
void launch_video_update(hipStream_t s, uint32_t npx, const int8_t *polarity, uint32_t *wf_n, double *wf_mean,
                         double *wf_m2, double *wf_ysum, double *wf_m34);

// Frame batches (see k_batch_* in the kernels).
void launch_batch_init(hipStream_t s, uint32_t n_frames, uint32_t npx, uint32_t *wf_n, double *wf_mean,
                       double *wf_m2, double *wf_ysum, uint32_t *item_idx, uint32_t *items, uint32_t *act,
                       uint2 *pair_items, uint32_t *cnt);
void launch_batch_items(hipStream_t s, const uint32_t *act, uint32_t nA, uint32_t npx, uint32_t *item_idx,
                        uint32_t *items, uint32_t *cnt);
void launch_batch_pair_items(hipStream_t s, const uint32_t *act, uint32_t nA, uint32_t npx,
                             const uint32_t *item_idx, uint2 *pair_items);
void launch_batch_clear(hipStream_t s, const uint32_t *items, uint32_t n_items, uint32_t npx, uint32_t *item_idx,
                        uint32_t *cnt);
// Batches of moving geometry: the round's items sorted by (frame, pixel)
// (radix sort into `sorted`, temp storage of batch_sort_temp_bytes), item
// indices renewed, first position of each frame in frame_start[nf]
// (0xffffffff for frames without items).
size_t batch_sort_temp_bytes(uint32_t n_items);
void launch_batch_regroup(hipStream_t s, uint32_t *items, uint32_t n_items, uint32_t *sorted, void *temp,
                          size_t temp_bytes, uint32_t npx, uint32_t *item_idx, uint32_t *frame_start, uint32_t nf);
void launch_batch_accumulate(hipStream_t s, const Piece &pc, const RenderParams &rp, const Decide &dc,
                             uint32_t npx, uint32_t item_base, uint32_t *wf_n, double *wf_mean, double *wf_m2,
                             double *wf_ysum, double *snap);
void launch_batch_decide(hipStream_t s, const Decide &dc, const uint32_t *act, uint32_t nA, uint32_t npx,
                         const uint2 *pair_items, const uint32_t *items, const uint32_t *wf_n,
                         const double *wf_mean, const double *wf_m2, const double *wf_ysum, const double *snap,
                         uint32_t *act_out, uint32_t *cnt, const Outputs &out);

// Entry point that allocates nothing (evrt_trace_rays_noalloc): at most
// kNoAllocRays rays per call, staged in a static device array of
// kNoAllocScratchBytes (44 bytes per ray: origin and direction float4, skip
// primitive, (tmin, tmax); then the counter words).  noalloc_scratch_address
// returns the array's device address on `device`, which must be current;
// it resolves the address once per device and keeps it.
constexpr uint32_t kNoAllocRays = 1u << 20;
constexpr size_t kNoAllocScratchBytes = 44 * (size_t)kNoAllocRays + 256;
struct NoAllocScratch {
    float4 *o, *d;
    uint32_t *skip;
    float *tminmax;
    uint32_t *cnt;
};
NoAllocScratch noalloc_layout(void *base);
hipError_t noalloc_scratch_address(int device, void **out);

void kernel_occupancy(int *trace_blocks_per_cu, int *shade_blocks_per_cu);
int traverse_block_threads();
int shade_block_threads();  // largest shade block (the kernel's launch bound)
int lds_treelet_nodes();   // 4-wide nodes a block can stage in LDS per instant
int traverse_max_depth();  // deepest 4-wide tree (inner levels) the traversal stack holds

}  // namespace evrt
