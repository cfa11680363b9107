// evrt_host.h -- host-side state of the library (internal).
#pragma once

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/evrt.h"
#include "evrt_kernels.h"

namespace evrt {

// Thrown inside the library, converted to a status at the ABI boundary.
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void hip_check(hipError_t e, const char *what);

// Device allocation that only grows.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    void ensure(size_t n);
    void upload(const void *src, size_t n, hipStream_t s);
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

struct MeshDesc {
    bool set = false;
    std::vector<float> xyz;
    std::vector<uint32_t> idx, mat;
};

struct InstanceDesc {
    bool set = false;
    uint32_t mesh = 0;
    std::vector<double> kt, kx;  // keys, 12 doubles per key
};

struct CameraDesc {
    bool set = false;
    uint32_t width = 0, height = 0;
    double vfov = 0.0;
    std::vector<double> kt, elu;  // 9 doubles per key
};

struct SceneDesc {
    // Grey materials, or with RGB radiance the largest albedo channel and
    // the emission's luminance (they drive the same decisions).
    std::vector<float> albedo, emission;
    bool rgb = false;                       // RGB radiance
    std::vector<float> albedo3, emission3;  // [n_mat][3] with RGB radiance
    std::vector<float> pl_int3;             // [n][3] RGB point-light intensities (empty: grey)
    std::vector<MeshDesc> meshes;
    std::vector<InstanceDesc> instances;
    std::vector<float> pl_pos, pl_int;
    CameraDesc cam;
    std::vector<float> env;      // [6][N][N] cube map (empty: black background)
    uint32_t env_res = 0;
    float lens_radius = 0.0f;    // thin lens aperture radius (0: pinhole)
    float focus_dist = 1.0f;     // distance of the plane in focus
};

// World-space geometry of one instant, built on the host and uploaded.
struct HostInstant {
    std::vector<float> tri;      // [n][9] world vertices in primitive order
    std::vector<float4> prim;    // [n] (unit normal, material bits)
    std::vector<float> area;     // [n]
    std::vector<uint32_t> emit_prim;
    std::vector<float> emit_cdf;
    float emit_S = 0.0f;
    DevCamera cam;
    // BVH
    std::vector<float4> nodes;   // 8 per 4-wide inner node
    std::vector<float4> tris;    // 3 per triangle in leaf order
    int32_t root = kEmptyRef;
    uint32_t n_lds = 0;
    uint32_t depth = 0;          // inner levels of the 4-wide tree
    float plane_scale = 1.0f;    // power of two dividing stored node origins and plane offsets
    double sah_cost = 0.0;       // SAH cost of the binary tree
};

struct DevInstantBufs {
    DevBuf nodes, tris, prim, emit_cdf, emit;
    DevInstant view{};
    HostInstant host;  // kept for statistics and validation
    // Owner of the buffers that view points to, when they are shared with
    // another time of a scene whose geometry does not move.
    std::shared_ptr<DevInstantBufs> geom;
};

// World geometry at time t (primitive order, FP64 transform, FP32 round).
void build_world(const SceneDesc &sd, double t, HostInstant &out);
// Emitter table of h (emit_prim, emit_cdf, emit_S) from its primitives'
// materials and areas and the scene's emission values.
void build_emitters(const SceneDesc &sd, HostInstant &h);
// Camera basis at time t (FP64 interpolation, FP32 round).
void camera_at(const SceneDesc &sd, double t, DevCamera &out);
// True when every instance has the same transform at all n times.
bool instances_static(const SceneDesc &sd, const double *times, uint32_t n);
// True when every instance's keys hold one transform (no motion at all).
bool scene_static(const SceneDesc &sd);
// 4-wide BVH over out.tri (a binned-SAH binary tree collapsed two levels
// at a time), breadth-first treelet of up to n_lds_max nodes first.
void build_bvh(HostInstant &h, uint32_t n_lds_max, float pad);
// Validates structural invariants of a built BVH; returns an empty string
// when they hold.
std::string check_bvh(const HostInstant &h, float pad);
// Padding of node boxes for a scene (see the box test in the kernels).
float bvh_padding(const SceneDesc &sd, const HostInstant &a, const HostInstant &b);

FastDiv make_fastdiv(uint32_t d);

// Student t quantile (integer df) and its memoized critical values.
double t_quantile(double p, uint32_t df);

// Wavefront queues of one piece in flight.  Two lanes let consecutive pieces
// run on two streams so that one piece's kernels fill the other's tails.
struct LaneBufs {
    DevBuf q_o[2], q_d[2], q_skip[2], hit;
    DevBuf q_bgb[2];  // RGB radiance: green and blue throughput of the ray queues
    DevBuf sh_o, sh_meta, sh_dir, sh_c;
    DevBuf rad;
    uint32_t queue_cap = 0, shadow_slots = 0;
};

struct FrameBuffers {
    DevBuf wf_n, wf_mean, wf_m2, wf_ysum, act0, act1;
    DevBuf wf_m34;                        // normality pre-test: m3, m4 per slot
    DevBuf cnt, stat;
    DevBuf cnt1;  // per-bounce queue counts of lane 1 (lane 0 uses cnt)
    DevBuf row_order;                   // first-round row order (first_rows)
    std::vector<uint32_t> row_order_h;  // its host copy (the upload's source)
    LaneBufs lane[2];
    DevBuf hook_tm;
    DevBuf diff_px, diff_L, diff_W;  // event-loss gradient: pixel list, path radiance, weights
    DevBuf diff_R;                       // adjoint replay: radiance
    DevBuf diff_sw[2], diff_semat[2];    // per lane: weight and emitter of each shadow entry
    DevBuf diff_hitlog, diff_vislog;     // ray log: closest hits, shadow visibility masks
    // Frame batches: per-(frame, pixel) state and item index, item list,
    // active pairs (two lists) with their items, checkpoint snapshots,
    // per-frame cameras.
    DevBuf b_wf_n, b_wf_mean, b_wf_m2, b_wf_ysum, b_item_idx, b_items, b_act0, b_act1, b_pair_items, b_snap,
        b_cams;
    DevBuf b_sorted, b_sort_tmp, b_frame_start;  // moving geometry: items regrouped by frame
};

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace evrt

struct evrt_ctx {
    int device = -1;
    bool host_only = true;
    std::string err;
    evrt::SceneDesc pending;
    evrt::SceneDesc scene;
    bool committed = false;
    bool static_geom = false;  // no instance moves: one geometry for all times
    uint64_t scene_version = 0;
    std::map<double, std::shared_ptr<evrt::DevInstantBufs>> cache;
    std::vector<double> cache_order;
    evrt::DevBuf mat, plights, env;
    evrt::DevBuf mat_rgb, plights_rgb;  // RGB radiance tables
    evrt::FrameBuffers fb;
    hipStream_t s2 = nullptr;                // second lane's stream (default priority)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    uint32_t *h_pinned = nullptr;            // pinned readback words
    unsigned long long *h_stat = nullptr;    // pinned stat readback
    std::vector<evrt::EventPair> events;
    std::map<std::pair<uint64_t, uint32_t>, double> crit_cache;
    evrt_frame_stats stats{};
    uint32_t cu_count = 0;
    uint32_t trace_blocks_per_cu = 0;
    uint32_t shade_blocks_per_cu = 0;
    void *noalloc_scratch = nullptr;         // this device's static scratch array
    uint32_t materials_only_commits = 0;     // commits that kept the instants
    size_t cache_cap = 0;                    // instants the cache holds (at least 4)
    std::vector<uint32_t> h_frame_start;     // readback of a batch round's frame starts
};

namespace evrt {
// Geometry of instant t on the device (built and cached on first use).
std::shared_ptr<DevInstantBufs> get_instant(evrt_ctx *c, double t, hipStream_t s, double *ms_build);
// Geometry of every time in times[0, n) on the device, the missing ones
// built on all host threads; the cache grows to hold them all.
void get_instants(evrt_ctx *c, const double *times, uint32_t n, hipStream_t s, double *ms_build);
// After a commit that changed only albedo and emission: the emitter tables
// of every cached instant rebuilt and uploaded; geometry and BVHs are kept.
void refresh_emitters(evrt_ctx *c);
DevScene make_dev_scene(evrt_ctx *c, const DevInstantBufs &a, const DevInstantBufs &b, uint32_t lds_nodes);
void render_frame(evrt_ctx *c, double t0, double t1, float C, float alpha, uint32_t spp_init,
                  uint32_t spp_batch, uint32_t spp_max, const evrt_render_opts &o,
                  const evrt_frame_out &out, hipStream_t s);
void render_paths(evrt_ctx *c, double t0, double t1, uint32_t n_pixels, const uint32_t *pixels,
                  uint32_t spp, const evrt_render_opts &o, float *L_out, hipStream_t s);
void trace_rays(evrt_ctx *c, double t, uint32_t n, const float *rays, const uint32_t *skip, int any,
                float *t_out, uint32_t *p_out, hipStream_t s);
// The same ray queries with the rays staged in the device's static scratch
// array: no allocation, no BVH build (the instant must be resident), no
// synchronization.
void trace_rays_noalloc(evrt_ctx *c, double t, uint32_t n, const float *rays, const uint32_t *skip, int any,
                        float *t_out, uint32_t *p_out, hipStream_t s);
void decide_stats(evrt_ctx *c, const double *x0, const double *x1, uint32_t n, uint32_t m, float C,
                  float alpha, uint8_t mode, uint8_t df_mode, double *t_out, uint8_t *stop_out, int8_t *pol_out,
                  double *p_out, hipStream_t s);
void render_video(evrt_ctx *c, uint32_t n_frames, const double *times, float C, float alpha, uint32_t spp_init,
                  uint32_t spp_batch, uint32_t spp_max, const evrt_render_opts &o, const evrt_frame_out &out,
                  hipStream_t s);
void render_batch(evrt_ctx *c, uint32_t n_pairs, const double *times, float C, float alpha, uint32_t spp_init,
                  uint32_t spp_batch, uint32_t spp_max, const evrt_render_opts &o, const evrt_frame_out &out,
                  hipStream_t s);
// upstream: the caller's dL/dDelta per pixel for a product through Delta
// (null: the smoothed event loss with C and tau); delta_only: Delta (and the
// forward statistics) without the replay.
void event_loss_grad(evrt_ctx *c, double t0, double t1, float C, float tau, uint32_t spp,
                     const evrt_render_opts &o, const evrt_diff_out &out, hipStream_t s,
                     const double *upstream = nullptr, bool delta_only = false);
void validate_opts(const evrt_render_opts &o);
}  // namespace evrt
