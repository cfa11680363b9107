// render.cpp -- host scheduler of the adaptive event renderer.
//
// One event frame (Algorithm 1 for one pair of instants): all pixels start
// active; each round traces the next sample range of every active pixel
// (split into pieces that bound the paths in flight), accumulates the
// mini-batch log-luminance, then runs the decision kernel, which writes the
// outputs of finished pixels and compacts the rest into the next active
// list.  The active count is read back once per round.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <future>
#include <map>
#include <thread>

#include "evrt_host.h"

namespace evrt {

static constexpr uint32_t kDefaultRayBatch = 1u << 26;
static constexpr uint32_t kMaxPathId = 1u << 31;
static constexpr size_t kCacheInstants = 4;
static constexpr uint64_t kMaxRayLog = 16ull << 30;  // bytes of a gradient's ray log

static void cache_insert(evrt_ctx *c, double t, const std::shared_ptr<DevInstantBufs> &bi)
{
    if (c->cache.size() >= std::max<size_t>(kCacheInstants, c->cache_cap)) {
        const double victim = c->cache_order.front();
        c->cache_order.erase(c->cache_order.begin());
        c->cache.erase(victim);
    }
    c->cache[t] = bi;
    c->cache_order.push_back(t);
}

static void build_host_instant(const evrt_ctx *c, double t, HostInstant &h);
static void upload_instant(evrt_ctx *c, DevInstantBufs &bi, hipStream_t s);

// Emitter table of an instant on the device: the CDF and, per emitter, its
// three vertices (the first with the emitted radiance in w) and (unit
// normal, primitive id); the view's emitter fields.
static void upload_emitters(DevInstantBufs &bi, const SceneDesc &sd, hipStream_t s)
{
    const HostInstant &h = bi.host;
    bi.emit_cdf.upload(h.emit_cdf.data(), h.emit_cdf.size() * sizeof(float), s);
    std::vector<float4> emit(4 * h.emit_prim.size());
    for (size_t j = 0; j < h.emit_prim.size(); ++j) {
        const uint32_t p = h.emit_prim[j];
        const float *v = &h.tri[9 * (size_t)p];
        uint32_t mat;
        std::memcpy(&mat, &h.prim[p].w, 4);
        emit[4 * j + 0] = make_float4(v[0], v[1], v[2], sd.emission[mat]);
        emit[4 * j + 1] = make_float4(v[3], v[4], v[5], 0.0f);
        emit[4 * j + 2] = make_float4(v[6], v[7], v[8], 0.0f);
        float pw;
        std::memcpy(&pw, &p, 4);
        emit[4 * j + 3] = make_float4(h.prim[p].x, h.prim[p].y, h.prim[p].z, pw);
    }
    bi.emit.upload(emit.data(), emit.size() * sizeof(float4), s);
    DevInstant &v = bi.view;
    v.emit_cdf = bi.emit_cdf.as<const float>();
    v.emit = bi.emit.as<const float4>();
    v.n_emit = (uint32_t)h.emit_prim.size();
    v.emit_S = h.emit_S;
}

void refresh_emitters(evrt_ctx *c)
{
    // Instants that own their buffers first (also an owner that left the
    // cache while a time sharing its geometry stayed), then the times that
    // share an owner's geometry (static scenes) take its new emitter fields.
    std::vector<DevInstantBufs *> owners;
    for (auto &kv : c->cache) {
        DevInstantBufs *o = kv.second->geom ? kv.second->geom.get() : kv.second.get();
        if (std::find(owners.begin(), owners.end(), o) == owners.end()) owners.push_back(o);
    }
    for (DevInstantBufs *o : owners) {
        build_emitters(c->scene, o->host);
        upload_emitters(*o, c->scene, nullptr);
    }
    for (auto &kv : c->cache) {
        DevInstantBufs &bi = *kv.second;
        if (!bi.geom) continue;
        const DevInstant &g = bi.geom->view;
        bi.view.emit_cdf = g.emit_cdf;
        bi.view.emit = g.emit;
        bi.view.n_emit = g.n_emit;
        bi.view.emit_S = g.emit_S;
    }
    hip_check(hipStreamSynchronize(nullptr), "emitter upload");
}

std::shared_ptr<DevInstantBufs> get_instant(evrt_ctx *c, double t, hipStream_t s, double *ms_build)
{
    auto it = c->cache.find(t);
    if (it != c->cache.end()) return it->second;
    const auto t_start = std::chrono::steady_clock::now();
    auto bi = std::make_shared<DevInstantBufs>();
    if (c->static_geom && !c->cache.empty()) {
        // Geometry that no instance moves is the same at every time: share
        // the device buffers of a cached instant, only the camera differs.
        const auto base = c->cache.begin()->second;
        bi->view = base->view;
        camera_at(c->scene, t, bi->view.cam);
        bi->geom = base->geom ? base->geom : base;
        cache_insert(c, t, bi);
        if (ms_build)
            *ms_build += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        return bi;
    }
    build_host_instant(c, t, bi->host);
    upload_instant(c, *bi, s);
    cache_insert(c, t, bi);
    if (ms_build)
        *ms_build += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return bi;
}

// World geometry and BVH of instant t on the host (reads only the committed
// scene: several may run at once).
static void build_host_instant(const evrt_ctx *c, double t, HostInstant &h)
{
    build_world(c->scene, t, h);
    const float pad = bvh_padding(c->scene, h, h);
    build_bvh(h, (uint32_t)lds_treelet_nodes(), pad);
    if (h.depth > (uint32_t)traverse_max_depth()) fail(EVRT_E_UNSUPPORTED, "BVH deeper than the traversal stack");
    // Traversal addresses nodes by 32-bit byte offsets (128 bytes a node).
    if (h.nodes.size() / 8 >= (1u << 25)) fail(EVRT_E_UNSUPPORTED, "more than 2^25 BVH nodes");
}

static void upload_instant(evrt_ctx *c, DevInstantBufs &bi, hipStream_t s)
{
    HostInstant &h = bi.host;
    bi.nodes.upload(h.nodes.data(), h.nodes.size() * sizeof(float4), s);
    bi.tris.upload(h.tris.data(), h.tris.size() * sizeof(float4), s);
    bi.prim.upload(h.prim.data(), h.prim.size() * sizeof(float4), s);
    upload_emitters(bi, c->scene, s);
    hip_check(hipStreamSynchronize(s), "geometry upload");
    DevInstant &v = bi.view;
    v.nodes = bi.nodes.as<const float4>();
    v.tris = bi.tris.as<const float4>();
    v.prim = bi.prim.as<const float4>();
    v.root = h.root;
    v.plane_scale = h.plane_scale;
    v.n_nodes = (uint32_t)(h.nodes.size() / 8);
    v.n_lds = h.n_lds;
    v.cam = h.cam;
    // The host keeps the world triangles, primitives and areas (emitter
    // tables of a material-only commit); the BVH lives on the device only.
    std::vector<float4>().swap(h.nodes);
    std::vector<float4>().swap(h.tris);
}

void get_instants(evrt_ctx *c, const double *times, uint32_t n, hipStream_t s, double *ms_build)
{
    c->cache_cap = std::max<size_t>(c->cache_cap, (size_t)n + 2);
    std::vector<double> todo;
    for (uint32_t k = 0; k < n; ++k)
        if (!c->cache.count(times[k]) && std::find(todo.begin(), todo.end(), times[k]) == todo.end())
            todo.push_back(times[k]);
    if (todo.empty()) return;
    if (c->static_geom || todo.size() == 1) {
        for (double t : todo) get_instant(c, t, s, ms_build);
        return;
    }
    // Host builds on every host thread (each one instant at a time), then
    // the uploads in order.
    const auto t_start = std::chrono::steady_clock::now();
    std::vector<std::shared_ptr<DevInstantBufs>> bis(todo.size());
    for (auto &b : bis) b = std::make_shared<DevInstantBufs>();
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const size_t nt = std::min<size_t>(hw, todo.size());
    std::atomic<size_t> next{0};
    std::vector<std::string> errs(nt);
    std::vector<int> codes(nt, 0);
    std::vector<std::thread> th;
    for (size_t w = 0; w < nt; ++w)
        th.emplace_back([&, w] {
            try {
                for (size_t k; (k = next.fetch_add(1)) < todo.size();) build_host_instant(c, todo[k], bis[k]->host);
            } catch (const Error &e) {
                codes[w] = e.code;
                errs[w] = e.msg;
            } catch (const std::exception &e) {
                codes[w] = EVRT_E_NOMEM;
                errs[w] = e.what();
            }
        });
    for (auto &t : th) t.join();
    for (size_t w = 0; w < nt; ++w)
        if (codes[w]) fail(codes[w], errs[w]);
    for (size_t k = 0; k < todo.size(); ++k) {
        upload_instant(c, *bis[k], s);
        cache_insert(c, todo[k], bis[k]);
    }
    if (ms_build)
        *ms_build += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
}

// The instants of a pair; two that both need building are built on two
// host threads at once.
static std::pair<std::shared_ptr<DevInstantBufs>, std::shared_ptr<DevInstantBufs>>
get_pair(evrt_ctx *c, double t0, double t1, hipStream_t s, double *ms_build)
{
    const double tt[2] = {t0, t1};
    get_instants(c, tt, 2, s, ms_build);
    auto ga = get_instant(c, t0, s, ms_build);
    auto gb = get_instant(c, t1, s, ms_build);
    return {ga, gb};
}

DevScene make_dev_scene(evrt_ctx *c, const DevInstantBufs &a, const DevInstantBufs &b, uint32_t lds_nodes)
{
    DevScene sc{};
    sc.inst[0] = a.view;
    sc.inst[1] = b.view;
    // The builder lays the top nodes out first; stage only as many as asked.
    sc.inst[0].n_lds = std::min(sc.inst[0].n_lds, lds_nodes);
    sc.inst[1].n_lds = std::min(sc.inst[1].n_lds, lds_nodes);
    sc.mat = c->mat.as<const float2>();
    sc.plights = c->plights.as<const float4>();
    sc.rgb = c->scene.rgb ? 1u : 0u;
    sc.mat_rgb = c->scene.rgb ? c->mat_rgb.as<const float4>() : nullptr;
    sc.plights_rgb = c->scene.rgb ? c->plights_rgb.as<const float4>() : nullptr;
    sc.n_plights = (uint32_t)c->scene.pl_int.size();
    sc.env = c->env.as<const float>();
    sc.env_res = c->scene.env_res;
    sc.lens_radius = c->scene.lens_radius;
    sc.focus_dist = c->scene.focus_dist;
    sc.width = c->scene.cam.width;
    sc.height = c->scene.cam.height;
    sc.div_w = make_fastdiv(sc.width);
    return sc;
}

static RenderParams make_params(evrt_ctx *c, const evrt_render_opts &o)
{
    RenderParams rp{};
    if (o.normality_alpha > 0.0f) {
        // Third and fourth moment sums of both accumulator slots per pixel.
        const size_t npx = (size_t)c->scene.cam.width * c->scene.cam.height;
        c->fb.wf_m34.ensure(sizeof(double) * 4 * npx);
        rp.wf_m34 = c->fb.wf_m34.as<double>();
    }
    rp.key0 = (uint32_t)(o.seed & 0xffffffffu);
    rp.key1 = (uint32_t)(o.seed >> 32);
    rp.max_depth = o.max_depth;
    rp.rr_start = o.rr_start_depth;
    rp.nee = o.nee;
    rp.jitter = o.jitter;
    rp.minibatch = o.minibatch;
    rp.n_slots = 1 + (uint32_t)c->scene.pl_int.size();
    rp.key_base = o.key_base;
    rp.mis = o.mis;
    rp.log_eps = o.log_eps;
    return rp;
}

// Device work buffers for npx pixels and a piece of `cap` paths in flight
// on lane `ln`.
static void ensure_buffers(evrt_ctx *c, uint32_t npx, uint32_t cap, uint32_t slots, int ln = 0)
{
    FrameBuffers &fb = c->fb;
    fb.wf_n.ensure(sizeof(uint32_t) * 2 * (size_t)npx);
    fb.wf_mean.ensure(sizeof(double) * 2 * (size_t)npx);
    fb.wf_m2.ensure(sizeof(double) * 2 * (size_t)npx);
    fb.wf_ysum.ensure(sizeof(double) * 2 * (size_t)npx);
    fb.act0.ensure(sizeof(uint32_t) * (size_t)npx);
    fb.act1.ensure(sizeof(uint32_t) * (size_t)npx);
    fb.cnt.ensure(sizeof(uint32_t) * kCntSize);
    fb.cnt1.ensure(sizeof(uint32_t) * kCntSize);
    fb.stat.ensure(sizeof(unsigned long long) * kStatCount);
    LaneBufs &L = fb.lane[ln];
    if (cap > L.queue_cap || slots > L.shadow_slots) {
        const uint32_t ncap = std::max(cap, L.queue_cap);
        const uint32_t nsl = std::max(slots, L.shadow_slots);
        for (int k = 0; k < 2; ++k) {
            L.q_o[k].ensure(sizeof(float4) * (size_t)ncap);
            L.q_d[k].ensure(sizeof(float4) * (size_t)ncap);
            L.q_skip[k].ensure(sizeof(uint32_t) * (size_t)ncap);
        }
        L.hit.ensure(sizeof(float2) * (size_t)ncap);
        L.sh_o.ensure(sizeof(float4) * (size_t)ncap);
        L.sh_meta.ensure(sizeof(uint32_t) * (size_t)ncap);
        // Slot-major shadow arrays: their stride is the capacity, so they are
        // reallocated whenever the capacity changes.
        L.sh_dir.ensure(sizeof(float4) * (size_t)ncap * nsl);
        L.sh_c.ensure(sizeof(float) * (size_t)ncap * nsl);
        L.rad.ensure(sizeof(float) * (size_t)ncap);
        L.queue_cap = ncap;
        L.shadow_slots = nsl;
    }
}

// Grid for a queue of up to `work` items: enough blocks to fill the chip or
// cover the work, rounded up to a multiple of the 8 XCDs (the per-instant
// queue split maps XCDs to instants).
static uint32_t blocks_for(uint32_t per_cu, uint32_t cu, uint32_t work, uint32_t tb)
{
    const uint32_t need = (work + tb - 1) / tb;
    const uint32_t fill = std::max(1u, per_cu * cu);
    const uint32_t b = std::max(1u, std::min(need, fill));
    return (b + 7u) & ~7u;
}

struct Profiler {
    evrt_ctx *c;
    bool on;
    size_t used = 0;
    std::vector<int> kind;  // 0 closest, 1 shadow
    // Events for the next traversal launch of this kind (null when off).
    EventPair take(int k)
    {
        if (!on) return EventPair{};
        if (used == c->events.size()) {
            EventPair e;
            hip_check(hipEventCreate(&e.a), "hipEventCreate");
            hip_check(hipEventCreate(&e.b), "hipEventCreate");
            c->events.push_back(e);
        }
        kind.push_back(k);
        return c->events[used++];
    }
    void collect(evrt_frame_stats &st)
    {
        for (size_t i = 0; i < used; ++i) {
            float ms = 0.0f;
            hip_check(hipEventElapsedTime(&ms, c->events[i].a, c->events[i].b), "hipEventElapsedTime");
            if (kind[i] == 0) st.ms_closest += ms;
            else st.ms_shadow += ms;
        }
    }
};

// Ray log of one piece of a gradient: slices of pc.n_paths entries per
// vertex, the closest hit by path id and the shadow entry's mask of
// unoccluded slots by radiance index (vis null: shadows are traced in both
// passes).  The forward pass writes it; the replay (replay true) reads it
// and traces nothing.
struct RayLog {
    float2 *hit;
    uint32_t *vis;
    bool replay;
};

// Traces one piece: camera rays, max_depth bounces of closest hit + shade
// + shadow rays.  Path radiances land in pc.rad.
static void trace_piece(evrt_ctx *c, const Piece &pc, const DevScene &sc, const RenderParams &rp,
                        const evrt_render_opts &o, hipStream_t s, Profiler &prof, int ln = 0,
                        const Adjoint *adj = nullptr, const RayLog *log = nullptr)
{
    FrameBuffers &fb = c->fb;
    LaneBufs &L = fb.lane[ln];
    uint32_t *cnt = ln ? fb.cnt1.as<uint32_t>() : fb.cnt.as<uint32_t>();
    unsigned long long *stat = fb.stat.as<unsigned long long>();
    RayQueue q[2];
    for (int k = 0; k < 2; ++k) {
        q[k] = RayQueue{L.q_o[k].as<float4>(), L.q_d[k].as<float4>(), L.q_skip[k].as<uint32_t>(), nullptr};
        if (sc.rgb) {
            L.q_bgb[k].ensure(sizeof(float2) * (size_t)L.queue_cap);
            q[k].bgb = L.q_bgb[k].as<float2>();
        }
    }
    ShadowQueue sq{L.sh_o.as<float4>(), L.sh_meta.as<uint32_t>(), L.sh_dir.as<float4>(), L.sh_c.as<float>(),
                   L.queue_cap};
    launch_raygen(s, pc, sc, rp, q[0], cnt);
    const uint32_t tb = (uint32_t)traverse_block_threads();
    const uint32_t tper = o.trace_blocks_per_cu ? std::min(o.trace_blocks_per_cu, c->trace_blocks_per_cu)
                                                : c->trace_blocks_per_cu;
    const uint32_t tblocks = blocks_for(tper, c->cu_count, pc.n_paths, tb);
    // Shade block: the largest when the piece has at least 64 samples per
    // pixel (a block then spans a few pixels and its appends are grouped by
    // direction), else 256 threads in pixel order (4-pair batch at 16
    // samples per round: 5.88 s with 512-thread grouped blocks, 5.69 s with
    // 256-thread grouped blocks, 5.40 s with 256 threads in pixel order).
    const uint32_t smax = (uint32_t)shade_block_threads();
    const uint32_t sthreads = pc.bp >= 64 ? smax : std::min<uint32_t>(256, smax);
    const uint32_t sblocks = blocks_for(c->shade_blocks_per_cu * (smax / sthreads), c->cu_count, pc.n_paths,
                                        sthreads);
    const bool count = o.count_work != 0;
    for (uint32_t d = 1; d <= rp.max_depth; ++d) {
        const RayQueue &qin = q[(d - 1) & 1];
        const RayQueue &qout = q[d & 1];
        const size_t slice = (size_t)(d - 1) * pc.n_paths;
        float2 *hit_log = log ? log->hit + slice : nullptr;
        uint32_t *vis_log = log && log->vis ? log->vis + slice : nullptr;
        if (!(log && log->replay)) {
            const EventPair ec = prof.take(0);
            launch_trace_closest(s, tblocks, count, sc, qin, cnt + kCntRay0 + 2 * (d - 1), pc.region, pc.n_inst,
                                 pc.inst_base, L.hit.as<float2>(), d == 1 ? kStatCamera : kStatExtension, stat,
                                 ec.a, ec.b);
            c->stats.n_closest_launches++;
        }
        launch_shade(s, sblocks, pc, sc, rp, qin, cnt + kCntRay0 + 2 * (d - 1), L.hit.as<float2>(), qout,
                     cnt + kCntRay0 + 2 * d, sq, cnt + kCntShadow0 + 2 * d, d, sthreads, adj, hit_log);
        if (rp.nee) {
            const EventPair es = prof.take(1);
            launch_trace_shadow(s, tblocks, count, sc, sq, rp.n_slots, cnt + kCntShadow0 + 2 * d, pc.region,
                                pc.n_inst, pc.inst_base, pc.rad, stat, es.a, es.b, adj, vis_log);
            if (!(vis_log && adj)) c->stats.n_shadow_launches++;
        }
    }
    c->stats.pieces++;
    c->stats.paths += pc.n_paths;
}

static double crit_value(evrt_ctx *c, double p, uint32_t df)
{
    uint64_t bits;
    std::memcpy(&bits, &p, 8);
    auto key = std::make_pair(bits, df);
    auto it = c->crit_cache.find(key);
    if (it != c->crit_cache.end()) return it->second;
    const double q = t_quantile(p, df);
    c->crit_cache[key] = q;
    return q;
}

// Tests of a round's checkpoints.  Pooled degrees of freedom that follow
// from the schedule (m0 mini-batches at the first instant: the checkpoint's
// own count in lock step, m0_fixed when the first instant holds a fixed
// count) become critical values per checkpoint; Welch degrees of freedom,
// or a first instant whose count differs per pixel (a video reference),
// make every pixel compare its own tail probability with alpha.
static void set_tests(evrt_ctx *c, Decide &dc, const evrt_render_opts &o, float alpha, uint32_t spp_max,
                      uint32_t m0_fixed, bool per_pixel_ref)
{
    dc.alpha = (double)alpha;
    dc.df_mode = o.df_mode;
    dc.df_per_pixel = (o.df_mode == EVRT_DF_WELCH || per_pixel_ref) ? 1u : 0u;
    dc.normality_alpha = (double)o.normality_alpha;
    if (dc.df_per_pixel) return;
    for (uint32_t j = 0; j < dc.n_checks; ++j) {
        if (dc.ck_end[j] >= spp_max) break;
        const uint32_t m1 = dc.ck_end[j] / dc.minibatch;
        const uint32_t m0 = m0_fixed ? m0_fixed : m1;
        const uint32_t df = m0 + m1 - 2;
        if (o.mode == EVRT_MODE_ADAPTIVE_1T) {
            dc.crit_lo[j] = crit_value(c, (double)alpha, df);
        } else if (o.mode == EVRT_MODE_ADAPTIVE_2T) {
            dc.crit_lo[j] = crit_value(c, 0.5 * (double)alpha, df);
            dc.crit_hi[j] = crit_value(c, 1.0 - 0.5 * (double)alpha, df);
        }
    }
}

// Pieces covering samples [lo, hi) of nA pixels at n_inst instants.  A
// piece holds at most `ray_batch` paths: blocks of consecutive active pixels
// with the whole sample range when that fits, otherwise every pixel with a
// sub-range of whole mini-batches.  Each pixel's samples are accumulated in
// increasing order either way.
// Entries per block when a round's n entries (pixels or items, each with
// its whole sample range) are cut into blocks of at most `block`: with two
// lanes, an even number (at least two) of equal blocks, so that both lanes
// get the same work and finish together.
static uint64_t balanced_block(const evrt_ctx *c, uint64_t n, uint64_t block)
{
    if (!c->s2 || n < 128) return block;
    uint64_t nb = (n + block - 1) / block;
    nb = std::max<uint64_t>(2, nb + (nb & 1));
    return (n + nb - 1) / nb;
}

static bool trace_range(evrt_ctx *c, const uint32_t *act, uint32_t nA, uint32_t n_inst, uint32_t inst_base,
                        uint32_t lo, uint32_t hi, const DevScene &sc, const RenderParams &rp,
                        const evrt_render_opts &o, hipStream_t s, Profiler &prof, const Decide *dc = nullptr,
                        uint32_t *act_out = nullptr, const Outputs *outs = nullptr)
{
    const uint32_t mb = rp.minibatch;
    // With two lanes a piece holds half of the paths in flight.
    const uint64_t full = o.ray_batch ? o.ray_batch : kDefaultRayBatch;
    const uint64_t batch = c->s2 ? (full + 1) / 2 : full;
    const uint64_t range = hi - lo;
    const uint64_t per_px = (uint64_t)n_inst * range;
    uint64_t px_block = std::max<uint64_t>(1, batch / per_px);
    uint64_t bp_max = range;
    if (px_block < 64 && px_block < nA) {
        // Too few pixels per block: split the samples instead.
        px_block = nA;
        bp_max = std::max<uint64_t>(mb, batch / ((uint64_t)nA * n_inst) / mb * mb);
    }
    px_block = std::min<uint64_t>(px_block, nA);
    bp_max = std::min<uint64_t>(bp_max, (uint64_t)(kMaxPathId - 1) / (px_block * n_inst) / mb * mb);
    if (bp_max == 0) fail(EVRT_E_UNSUPPORTED, "too many pixels for one piece");
    if (bp_max >= range) px_block = balanced_block(c, nA, px_block);
    // Pieces that hold the whole range of their pixels also take the
    // decisions; split sample ranges leave them to a separate kernel.
    const bool fused = dc != nullptr && bp_max >= range;
    if (dc != nullptr && !fused && dc->n_checks != 1) fail(EVRT_E_UNSUPPORTED, "checkpoints over split samples");
    // Consecutive pieces alternate between the caller's stream and the
    // second lane's, ordered after the work already on the caller's stream
    // and joined back before the decisions that follow.
    // Split sample ranges of one pixel block must be accumulated in order:
    // they stay on one stream.
    const uint64_t n_pieces = ((nA + px_block - 1) / px_block) * ((range + bp_max - 1) / bp_max);
    const bool two = c->s2 != nullptr && n_pieces > 1 && bp_max >= range;
    if (two) {
        hip_check(hipEventRecord(c->ev_fork, s), "fork");
        hip_check(hipStreamWaitEvent(c->s2, c->ev_fork, 0), "fork wait");
    }
    uint32_t piece = 0;
    for (uint32_t a0 = 0; a0 < nA; a0 += (uint32_t)px_block) {
        const uint32_t na = (uint32_t)std::min<uint64_t>(px_block, nA - a0);
        for (uint32_t s0 = lo; s0 < hi;) {
            const uint32_t bp = (uint32_t)std::min<uint64_t>(bp_max, hi - s0);
            Piece pc{};
            pc.act = act + a0;
            pc.nA = na;
            pc.bp = bp;
            pc.n_inst = n_inst;
            pc.inst_base = inst_base;
            pc.s0 = s0;
            pc.n_paths = na * n_inst * bp;
            pc.region = na * bp;
            pc.div_bp = make_fastdiv(bp);
            pc.div_nA = make_fastdiv(na);
            pc.rs_a = bp;
            pc.rs_i = na * bp;
            const int ln = two ? (int)(piece & 1u) : 0;
            hipStream_t ps = ln ? c->s2 : s;
            ++piece;
            ensure_buffers(c, sc.width * sc.height, pc.n_paths, rp.n_slots, ln);
            pc.rad = c->fb.lane[ln].rad.as<float>();
            trace_piece(c, pc, sc, rp, o, ps, prof, ln);
            if (fused)
                launch_accumulate_decide(ps, pc, rp, *dc, act_out, c->fb.cnt.as<uint32_t>(),
                                         c->fb.wf_n.as<uint32_t>(), c->fb.wf_mean.as<double>(),
                                         c->fb.wf_m2.as<double>(), c->fb.wf_ysum.as<double>(), *outs);
            else
                launch_accumulate(ps, pc, rp, c->fb.wf_n.as<uint32_t>(), c->fb.wf_mean.as<double>(),
                                  c->fb.wf_m2.as<double>(), c->fb.wf_ysum.as<double>());
            s0 += bp;
        }
    }
    if (two) {
        hip_check(hipEventRecord(c->ev_join, c->s2), "join");
        hip_check(hipStreamWaitEvent(s, c->ev_join, 0), "join wait");
    }
    return fused;
}

static void read_stats(evrt_ctx *c, hipStream_t s)
{
    hip_check(hipMemcpyAsync(c->h_stat, c->fb.stat.ptr, sizeof(unsigned long long) * kStatCount,
                             hipMemcpyDeviceToHost, s),
              "stat readback");
    hip_check(hipStreamSynchronize(s), "stat readback");
    c->stats.camera_rays = c->h_stat[kStatCamera];
    c->stats.extension_rays = c->h_stat[kStatExtension];
    c->stats.shadow_rays = c->h_stat[kStatShadow];
    c->stats.node_visits = c->h_stat[kStatNodes];
    c->stats.tri_tests = c->h_stat[kStatTris];
    c->stats.node_visits_shadow = c->h_stat[kStatNodesShadow];
    c->stats.tri_tests_shadow = c->h_stat[kStatTrisShadow];
}

// The adaptive rounds of one pair over the active list (every pixel of
// fb.act0 at entry): both instants in lock step, or only the second one
// against a first instant already held at the full count (ref_full).
// ref_per_pixel: the first instant holds a count of its own per pixel (a
// video reference), so the tests take each pixel's degrees of freedom.
static void run_rounds(evrt_ctx *c, const DevScene &sc, const RenderParams &rp, const evrt_render_opts &o,
                       float C, float alpha, uint32_t spp_init, uint32_t spp_batch, uint32_t spp_max,
                       bool ref_full, uint32_t nA, const Outputs &outs, hipStream_t s, Profiler &prof,
                       bool ref_per_pixel = false)
{
    FrameBuffers &fb = c->fb;
    const uint32_t mb = o.minibatch;
    const uint32_t batch = o.ray_batch ? o.ray_batch : kDefaultRayBatch;
    const bool fixed = o.mode == EVRT_MODE_FIXED;
    uint32_t *act_in = fb.act0.as<uint32_t>();
    uint32_t *act_out = fb.act1.as<uint32_t>();
    const uint32_t n_inst = ref_full ? 1 : 2;
    const uint32_t inst_base = ref_full ? 1 : 0;
    uint32_t n_prev = 0;
    uint32_t n_next = fixed ? spp_max : spp_init;  // first checkpoint of the next round
    for (uint32_t r = 0;; ++r) {
        // Checkpoints of this round: the schedule's next sample counts, as
        // many as keep the round's paths within one batch (at least one).
        // Every checkpoint is tested in order, so a pixel stops exactly
        // where one checkpoint per round would stop it; samples traced past
        // its stop are the price of fuller launches.
        Decide dc{};
        dc.C = (double)C;
        dc.mode = o.mode;
        dc.minibatch = mb;
        dc.cnt_slot = r & 1u;
        uint32_t hi = n_next;
        dc.ck_end[0] = hi;
        dc.n_checks = 1;
        while (hi < spp_max && dc.n_checks < kMaxChecks) {
            const uint32_t nx = std::min(hi + spp_batch, spp_max);
            if ((uint64_t)nA * n_inst * (nx - n_prev) > batch) break;
            hi = nx;
            dc.ck_end[dc.n_checks++] = hi;
        }
        dc.final_round = hi >= spp_max ? 1u : 0u;
        set_tests(c, dc, o, alpha, spp_max, ref_full ? spp_max / mb : 0u, ref_per_pixel);
        const bool fused = trace_range(c, act_in, nA, n_inst, inst_base, n_prev, hi, sc, rp, o, s, prof, &dc,
                                       act_out, &outs);
        if (!fused)
            launch_decide_compact(s, rp, dc, act_in, nA, act_out, fb.cnt.as<uint32_t>(), fb.wf_n.as<uint32_t>(),
                                  fb.wf_mean.as<double>(), fb.wf_m2.as<double>(), fb.wf_ysum.as<double>(),
                                  outs);
        hip_check(hipMemcpyAsync(c->h_pinned, fb.cnt.as<uint32_t>() + kCntActive + dc.cnt_slot, sizeof(uint32_t),
                                 hipMemcpyDeviceToHost, s),
                  "active count readback");
        hip_check(hipStreamSynchronize(s), "round");
        const uint32_t next = c->h_pinned[0];
        if (c->stats.rounds < 64) c->stats.active_after_round[c->stats.rounds] = next;
        c->stats.rounds += 1;
        std::swap(act_in, act_out);
        nA = next;
        if (nA == 0 || dc.final_round) break;
        n_prev = hi;
        n_next = std::min(hi + spp_batch, spp_max);
    }
}

// Work buffers of a frame of npx pixels with paths in flight per piece.
static void frame_buffers(evrt_ctx *c, uint32_t npx, uint32_t spp_max, const evrt_render_opts &o,
                          uint32_t n_slots)
{
    const uint32_t mb = o.minibatch;
    // Largest piece of the frame: at most ray_batch paths (half with two
    // lanes), or one mini-batch of every pixel when that is larger, or 64
    // pixels' ranges.
    const uint32_t full = o.ray_batch ? o.ray_batch : kDefaultRayBatch;
    const uint32_t batch = c->s2 ? (full + 1) / 2 : full;
    const uint64_t all = 2ull * npx * spp_max;
    const uint64_t floor_piece = std::min<uint64_t>(2ull * npx * mb, 2ull * 64 * spp_max);
    const uint64_t cap = std::max<uint64_t>(std::min<uint64_t>(batch, all), floor_piece);
    if (cap >= kMaxPathId) fail(EVRT_E_UNSUPPORTED, "image too large for one mini-batch piece");
    ensure_buffers(c, npx, (uint32_t)cap, n_slots);
}

// Row order of a frame's first active list: rows by their bit-reversed
// index (van der Corput order), so that cutting the list into 2, 4, 8 ...
// equal blocks gives each block rows spread over the whole image and the
// two lanes' pieces of the first round alike work (with the rows in image
// order the lanes of the sensor frame's first round ended 3.6 ms apart).
static const uint32_t *first_rows(evrt_ctx *c, uint32_t height, hipStream_t s)
{
    FrameBuffers &fb = c->fb;
    if (fb.row_order_h.size() != height) {
        uint32_t bits = 0;
        while ((1u << bits) < height) ++bits;
        std::vector<std::pair<uint32_t, uint32_t>> key(height);
        for (uint32_t r = 0; r < height; ++r) {
            uint32_t v = 0;
            for (uint32_t b = 0; b < bits; ++b) v |= ((r >> b) & 1u) << (bits - 1 - b);
            key[r] = {v, r};
        }
        std::sort(key.begin(), key.end());
        fb.row_order_h.resize(height);
        for (uint32_t k = 0; k < height; ++k) fb.row_order_h[k] = key[k].second;
        fb.row_order.upload(fb.row_order_h.data(), sizeof(uint32_t) * height, s);
    }
    return fb.row_order.as<uint32_t>();
}

void render_frame(evrt_ctx *c, double t0, double t1, float C, float alpha, uint32_t spp_init,
                  uint32_t spp_batch, uint32_t spp_max, const evrt_render_opts &o,
                  const evrt_frame_out &out, hipStream_t s)
{
    const auto wall0 = std::chrono::steady_clock::now();
    std::memset(&c->stats, 0, sizeof(c->stats));
    auto [ga, gb] = get_pair(c, t0, t1, s, &c->stats.ms_build);
    const DevScene sc = make_dev_scene(c, *ga, *gb, o.lds_nodes);
    const RenderParams rp = make_params(c, o);
    const uint32_t npx = sc.width * sc.height;
    frame_buffers(c, npx, spp_max, o, rp.n_slots);
    FrameBuffers &fb = c->fb;
    const uint32_t *rows = first_rows(c, sc.height, s);
    launch_init_frame(s, npx, fb.wf_n.as<uint32_t>(), fb.wf_mean.as<double>(), fb.wf_m2.as<double>(),
                      fb.wf_ysum.as<double>(), fb.act0.as<uint32_t>(), fb.cnt.as<uint32_t>(),
                      fb.stat.as<unsigned long long>(), sc.width, rows);
    Profiler prof{c, o.profile != 0, 0, {}};
    const bool ref_full = o.ref_mode == EVRT_REF_FULL;
    if (ref_full) {
        // The first instant at the full count for every pixel.
        trace_range(c, fb.act0.as<uint32_t>(), npx, 1, 0, 0, spp_max, sc, rp, o, s, prof);
    }
    Outputs outs{out.polarity, out.n_paths, out.mean, out.var, out.t_last, out.mean_radiance, out.flags};
    run_rounds(c, sc, rp, o, C, alpha, spp_init, spp_batch, spp_max, ref_full, npx, outs, s, prof);
    read_stats(c, s);
    prof.collect(c->stats);
    c->stats.ms_wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
}

// Sequential event video over frames times[0 .. n_frames): frame 0 at the
// full count fills the reference slot of every pixel; each later frame k is
// sampled adaptively against the pixel's reference (frame keys key_base + k)
// and replaces it where the frame fires an event.  Outputs frame-major.
// Host builds of the instants a frame loop needs next, on worker threads
// while the calling thread drives the device: at most `depth` frames ahead
// (geometry that moves; a static scene shares one instant).  take() uploads
// and caches a frame's instant, waiting for its build if needed; the
// destructor waits for builds still running (their results are dropped).
class InstantPrefetch {
public:
    InstantPrefetch(evrt_ctx *c, const double *times, uint32_t n, uint32_t depth)
        : c_(c), times_(times), n_(n), depth_(c->static_geom ? 0u : depth)
    {
    }

    std::shared_ptr<DevInstantBufs> take(uint32_t k, hipStream_t s, double *ms_build)
    {
        launch_upto(std::min(n_, k + 1 + depth_));
        const double t = times_[k];
        auto it = inflight_.find(t);
        if (it == inflight_.end()) return get_instant(c_, t, s, ms_build);
        const auto t0 = std::chrono::steady_clock::now();
        std::shared_ptr<DevInstantBufs> bi = it->second.get();  // rethrows a build's error
        inflight_.erase(it);
        upload_instant(c_, *bi, s);
        cache_insert(c_, t, bi);
        if (ms_build)
            *ms_build += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return bi;
    }

private:
    void launch_upto(uint32_t end)
    {
        for (; next_ < end; ++next_) {
            const double t = times_[next_];
            if (c_->cache.count(t) || inflight_.count(t)) continue;
            const evrt_ctx *cc = c_;
            inflight_[t] = std::async(std::launch::async, [cc, t] {
                auto bi = std::make_shared<DevInstantBufs>();
                build_host_instant(cc, t, bi->host);
                return bi;
            });
        }
    }

    evrt_ctx *c_;
    const double *times_;
    uint32_t n_, depth_;
    uint32_t next_ = 0;
    std::map<double, std::future<std::shared_ptr<DevInstantBufs>>> inflight_;
};

void render_video(evrt_ctx *c, uint32_t n_frames, const double *times, float C, float alpha, uint32_t spp_init,
                  uint32_t spp_batch, uint32_t spp_max, const evrt_render_opts &o, const evrt_frame_out &out,
                  hipStream_t s)
{
    const auto wall0 = std::chrono::steady_clock::now();
    std::memset(&c->stats, 0, sizeof(c->stats));
    // The next frames' geometry is built on host threads while the device
    // renders (a frame's host build costs about as much as its tracing on
    // the sensor scene).  The cache keeps the frames in flight.
    const uint32_t ahead = std::min(8u, std::max(1u, std::thread::hardware_concurrency() / 2));
    c->cache_cap = std::max<size_t>(c->cache_cap, (size_t)ahead + 3);
    InstantPrefetch pre(c, times, n_frames, ahead);
    auto g0 = pre.take(0, s, &c->stats.ms_build);
    const DevScene sc0 = make_dev_scene(c, *g0, *g0, o.lds_nodes);
    const RenderParams rp0 = make_params(c, o);
    const uint32_t npx = sc0.width * sc0.height;
    frame_buffers(c, npx, spp_max, o, rp0.n_slots);
    FrameBuffers &fb = c->fb;
    const uint32_t *rows = first_rows(c, sc0.height, s);
    launch_init_frame(s, npx, fb.wf_n.as<uint32_t>(), fb.wf_mean.as<double>(), fb.wf_m2.as<double>(),
                      fb.wf_ysum.as<double>(), fb.act0.as<uint32_t>(), fb.cnt.as<uint32_t>(),
                      fb.stat.as<unsigned long long>(), sc0.width, rows);
    Profiler prof{c, o.profile != 0, 0, {}};
    trace_range(c, fb.act0.as<uint32_t>(), npx, 1, 0, 0, spp_max, sc0, rp0, o, s, prof);
    for (uint32_t k = 1; k < n_frames; ++k) {
        auto gk = pre.take(k, s, &c->stats.ms_build);
        const DevScene sc = make_dev_scene(c, *gk, *gk, o.lds_nodes);
        evrt_render_opts ok = o;
        ok.key_base = o.key_base + k - 1;  // the second instant is frame key_base + k
        const RenderParams rp = make_params(c, ok);
        launch_video_frame_init(s, npx, fb.wf_n.as<uint32_t>(), fb.wf_mean.as<double>(), fb.wf_m2.as<double>(),
                                fb.wf_ysum.as<double>(), fb.act0.as<uint32_t>(), fb.cnt.as<uint32_t>(), sc.width,
                                rows);
        const size_t f = (size_t)(k - 1) * npx;
        Outputs outs{out.polarity + f, out.n_paths + f, out.mean + 2 * f, out.var + 2 * f,
                     out.t_last ? out.t_last + f : nullptr, out.mean_radiance ? out.mean_radiance + 2 * f : nullptr,
                     out.flags ? out.flags + f : nullptr};
        // A two-tailed test can fire an event before spp_max (upper tail), so
        // references then hold fewer samples than spp_max.
        run_rounds(c, sc, rp, ok, C, alpha, spp_init, spp_batch, spp_max, true, npx, outs, s, prof,
                   o.mode == EVRT_MODE_ADAPTIVE_2T);
        launch_video_update(s, npx, outs.polarity, fb.wf_n.as<uint32_t>(), fb.wf_mean.as<double>(),
                            fb.wf_m2.as<double>(), fb.wf_ysum.as<double>(), rp.wf_m34);
    }
    read_stats(c, s);
    prof.collect(c->stats);
    c->stats.ms_wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
}

// With EVRT_LOG_ROUNDS set to anything but "0" in the environment, a batch
// prints one line per round to stderr, so that a call of many minutes shows
// how far it has got.  Read once per process.
static bool log_rounds()
{
    static const bool on = [] {
        const char *v = std::getenv("EVRT_LOG_ROUNDS");
        return v != nullptr && *v != '\0' && std::strcmp(v, "0") != 0;
    }();
    return on;
}

// A batch of consecutive pairs (times[k], times[k+1]), k < n_pairs, of a
// scene whose geometry is the same at every time (the camera may move).
// Frame f is keyed as key_base + f, so pair k equals render_frame of
// (times[k], times[k+1]) with key_base + k bit for bit; the frames a pair
// shares with its neighbours are traced once.  Each round: the items
// (frame, pixel) of the active pairs, pieces of items over the round's
// samples (the checkpoints that fit one batch of paths), Welford updates
// per item, decisions per (pair, pixel).
void render_batch(evrt_ctx *c, uint32_t n_pairs, const double *times, float C, float alpha, uint32_t spp_init,
                  uint32_t spp_batch, uint32_t spp_max, const evrt_render_opts &o, const evrt_frame_out &out,
                  hipStream_t s)
{
    const auto wall0 = std::chrono::steady_clock::now();
    std::memset(&c->stats, 0, sizeof(c->stats));
    const uint32_t nf = n_pairs + 1;
    // Geometry that moves across the batch: every frame's own instant, and
    // each round's items grouped by frame so that a piece holds one frame.
    const bool moving = !instances_static(c->scene, times, nf);
    std::vector<DevScene> frame_sc;
    if (moving) {
        get_instants(c, times, nf, s, &c->stats.ms_build);
        for (uint32_t f = 0; f < nf; ++f) {
            auto gf = get_instant(c, times[f], s, &c->stats.ms_build);
            frame_sc.push_back(make_dev_scene(c, *gf, *gf, o.lds_nodes));
        }
    }
    auto g = get_instant(c, times[0], s, &c->stats.ms_build);
    const DevScene sc = make_dev_scene(c, *g, *g, o.lds_nodes);
    const RenderParams rp = make_params(c, o);
    const uint32_t npx = sc.width * sc.height;
    const uint32_t mb = o.minibatch;
    const uint64_t batch = o.ray_batch ? o.ray_batch : kDefaultRayBatch;
    FrameBuffers &fb = c->fb;
    std::vector<DevCamera> cams(nf);
    for (uint32_t k = 0; k < nf; ++k) camera_at(c->scene, times[k], cams[k]);
    fb.b_cams.upload(cams.data(), sizeof(DevCamera) * nf, s);
    const size_t nfp = (size_t)nf * npx, npp = (size_t)n_pairs * npx;
    fb.b_wf_n.ensure(sizeof(uint32_t) * nfp);
    fb.b_wf_mean.ensure(sizeof(double) * nfp);
    fb.b_wf_m2.ensure(sizeof(double) * nfp);
    fb.b_wf_ysum.ensure(sizeof(double) * nfp);
    fb.b_item_idx.ensure(sizeof(uint32_t) * nfp);
    fb.b_items.ensure(sizeof(uint32_t) * nfp);
    fb.b_act0.ensure(sizeof(uint32_t) * npp);
    fb.b_act1.ensure(sizeof(uint32_t) * npp);
    fb.b_pair_items.ensure(sizeof(uint2) * npp);
    if (moving) {
        fb.b_sorted.ensure(sizeof(uint32_t) * nfp);
        fb.b_sort_tmp.ensure(batch_sort_temp_bytes((uint32_t)nfp));
        fb.b_frame_start.ensure(sizeof(uint32_t) * nf);
        c->h_frame_start.resize(nf);
    }
    ensure_buffers(c, npx, 1, rp.n_slots);
    uint32_t *cnt = fb.cnt.as<uint32_t>();
    uint32_t *wf_n = fb.b_wf_n.as<uint32_t>();
    double *wf_mean = fb.b_wf_mean.as<double>(), *wf_m2 = fb.b_wf_m2.as<double>();
    double *wf_ysum = fb.b_wf_ysum.as<double>();
    uint32_t *item_idx = fb.b_item_idx.as<uint32_t>(), *items = fb.b_items.as<uint32_t>();
    uint2 *pair_items = fb.b_pair_items.as<uint2>();
    launch_init_frame(s, 0, nullptr, nullptr, nullptr, nullptr, nullptr, cnt, fb.stat.as<unsigned long long>());
    uint32_t *act_in = fb.b_act0.as<uint32_t>();
    uint32_t *act_out = fb.b_act1.as<uint32_t>();
    launch_batch_init(s, nf, npx, wf_n, wf_mean, wf_m2, wf_ysum, item_idx, items, act_in, pair_items, cnt);
    Profiler prof{c, o.profile != 0, 0, {}};
    const bool fixed = o.mode == EVRT_MODE_FIXED;
    uint32_t nA = n_pairs * npx;
    uint32_t n_items = nf * npx;
    uint32_t n_prev = 0;
    uint32_t n_next = fixed ? spp_max : spp_init;
    Outputs outs{out.polarity, out.n_paths, out.mean, out.var, out.t_last, out.mean_radiance, out.flags};
    // First item of each frame (round 0 holds every item in frame order).
    std::vector<uint32_t> fstart(nf + 1);
    for (uint32_t f = 0; f <= nf; ++f) fstart[f] = f * npx;
    for (uint32_t r = 0;; ++r) {
        if (r > 0) {
            launch_batch_items(s, act_in, nA, npx, item_idx, items, cnt);
            hip_check(hipMemcpyAsync(c->h_pinned, cnt + kCntItems, sizeof(uint32_t), hipMemcpyDeviceToHost, s),
                      "item count readback");
            hip_check(hipStreamSynchronize(s), "batch items");
            n_items = c->h_pinned[0];
            if (moving) {
                launch_batch_regroup(s, items, n_items, fb.b_sorted.as<uint32_t>(), fb.b_sort_tmp.ptr,
                                     fb.b_sort_tmp.bytes, npx, item_idx, fb.b_frame_start.as<uint32_t>(), nf);
                hip_check(hipGetLastError(), "item regroup");
                hip_check(hipMemcpyAsync(c->h_frame_start.data(), fb.b_frame_start.ptr, sizeof(uint32_t) * nf,
                                         hipMemcpyDeviceToHost, s),
                          "frame start readback");
                hip_check(hipStreamSynchronize(s), "item regroup");
                // Frames without items start where the next frame does.
                fstart[nf] = n_items;
                for (uint32_t f = nf; f-- > 0;)
                    fstart[f] = c->h_frame_start[f] == 0xffffffffu ? fstart[f + 1] : c->h_frame_start[f];
            }
            launch_batch_pair_items(s, act_in, nA, npx, item_idx, pair_items);
        }
        Decide dc{};
        dc.C = (double)C;
        dc.mode = o.mode;
        dc.minibatch = mb;
        dc.cnt_slot = r & 1u;
        uint32_t hi = n_next;
        dc.ck_end[0] = hi;
        dc.n_checks = 1;
        while (hi < spp_max && dc.n_checks < kMaxChecks) {
            const uint32_t nx = std::min(hi + spp_batch, spp_max);
            if ((uint64_t)n_items * (nx - n_prev) > batch) break;
            hi = nx;
            dc.ck_end[dc.n_checks++] = hi;
        }
        dc.final_round = hi >= spp_max ? 1u : 0u;
        set_tests(c, dc, o, alpha, spp_max, 0u, false);
        double *snap = nullptr;
        if (dc.n_checks > 1) {
            fb.b_snap.ensure(sizeof(double) * 3 * (size_t)n_items * dc.n_checks);
            snap = fb.b_snap.as<double>();
        }
        // Pieces over the items: blocks of items with the whole sample range,
        // or every item over sub-ranges when the blocks would be too small
        // (then the round has one checkpoint).  With two lanes a piece holds
        // half of the paths in flight and consecutive pieces alternate
        // streams, as in the single-pair rounds.
        const uint64_t range = hi - n_prev;
        const uint64_t pbatch = c->s2 ? (batch + 1) / 2 : batch;
        // Item ranges traced with one geometry: all items, or each frame's.
        struct Span {
            uint32_t a_begin, a_end;
            const DevScene *scene;
        };
        std::vector<Span> spans;
        if (moving) {
            for (uint32_t f = 0; f < nf; ++f)
                if (fstart[f + 1] > fstart[f]) spans.push_back({fstart[f], fstart[f + 1], &frame_sc[f]});
        } else {
            spans.push_back({0u, n_items, &sc});
        }
        // Blocks of items with the whole sample range, or every item of the
        // span over sub-ranges when the blocks would be too small (then the
        // round has one checkpoint).
        struct Cut {
            uint64_t it_block, bp_max;
            bool split;
        };
        auto cut = [&](uint32_t n) {
            uint64_t it_block = std::max<uint64_t>(1, pbatch / range);
            uint64_t bp_max = range;
            if (it_block < 64 && it_block < n) {
                it_block = n;
                bp_max = std::max<uint64_t>(mb, pbatch / n / mb * mb);
            }
            it_block = std::min<uint64_t>(it_block, n);
            bp_max = std::min<uint64_t>(bp_max, (uint64_t)(kMaxPathId - 1) / it_block / mb * mb);
            if (bp_max == 0) fail(EVRT_E_UNSUPPORTED, "too many items for one piece");
            const bool split = bp_max < range;
            // Two lanes of one span get equal blocks; many frames' spans
            // alternate between the lanes anyway.
            if (!split && !moving) it_block = balanced_block(c, n, it_block);
            if (dc.n_checks > 1 && split) fail(EVRT_E_UNSUPPORTED, "checkpoints over split samples");
            return Cut{it_block, bp_max, split};
        };
        uint64_t n_pieces = 0;
        bool any_split = false;
        for (const Span &sp : spans) {
            const Cut ct = cut(sp.a_end - sp.a_begin);
            n_pieces += ((sp.a_end - sp.a_begin + ct.it_block - 1) / ct.it_block) * ((range + ct.bp_max - 1) / ct.bp_max);
            any_split = any_split || ct.split;
        }
        // Split sample ranges of one item must be accumulated in order: they
        // stay on one stream.
        const bool two = c->s2 != nullptr && n_pieces > 1 && !any_split;
        if (two) {
            hip_check(hipEventRecord(c->ev_fork, s), "fork");
            hip_check(hipStreamWaitEvent(c->s2, c->ev_fork, 0), "fork wait");
        }
        uint32_t piece = 0;
        for (const Span &sp : spans) {
          const Cut ct = cut(sp.a_end - sp.a_begin);
          const uint64_t it_block = ct.it_block, bp_max = ct.bp_max;
          for (uint32_t a0 = sp.a_begin; a0 < sp.a_end; a0 += (uint32_t)it_block) {
            const uint32_t na = (uint32_t)std::min<uint64_t>(it_block, sp.a_end - a0);
            for (uint32_t s0 = n_prev; s0 < hi;) {
                const uint32_t bp = (uint32_t)std::min<uint64_t>(bp_max, hi - s0);
                Piece pc{};
                pc.act = items + a0;
                pc.nA = na;
                pc.bp = bp;
                pc.n_inst = 1;
                pc.inst_base = 0;
                pc.s0 = s0;
                pc.n_paths = na * bp;
                pc.region = na * bp;
                pc.div_bp = make_fastdiv(bp);
                pc.div_nA = make_fastdiv(na);
                pc.rs_a = bp;
                pc.rs_i = na * bp;
                pc.cams = fb.b_cams.as<DevCamera>();
                const int ln = two ? (int)(piece & 1u) : 0;
                hipStream_t ps = ln ? c->s2 : s;
                ++piece;
                ensure_buffers(c, npx, pc.n_paths, rp.n_slots, ln);
                pc.rad = fb.lane[ln].rad.as<float>();
                trace_piece(c, pc, *sp.scene, rp, o, ps, prof, ln);
                launch_batch_accumulate(ps, pc, rp, dc, npx, a0, wf_n, wf_mean, wf_m2, wf_ysum, snap);
                s0 += bp;
            }
          }
        }
        if (two) {
            hip_check(hipEventRecord(c->ev_join, c->s2), "join");
            hip_check(hipStreamWaitEvent(s, c->ev_join, 0), "join wait");
        }
        launch_batch_decide(s, dc, act_in, nA, npx, pair_items, items, wf_n, wf_mean, wf_m2, wf_ysum, snap,
                            act_out, cnt, outs);
        launch_batch_clear(s, items, n_items, npx, item_idx, cnt);
        hip_check(hipMemcpyAsync(c->h_pinned, cnt + kCntActive + dc.cnt_slot, sizeof(uint32_t),
                                 hipMemcpyDeviceToHost, s),
                  "active count readback");
        hip_check(hipStreamSynchronize(s), "batch round");
        const uint32_t next = c->h_pinned[0];
        if (r < 64) c->stats.active_after_round[r] = next;
        c->stats.rounds = r + 1;
        if (log_rounds()) {
            std::fprintf(stderr, "evrt: batch round %u: %u items over samples [%u, %u) in %u checkpoints, "
                         "%u of %u (pair, pixel) entries still undecided, %.1f s\n", r, n_items, n_prev, hi,
                         dc.n_checks, next, nA,
                         std::chrono::duration<double>(std::chrono::steady_clock::now() - wall0).count());
            std::fflush(stderr);
        }
        std::swap(act_in, act_out);
        nA = next;
        if (nA == 0 || dc.final_round) break;
        n_prev = hi;
        n_next = std::min(hi + spp_batch, spp_max);
    }
    read_stats(c, s);
    prof.collect(c->stats);
    c->stats.ms_wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - wall0).count();
}

// Every path sample s in [0, spp) of the listed pixels at both instants, in
// pieces of the usual wavefront; radiances go to L_out[pixel][instant][s].
// With adj, the pieces are the adjoint replay (same keys, same arithmetic).
// log: the gradient's ray log over all pieces (piece at pixel a0 starts
// at entry a0 * 2 spp * max_depth), or null.  Pieces alternate between the
// caller's stream and the second lane's, in an even number of equal pixel
// blocks, as in the frame.
static void trace_paths(evrt_ctx *c, const DevScene &sc, const RenderParams &rp, const evrt_render_opts &o,
                        uint32_t n_pixels, const uint32_t *pixels, uint32_t spp, float *L_out,
                        const Adjoint *adj, hipStream_t s, const RayLog *log = nullptr)
{
    const uint32_t npx = sc.width * sc.height;
    const uint32_t batch = o.ray_batch ? o.ray_batch : kDefaultRayBatch;
    const uint64_t per_px = 2ull * spp;
    const uint64_t block = std::max<uint64_t>(1, std::min<uint64_t>(n_pixels, batch / per_px));
    const uint32_t chunk = (uint32_t)balanced_block(c, n_pixels, block);
    const bool two = c->s2 != nullptr && n_pixels > chunk;
    const uint32_t cap = (uint32_t)std::min<uint64_t>((uint64_t)chunk * per_px, kMaxPathId - 1);
    for (int ln = 0; ln < (two ? 2 : 1); ++ln) ensure_buffers(c, npx, cap, rp.n_slots, ln);
    Adjoint a[2]{};
    if (adj) {
        // Weight and emitter of each shadow entry (queue slots of the lane).
        FrameBuffers &fb = c->fb;
        for (int ln = 0; ln < (two ? 2 : 1); ++ln) {
            const uint32_t qcap = fb.lane[ln].queue_cap;
            fb.diff_sw[ln].ensure(sizeof(double) * qcap);
            fb.diff_semat[ln].ensure(sizeof(uint32_t) * qcap);
            a[ln] = *adj;
            a[ln].sw = fb.diff_sw[ln].as<double>();
            a[ln].semat = fb.diff_semat[ln].as<uint32_t>();
        }
    }
    launch_init_frame(s, 0, nullptr, nullptr, nullptr, nullptr, nullptr, c->fb.cnt.as<uint32_t>(),
                      c->fb.stat.as<unsigned long long>());
    if (two) {
        hip_check(hipEventRecord(c->ev_fork, s), "fork");
        hip_check(hipStreamWaitEvent(c->s2, c->ev_fork, 0), "fork wait");
    }
    Profiler prof{c, false, 0, {}};
    uint32_t piece = 0;
    for (uint32_t a0 = 0; a0 < n_pixels; a0 += chunk) {
        const uint32_t na = std::min(chunk, n_pixels - a0);
        Piece pc{};
        pc.act = pixels + a0;
        pc.nA = na;
        pc.bp = spp;
        pc.n_inst = 2;
        pc.inst_base = 0;
        pc.s0 = 0;
        pc.n_paths = (uint32_t)(per_px * na);
        pc.region = na * spp;
        pc.div_bp = make_fastdiv(spp);
        pc.div_nA = make_fastdiv(na);
        pc.rad = L_out + (size_t)a0 * per_px;  // [pixel][instant][sample]
        pc.rs_a = 2 * spp;
        pc.rs_i = spp;
        RayLog pl{};
        if (log) {
            const size_t base = (size_t)a0 * per_px * rp.max_depth;
            pl.hit = log->hit + base;
            pl.vis = log->vis ? log->vis + base : nullptr;
            pl.replay = log->replay;
        }
        const int ln = two ? (int)(piece & 1u) : 0;
        ++piece;
        trace_piece(c, pc, sc, rp, o, ln ? c->s2 : s, prof, ln, adj ? &a[ln] : nullptr, log ? &pl : nullptr);
    }
    if (two) {
        hip_check(hipEventRecord(c->ev_join, c->s2), "join");
        hip_check(hipStreamWaitEvent(s, c->ev_join, 0), "join wait");
    }
}

void render_paths(evrt_ctx *c, double t0, double t1, uint32_t n_pixels, const uint32_t *pixels,
                  uint32_t spp, const evrt_render_opts &o, float *L_out, hipStream_t s)
{
    std::memset(&c->stats, 0, sizeof(c->stats));
    auto [ga, gb] = get_pair(c, t0, t1, s, &c->stats.ms_build);
    const DevScene sc = make_dev_scene(c, *ga, *gb, o.lds_nodes);
    const RenderParams rp = make_params(c, o);
    trace_paths(c, sc, rp, o, n_pixels, pixels, spp, L_out, nullptr, s);
    read_stats(c, s);
}

// Smoothed event loss at spp paths per pixel and instant and its gradient:
// forward path radiances of every pixel (the wavefront renderer), per-pixel
// statistics and mini-batch weights, then the path-replay adjoint.
void event_loss_grad(evrt_ctx *c, double t0, double t1, float C, float tau, uint32_t spp,
                     const evrt_render_opts &o, const evrt_diff_out &out, hipStream_t s, const double *upstream,
                     bool delta_only)
{
    std::memset(&c->stats, 0, sizeof(c->stats));
    auto [ga, gb] = get_pair(c, t0, t1, s, &c->stats.ms_build);
    const uint32_t npx = c->scene.cam.width * c->scene.cam.height;
    const uint32_t n_mat = (uint32_t)c->scene.albedo.size();
    const uint32_t mb = o.minibatch, m = spp / mb;
    FrameBuffers &fb = c->fb;
    fb.diff_px.ensure(sizeof(uint32_t) * npx);
    {
        std::vector<uint32_t> iota(npx);
        for (uint32_t i = 0; i < npx; ++i) iota[i] = i;
        fb.diff_px.upload(iota.data(), sizeof(uint32_t) * npx, s);
    }
    fb.diff_L.ensure(sizeof(float) * 2 * (size_t)npx * spp);
    fb.diff_W.ensure(sizeof(double) * 2 * (size_t)npx * m);
    launch_diff_zero(s, out.loss, out.grad, out.grad ? 2 * n_mat : 0u, out.replay_mismatch);
    const DevScene sc = make_dev_scene(c, *ga, *gb, o.lds_nodes);
    const RenderParams rp = make_params(c, o);
    // Ray log: the forward pass keeps every ray's closest hit (8 bytes per
    // path and vertex) and, for up to 32 shadow slots without work counting
    // or an LDS treelet, each shadow entry's visibility mask (4 bytes), so
    // that the replay re-shades without tracing.  Above kMaxRayLog bytes or
    // half of the free device memory (besides the log's current buffers), or
    // with replay_retrace set, the replay traces its rays again.
    const uint64_t log_n = 2ull * npx * spp * rp.max_depth;
    const bool vis_ok = rp.nee && rp.n_slots <= 32 && !o.count_work && o.lds_nodes == 0;
    size_t free_b = 0, total_b = 0;
    hip_check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    const uint64_t room =
        std::min<uint64_t>(kMaxRayLog, fb.diff_hitlog.bytes + fb.diff_vislog.bytes + free_b / 2);
    const bool use_log = !delta_only && !o.replay_retrace && log_n * (8 + (vis_ok ? 4 : 0)) <= room;
    RayLog log{};
    if (use_log) {
        fb.diff_hitlog.ensure(sizeof(float2) * log_n);
        log.hit = fb.diff_hitlog.as<float2>();
        if (vis_ok) {
            fb.diff_vislog.ensure(sizeof(uint32_t) * log_n);
            log.vis = fb.diff_vislog.as<uint32_t>();
        }
    }
    trace_paths(c, sc, rp, o, npx, fb.diff_px.as<uint32_t>(), spp, fb.diff_L.as<float>(), nullptr, s,
                use_log ? &log : nullptr);
    launch_diff_stats(s, npx, spp, mb, (double)o.log_eps, (double)C, (double)tau, upstream, fb.diff_L.as<float>(),
                      fb.diff_W.as<double>(), out.loss, out.loss_px, out.delta);
    if (delta_only) {
        read_stats(c, s);
        hip_check(hipGetLastError(), "delta launch");
        return;
    }
    // Adjoint: the same pieces again with the gradient terms of every vertex,
    // then every replayed path radiance against the forward one.
    fb.diff_R.ensure(sizeof(float) * 2 * (size_t)npx * spp);
    Adjoint adj{};
    adj.W = fb.diff_W.as<double>();
    adj.Lfwd = fb.diff_L.as<float>();
    adj.g = out.grad;
    adj.n_mat = n_mat;
    adj.m = m;
    adj.mb = mb;
    adj.spp = spp;
    log.replay = true;
    trace_paths(c, sc, rp, o, npx, fb.diff_px.as<uint32_t>(), spp, fb.diff_R.as<float>(), &adj, s,
                use_log ? &log : nullptr);
    if (out.replay_mismatch)
        launch_diff_compare(s, 2ull * npx * spp, fb.diff_R.as<float>(), fb.diff_L.as<float>(), out.replay_mismatch);
    read_stats(c, s);
    hip_check(hipGetLastError(), "adjoint launch");
}

void trace_rays(evrt_ctx *c, double t, uint32_t n, const float *rays, const uint32_t *skip, int any,
                float *t_out, uint32_t *p_out, hipStream_t s)
{
    std::memset(&c->stats, 0, sizeof(c->stats));
    auto g = get_instant(c, t, s, &c->stats.ms_build);
    const DevScene sc = make_dev_scene(c, *g, *g, (uint32_t)lds_treelet_nodes());
    ensure_buffers(c, sc.width * sc.height, n, 1);
    FrameBuffers &fb = c->fb;
    fb.hook_tm.ensure(sizeof(float) * 2 * (size_t)n);
    RayQueue q{fb.lane[0].q_o[0].as<float4>(), fb.lane[0].q_d[0].as<float4>(), fb.lane[0].q_skip[0].as<uint32_t>()};
    launch_hook_rays(s, n, rays, skip, q, fb.hook_tm.as<float>(), fb.cnt.as<uint32_t>());
    const uint32_t tb = (uint32_t)traverse_block_threads();
    launch_hook_trace(s, blocks_for(c->trace_blocks_per_cu, c->cu_count, n, tb), any != 0, sc, q,
                      fb.hook_tm.as<float>(), n, t_out, p_out);
    hip_check(hipStreamSynchronize(s), "trace hook");
}

void trace_rays_noalloc(evrt_ctx *c, double t, uint32_t n, const float *rays, const uint32_t *skip, int any,
                        float *t_out, uint32_t *p_out, hipStream_t s)
{
    // The geometry at t must already be on the device: cached by an earlier
    // call at t, or, when no instance moves, any cached instant (the camera
    // plays no part in ray queries).
    const DevInstantBufs *g = nullptr;
    auto it = c->cache.find(t);
    if (it != c->cache.end()) g = it->second.get();
    else if (c->static_geom && !c->cache.empty()) g = c->cache.begin()->second.get();
    if (!g) fail(EVRT_E_STATE, "the scene at this time is not resident on the device (trace or render at it first)");
    if (!c->noalloc_scratch) fail(EVRT_E_DEVICE, "no scratch array on this device");
    const DevScene sc = make_dev_scene(c, *g, *g, (uint32_t)lds_treelet_nodes());
    const NoAllocScratch l = noalloc_layout(c->noalloc_scratch);
    RayQueue q{l.o, l.d, l.skip};
    launch_hook_rays(s, n, rays, skip, q, l.tminmax, l.cnt);
    const uint32_t tb = (uint32_t)traverse_block_threads();
    launch_hook_trace(s, blocks_for(c->trace_blocks_per_cu, c->cu_count, n, tb), any != 0, sc, q, l.tminmax, n,
                      t_out, p_out);
    hip_check(hipGetLastError(), "trace hook launch");
}

void decide_stats(evrt_ctx *c, const double *x0, const double *x1, uint32_t n, uint32_t m, float C,
                  float alpha, uint8_t mode, uint8_t df_mode, double *t_out, uint8_t *stop_out, int8_t *pol_out,
                  double *p_out, hipStream_t s)
{
    Decide dc{};
    dc.C = (double)C;
    dc.mode = mode;
    dc.minibatch = 1;
    dc.n_checks = 1;
    dc.ck_end[0] = m;
    evrt_render_opts o{};
    o.mode = mode;
    o.df_mode = df_mode;
    set_tests(c, dc, o, alpha, m + 1, 0u, false);
    launch_hook_decide(s, x0, x1, n, m, dc, t_out, stop_out, pol_out, p_out);
    hip_check(hipStreamSynchronize(s), "decide hook");
}

}  // namespace evrt
