// api.cpp -- the extern "C" boundary: context, scene upload, argument
// validation and error reporting.  Every entry point converts internal
// errors into a status code; nothing throws across the ABI.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "evrt_host.h"

namespace evrt {

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what)
{
    if (e != hipSuccess) fail(EVRT_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

DevBuf::~DevBuf()
{
    if (ptr) (void)hipFree(ptr);
}

void DevBuf::ensure(size_t n)
{
    if (n <= bytes && ptr) return;
    if (ptr) {
        hip_check(hipFree(ptr), "hipFree");
        ptr = nullptr;
        bytes = 0;
    }
    const size_t alloc = n ? n : 16;
    const hipError_t e = hipMalloc(&ptr, alloc);
    if (e != hipSuccess) {
        ptr = nullptr;
        fail(e == hipErrorOutOfMemory ? EVRT_E_NOMEM : EVRT_E_DEVICE,
             std::string("hipMalloc of ") + std::to_string(alloc) + " bytes: " + hipGetErrorString(e));
    }
    bytes = alloc;
}

void DevBuf::upload(const void *src, size_t n, hipStream_t s)
{
    ensure(n);
    if (n) hip_check(hipMemcpyAsync(ptr, src, n, hipMemcpyHostToDevice, s), "upload");
}

void validate_opts(const evrt_render_opts &o)
{
    if (!(o.minibatch == 1 || o.minibatch == 2 || o.minibatch == 4 || o.minibatch == 8))
        fail(EVRT_E_INVALID, "minibatch must be 1, 2, 4 or 8");
    if (o.max_depth < 1 || o.max_depth > (uint32_t)kCntMaxDepth)
        fail(EVRT_E_INVALID, "max_depth must be in [1, 64]");
    if (o.rr_start_depth < 1) fail(EVRT_E_INVALID, "rr_start_depth must be >= 1");
    if (!std::isfinite(o.log_eps) || o.log_eps < 0.0) fail(EVRT_E_INVALID, "log_eps must be finite and >= 0");
    if (o.nee > 1 || o.jitter > 1 || o.profile > 1 || o.count_work > 1)
        fail(EVRT_E_INVALID, "boolean options must be 0 or 1");
    if (o.mode > EVRT_MODE_MEAN_ONLY) fail(EVRT_E_INVALID, "unknown mode");
    if (o.df_mode > EVRT_DF_WELCH) fail(EVRT_E_INVALID, "unknown df_mode");
    if (o.ref_mode > EVRT_REF_FULL) fail(EVRT_E_INVALID, "unknown ref_mode");
    if (o.lds_nodes > (uint32_t)lds_treelet_nodes()) fail(EVRT_E_INVALID, "lds_nodes above the treelet capacity");
    if (o.key_base > (1u << 24)) fail(EVRT_E_INVALID, "key_base above 2^24");
    if (o.replay_retrace > 1) fail(EVRT_E_INVALID, "replay_retrace must be 0 or 1");
    if (o.mis > 1) fail(EVRT_E_INVALID, "mis must be 0 or 1");
    if (!(o.normality_alpha >= 0.0f && o.normality_alpha < 1.0f))
        fail(EVRT_E_INVALID, "normality_alpha must be in [0, 1)");
}

}  // namespace evrt

using namespace evrt;

namespace {

thread_local std::string g_create_error;

template <class F>
int guarded(evrt_ctx *c, F &&f)
{
    try {
        f();
        if (c) c->err.clear();
        return EVRT_OK;
    } catch (const Error &e) {
        if (c) c->err = e.msg;
        else g_create_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        if (c) c->err = "host allocation failed";
        return EVRT_E_NOMEM;
    } catch (...) {
        if (c) c->err = "internal error";
        return EVRT_E_DEVICE;
    }
}

void need_ctx(evrt_ctx *c)
{
    if (!c) fail(EVRT_E_INVALID, "ctx is NULL");
}

void need_device(evrt_ctx *c)
{
    if (c->host_only) fail(EVRT_E_DEVICE, "host-only context has no device");
    hip_check(hipSetDevice(c->device), "hipSetDevice");
}

void need_finite(const double *v, size_t n, const char *what)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) fail(EVRT_E_INVALID, std::string(what) + " must be finite");
}

void need_finite(const float *v, size_t n, const char *what)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) fail(EVRT_E_INVALID, std::string(what) + " must be finite");
}

void scene_changed(evrt_ctx *c) { c->committed = false; }

}  // namespace

#pragma GCC visibility push(default)
extern "C" {

int evrt_abi_version(void) { return EVRT_ABI_VERSION; }

int evrt_create(int hip_device, evrt_ctx **out)
{
    if (!out) {
        g_create_error = "out is NULL";
        return EVRT_E_INVALID;
    }
    *out = nullptr;
    evrt_ctx *c = nullptr;
    const int rc = guarded(nullptr, [&] {
        if (hip_device < -1) fail(EVRT_E_INVALID, "hip_device must be >= -1");
        c = new evrt_ctx();
        if (hip_device >= 0) {
            int n = 0;
            if (hipGetDeviceCount(&n) != hipSuccess || n <= hip_device)
                fail(EVRT_E_DEVICE, "no HIP device " + std::to_string(hip_device));
            hip_check(hipSetDevice(hip_device), "hipSetDevice");
            hipDeviceProp_t prop;
            hip_check(hipGetDeviceProperties(&prop, hip_device), "hipGetDeviceProperties");
            if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
                fail(EVRT_E_UNSUPPORTED, std::string("built for gfx950, device is ") + prop.gcnArchName);
            c->device = hip_device;
            c->host_only = false;
            c->cu_count = (uint32_t)prop.multiProcessorCount;
            int tb = 1, sb = 1;
            kernel_occupancy(&tb, &sb);
            c->trace_blocks_per_cu = (uint32_t)tb;
            c->shade_blocks_per_cu = (uint32_t)sb;
#ifndef EVRT_ONE_LANE
            hip_check(hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking), "hipStreamCreate");
            hip_check(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "hipEventCreate");
            hip_check(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "hipEventCreate");
#endif
            void *p = nullptr;
            hip_check(hipHostMalloc(&p, 64, hipHostMallocDefault), "hipHostMalloc");
            c->h_pinned = static_cast<uint32_t *>(p);
            hip_check(hipHostMalloc(&p, sizeof(unsigned long long) * kStatCount, hipHostMallocDefault),
                      "hipHostMalloc");
            c->h_stat = static_cast<unsigned long long *>(p);
            hip_check(noalloc_scratch_address(hip_device, &c->noalloc_scratch), "hipGetSymbolAddress(scratch)");
        }
    });
    if (rc != EVRT_OK) {
        if (c) evrt_destroy(c);
        return rc;
    }
    *out = c;
    return EVRT_OK;
}

void evrt_destroy(evrt_ctx *c)
{
    if (!c) return;
    if (!c->host_only) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        for (auto &e : c->events) {
            if (e.a) (void)hipEventDestroy(e.a);
            if (e.b) (void)hipEventDestroy(e.b);
        }
        if (c->h_pinned) (void)hipHostFree(c->h_pinned);
        if (c->h_stat) (void)hipHostFree(c->h_stat);
        if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
        if (c->ev_join) (void)hipEventDestroy(c->ev_join);
        if (c->s2) (void)hipStreamDestroy(c->s2);
    }
    delete c;
}

const char *evrt_last_error(const evrt_ctx *c)
{
    return c ? c->err.c_str() : g_create_error.c_str();
}

int evrt_scene_set_materials(evrt_ctx *c, const float *albedo, const float *emission, uint32_t n_mat)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (n_mat == 0 || !albedo || !emission) fail(EVRT_E_INVALID, "need at least one material");
        for (uint32_t i = 0; i < n_mat; ++i) {
            if (!(albedo[i] >= 0.0f && albedo[i] < 1.0f)) fail(EVRT_E_INVALID, "albedo must be in [0, 1)");
            if (!(emission[i] >= 0.0f) || !std::isfinite(emission[i]))
                fail(EVRT_E_INVALID, "emission must be finite and >= 0");
        }
        c->pending.albedo.assign(albedo, albedo + n_mat);
        c->pending.emission.assign(emission, emission + n_mat);
        c->pending.rgb = false;
        c->pending.albedo3.clear();
        c->pending.emission3.clear();
        scene_changed(c);
    });
}

int evrt_scene_set_materials_rgb(evrt_ctx *c, const float *albedo_rgb, const float *emission_rgb, uint32_t n_mat)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (n_mat == 0 || !albedo_rgb || !emission_rgb) fail(EVRT_E_INVALID, "need at least one material");
        for (size_t i = 0; i < 3 * (size_t)n_mat; ++i) {
            if (!(albedo_rgb[i] >= 0.0f && albedo_rgb[i] < 1.0f)) fail(EVRT_E_INVALID, "albedo must be in [0, 1)");
            if (!(emission_rgb[i] >= 0.0f) || !std::isfinite(emission_rgb[i]))
                fail(EVRT_E_INVALID, "emission must be finite and >= 0");
        }
        SceneDesc &p = c->pending;
        p.rgb = true;
        p.albedo3.assign(albedo_rgb, albedo_rgb + 3 * (size_t)n_mat);
        p.emission3.assign(emission_rgb, emission_rgb + 3 * (size_t)n_mat);
        p.albedo.resize(n_mat);
        p.emission.resize(n_mat);
        for (uint32_t i = 0; i < n_mat; ++i) {
            const float *a = albedo_rgb + 3 * (size_t)i, *e = emission_rgb + 3 * (size_t)i;
            p.albedo[i] = std::max(a[0], std::max(a[1], a[2]));
            p.emission[i] = luminance(e[0], e[1], e[2]);
        }
        scene_changed(c);
    });
}

int evrt_scene_set_mesh(evrt_ctx *c, uint32_t mesh_id, const float *xyz, uint32_t nv,
                        const uint32_t *tri_idx, const uint32_t *tri_mat, uint32_t nt)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (mesh_id > (1u << 24)) fail(EVRT_E_INVALID, "mesh_id too large");
        if ((nv && !xyz) || (nt && (!tri_idx || !tri_mat))) fail(EVRT_E_INVALID, "NULL mesh array");
        need_finite(xyz, 3 * (size_t)nv, "vertex coordinates");
        for (size_t i = 0; i < 3 * (size_t)nt; ++i)
            if (tri_idx[i] >= nv) fail(EVRT_E_INVALID, "triangle vertex index out of range");
        if (c->pending.meshes.size() <= mesh_id) c->pending.meshes.resize(mesh_id + 1);
        MeshDesc &m = c->pending.meshes[mesh_id];
        m.set = true;
        m.xyz.assign(xyz, xyz + 3 * (size_t)nv);
        m.idx.assign(tri_idx, tri_idx + 3 * (size_t)nt);
        m.mat.assign(tri_mat, tri_mat + nt);
        scene_changed(c);
    });
}

int evrt_scene_set_instance(evrt_ctx *c, uint32_t inst_id, uint32_t mesh_id, uint32_t n_keys,
                            const double *key_t, const double *xform3x4)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (inst_id > (1u << 24)) fail(EVRT_E_INVALID, "inst_id too large");
        if (n_keys == 0 || !key_t || !xform3x4) fail(EVRT_E_INVALID, "instance needs at least one key");
        need_finite(key_t, n_keys, "key times");
        need_finite(xform3x4, 12 * (size_t)n_keys, "key matrices");
        for (uint32_t k = 1; k < n_keys; ++k)
            if (!(key_t[k] > key_t[k - 1])) fail(EVRT_E_INVALID, "key times must increase");
        if (c->pending.instances.size() <= inst_id) c->pending.instances.resize(inst_id + 1);
        InstanceDesc &in = c->pending.instances[inst_id];
        in.set = true;
        in.mesh = mesh_id;
        in.kt.assign(key_t, key_t + n_keys);
        in.kx.assign(xform3x4, xform3x4 + 12 * (size_t)n_keys);
        scene_changed(c);
    });
}

int evrt_scene_set_point_lights(evrt_ctx *c, const float *pos_xyz, const float *intensity, uint32_t n)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (n && (!pos_xyz || !intensity)) fail(EVRT_E_INVALID, "NULL point light array");
        if (n > 64) fail(EVRT_E_UNSUPPORTED, "at most 64 point lights");
        need_finite(pos_xyz, 3 * (size_t)n, "point light positions");
        for (uint32_t i = 0; i < n; ++i)
            if (!(intensity[i] >= 0.0f) || !std::isfinite(intensity[i]))
                fail(EVRT_E_INVALID, "point light intensity must be finite and >= 0");
        c->pending.pl_pos.assign(pos_xyz, pos_xyz + 3 * (size_t)n);
        c->pending.pl_int.assign(intensity, intensity + n);
        c->pending.pl_int3.clear();
        scene_changed(c);
    });
}

int evrt_scene_set_point_lights_rgb(evrt_ctx *c, const float *pos_xyz, const float *intensity_rgb, uint32_t n)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (n && (!pos_xyz || !intensity_rgb)) fail(EVRT_E_INVALID, "NULL point light array");
        if (n > 64) fail(EVRT_E_UNSUPPORTED, "at most 64 point lights");
        need_finite(pos_xyz, 3 * (size_t)n, "point light positions");
        for (size_t i = 0; i < 3 * (size_t)n; ++i)
            if (!(intensity_rgb[i] >= 0.0f) || !std::isfinite(intensity_rgb[i]))
                fail(EVRT_E_INVALID, "point light intensity must be finite and >= 0");
        SceneDesc &p = c->pending;
        p.pl_pos.assign(pos_xyz, pos_xyz + 3 * (size_t)n);
        p.pl_int3.assign(intensity_rgb, intensity_rgb + 3 * (size_t)n);
        p.pl_int.resize(n);
        for (uint32_t i = 0; i < n; ++i) {
            const float *v = intensity_rgb + 3 * (size_t)i;
            p.pl_int[i] = luminance(v[0], v[1], v[2]);
        }
        scene_changed(c);
    });
}

int evrt_scene_set_camera(evrt_ctx *c, uint32_t width, uint32_t height, double vfov_deg, uint32_t n_keys,
                          const double *key_t, const double *eye_look_up)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (width == 0 || height == 0) fail(EVRT_E_INVALID, "image size must be positive");
        if ((uint64_t)width * height > (1ull << 28)) fail(EVRT_E_UNSUPPORTED, "image larger than 2^28 pixels");
        if (!(vfov_deg > 0.0 && vfov_deg < 180.0)) fail(EVRT_E_INVALID, "vfov_deg must be in (0, 180)");
        if (n_keys == 0 || !key_t || !eye_look_up) fail(EVRT_E_INVALID, "camera needs at least one key");
        need_finite(key_t, n_keys, "camera key times");
        need_finite(eye_look_up, 9 * (size_t)n_keys, "camera keys");
        for (uint32_t k = 1; k < n_keys; ++k)
            if (!(key_t[k] > key_t[k - 1])) fail(EVRT_E_INVALID, "camera key times must increase");
        for (uint32_t k = 0; k < n_keys; ++k) {
            const double *e = eye_look_up + 9 * (size_t)k;
            const double f[3] = {e[3] - e[0], e[4] - e[1], e[5] - e[2]};
            const double r[3] = {f[1] * e[8] - f[2] * e[7], f[2] * e[6] - f[0] * e[8], f[0] * e[7] - f[1] * e[6]};
            if (f[0] * f[0] + f[1] * f[1] + f[2] * f[2] == 0.0 || r[0] * r[0] + r[1] * r[1] + r[2] * r[2] == 0.0)
                fail(EVRT_E_INVALID, "camera look direction is zero or parallel to up");
        }
        CameraDesc &cd = c->pending.cam;
        cd.set = true;
        cd.width = width;
        cd.height = height;
        cd.vfov = vfov_deg;
        cd.kt.assign(key_t, key_t + n_keys);
        cd.elu.assign(eye_look_up, eye_look_up + 9 * (size_t)n_keys);
        scene_changed(c);
    });
}

int evrt_scene_set_environment(evrt_ctx *c, const float *texels, uint32_t face_res)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (face_res > 4096) fail(EVRT_E_UNSUPPORTED, "environment faces above 4096 x 4096 texels");
        if (face_res && !texels) fail(EVRT_E_INVALID, "NULL environment texels");
        const size_t n = 6 * (size_t)face_res * face_res;
        for (size_t i = 0; i < n; ++i)
            if (!(texels[i] >= 0.0f) || !std::isfinite(texels[i]))
                fail(EVRT_E_INVALID, "environment radiance must be finite and >= 0");
        c->pending.env.assign(texels, texels + n);
        c->pending.env_res = face_res;
        scene_changed(c);
    });
}

int evrt_scene_set_lens(evrt_ctx *c, float aperture_radius, float focus_distance)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (!(aperture_radius >= 0.0f) || !std::isfinite(aperture_radius))
            fail(EVRT_E_INVALID, "aperture radius must be finite and >= 0");
        if (!(focus_distance > 0.0f) || !std::isfinite(focus_distance))
            fail(EVRT_E_INVALID, "focus distance must be finite and > 0");
        c->pending.lens_radius = aperture_radius;
        c->pending.focus_dist = focus_distance;
        scene_changed(c);
    });
}

int evrt_scene_reset(evrt_ctx *c)
{
    return guarded(c, [&] {
        need_ctx(c);
        c->pending = SceneDesc();
    });
}

// Everything but the material values equal: meshes (with their triangle
// materials), instances, camera and point lights.
static bool same_geometry(const SceneDesc &a, const SceneDesc &b)
{
    if (a.meshes.size() != b.meshes.size() || a.instances.size() != b.instances.size()) return false;
    for (size_t i = 0; i < a.meshes.size(); ++i) {
        const MeshDesc &x = a.meshes[i], &y = b.meshes[i];
        if (x.set != y.set || x.xyz != y.xyz || x.idx != y.idx || x.mat != y.mat) return false;
    }
    for (size_t i = 0; i < a.instances.size(); ++i) {
        const InstanceDesc &x = a.instances[i], &y = b.instances[i];
        if (x.set != y.set || x.mesh != y.mesh || x.kt != y.kt || x.kx != y.kx) return false;
    }
    const CameraDesc &x = a.cam, &y = b.cam;
    if (x.set != y.set || x.width != y.width || x.height != y.height || x.vfov != y.vfov || x.kt != y.kt ||
        x.elu != y.elu)
        return false;
    // The lens radius enters the box padding.
    return a.pl_pos == b.pl_pos && a.pl_int == b.pl_int && a.pl_int3 == b.pl_int3 && a.lens_radius == b.lens_radius;
}

int evrt_scene_commit(evrt_ctx *c)
{
    return guarded(c, [&] {
        need_ctx(c);
        SceneDesc &p = c->pending;
        if (p.albedo.empty()) fail(EVRT_E_STATE, "materials not set");
        if (!p.rgb && !p.pl_int3.empty()) fail(EVRT_E_INVALID, "RGB point lights need RGB materials");
        if (!p.cam.set) fail(EVRT_E_STATE, "camera not set");
        for (size_t i = 0; i < p.meshes.size(); ++i)
            if (!p.meshes[i].set) fail(EVRT_E_INVALID, "mesh ids are not dense: mesh " + std::to_string(i) + " missing");
        uint64_t nt = 0;
        for (size_t i = 0; i < p.instances.size(); ++i) {
            const InstanceDesc &in = p.instances[i];
            if (!in.set) fail(EVRT_E_INVALID, "instance ids are not dense: instance " + std::to_string(i) + " missing");
            if (in.mesh >= p.meshes.size()) fail(EVRT_E_INVALID, "instance refers to a missing mesh");
            nt += p.meshes[in.mesh].mat.size();
        }
        if (nt >= (1ull << 28)) fail(EVRT_E_UNSUPPORTED, "more than 2^28 world triangles");
        for (const auto &m : p.meshes)
            for (uint32_t mt : m.mat)
                if (mt >= p.albedo.size()) fail(EVRT_E_INVALID, "triangle material out of range");
        // Only albedo and emission changed: geometry, BVHs and box padding
        // stay valid, so the cached instants are kept and only their emitter
        // tables are rebuilt (a material update of an optimization loop).
        // (c->scene is the last committed scene; a commit needs a camera.)
        const bool materials_only = c->scene.cam.set && !c->host_only && c->scene.albedo.size() == p.albedo.size() &&
                                    same_geometry(c->scene, p);
        c->scene = p;
        c->static_geom = scene_static(p);
        if (!materials_only) {
            c->cache.clear();
            c->cache_order.clear();
        }
        ++c->scene_version;
        if (!c->host_only) {
            hip_check(hipSetDevice(c->device), "hipSetDevice");
            std::vector<float2> mats(p.albedo.size());
            for (size_t i = 0; i < mats.size(); ++i) mats[i] = make_float2(p.albedo[i], p.emission[i]);
            c->mat.upload(mats.data(), mats.size() * sizeof(float2), nullptr);
            std::vector<float4> pl(p.pl_int.size() ? p.pl_int.size() : 1, make_float4(0, 0, 0, 0));
            for (size_t i = 0; i < p.pl_int.size(); ++i)
                pl[i] = make_float4(p.pl_pos[3 * i], p.pl_pos[3 * i + 1], p.pl_pos[3 * i + 2], p.pl_int[i]);
            c->plights.upload(pl.data(), pl.size() * sizeof(float4), nullptr);
            if (p.rgb) {
                // (albedo rgb, 0), (emission rgb, its luminance) per material;
                // (intensity rgb, 0) per point light (grey lights: the
                // intensity in every channel).
                std::vector<float4> mr(2 * p.albedo.size());
                for (size_t i = 0; i < p.albedo.size(); ++i) {
                    const float *a = &p.albedo3[3 * i], *e = &p.emission3[3 * i];
                    mr[2 * i] = make_float4(a[0], a[1], a[2], 0.0f);
                    mr[2 * i + 1] = make_float4(e[0], e[1], e[2], p.emission[i]);
                }
                c->mat_rgb.upload(mr.data(), mr.size() * sizeof(float4), nullptr);
                std::vector<float4> plr(pl.size(), make_float4(0, 0, 0, 0));
                for (size_t i = 0; i < p.pl_int.size(); ++i)
                    plr[i] = p.pl_int3.empty() ? make_float4(p.pl_int[i], p.pl_int[i], p.pl_int[i], 0.0f)
                                               : make_float4(p.pl_int3[3 * i], p.pl_int3[3 * i + 1],
                                                             p.pl_int3[3 * i + 2], 0.0f);
                c->plights_rgb.upload(plr.data(), plr.size() * sizeof(float4), nullptr);
            }
            if (p.env_res) c->env.upload(p.env.data(), p.env.size() * sizeof(float), nullptr);
            hip_check(hipStreamSynchronize(nullptr), "scene upload");
            if (materials_only) refresh_emitters(c);
        }
        c->materials_only_commits += materials_only ? 1u : 0u;
        c->committed = true;
    });
}

void evrt_default_opts(evrt_render_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->seed = 0;
    o->max_depth = 4;
    o->rr_start_depth = 2;
    o->minibatch = 4;
    o->log_eps = 1e-4;
    o->nee = 1;
    o->jitter = 1;
    o->mode = EVRT_MODE_ADAPTIVE_1T;
    o->df_mode = EVRT_DF_STUDENT;
    o->ref_mode = EVRT_REF_LOCKSTEP;
}

static void validate_frame_args(const evrt_render_opts &o, float C, float alpha, uint32_t spp_init,
                                uint32_t spp_batch, uint32_t spp_max, const evrt_frame_out *out)
{
    if (!out || !out->polarity || !out->n_paths || !out->mean || !out->var)
        fail(EVRT_E_INVALID, "polarity, n_paths, mean and var outputs are required");
    if (!std::isfinite(C) || C < 0.0f) fail(EVRT_E_INVALID, "C must be finite and >= 0");
    if (!(alpha > 0.0f && alpha < 1.0f)) fail(EVRT_E_INVALID, "alpha must be in (0, 1)");
    const uint32_t mb = o.minibatch;
    if (spp_init % mb || spp_batch % mb || spp_max % mb)
        fail(EVRT_E_INVALID, "spp_init, spp_batch and spp_max must be multiples of minibatch");
    if (spp_init < 2 * mb) fail(EVRT_E_INVALID, "spp_init must hold at least two mini-batches");
    if (spp_init > spp_max) fail(EVRT_E_INVALID, "spp_init must not exceed spp_max");
    if (spp_batch == 0 && spp_init < spp_max && o.mode != EVRT_MODE_FIXED)
        fail(EVRT_E_INVALID, "spp_batch must be positive");
    if (spp_max > (1u << 24)) fail(EVRT_E_UNSUPPORTED, "spp_max above 2^24");
}

int evrt_render_event_frame(evrt_ctx *c, double t0, double t1, float C, float alpha, uint32_t spp_init,
                            uint32_t spp_batch, uint32_t spp_max, const evrt_render_opts *opts,
                            const evrt_frame_out *out, void *stream)
{
    return guarded(c, [&] {
        need_ctx(c);
        evrt_render_opts o;
        if (opts) o = *opts;
        else evrt_default_opts(&o);
        validate_opts(o);
        if (!c->committed) fail(EVRT_E_STATE, "scene not committed");
        if (!std::isfinite(t0) || !std::isfinite(t1)) fail(EVRT_E_INVALID, "t0 and t1 must be finite");
        validate_frame_args(o, C, alpha, spp_init, spp_batch, spp_max, out);
        need_device(c);
        render_frame(c, t0, t1, C, alpha, spp_init, spp_batch, spp_max, o, *out,
                     static_cast<hipStream_t>(stream));
    });
}

int evrt_render_event_video(evrt_ctx *c, uint32_t n_frames, const double *times, float C, float alpha,
                            uint32_t spp_init, uint32_t spp_batch, uint32_t spp_max, const evrt_render_opts *opts,
                            const evrt_frame_out *out, void *stream)
{
    return guarded(c, [&] {
        need_ctx(c);
        evrt_render_opts o;
        if (opts) o = *opts;
        else evrt_default_opts(&o);
        validate_opts(o);
        if (!c->committed) fail(EVRT_E_STATE, "scene not committed");
        if (n_frames < 2) fail(EVRT_E_INVALID, "n_frames must be at least 2");
        if ((uint64_t)o.key_base + n_frames > (1u << 24)) fail(EVRT_E_INVALID, "key_base + n_frames above 2^24");
        if (!times) fail(EVRT_E_INVALID, "NULL times");
        for (uint32_t k = 0; k < n_frames; ++k)
            if (!std::isfinite(times[k])) fail(EVRT_E_INVALID, "times must be finite");
        validate_frame_args(o, C, alpha, spp_init, spp_batch, spp_max, out);
        need_device(c);
        render_video(c, n_frames, times, C, alpha, spp_init, spp_batch, spp_max, o, *out,
                     static_cast<hipStream_t>(stream));
    });
}

int evrt_render_event_batch(evrt_ctx *c, uint32_t n_pairs, const double *times, float C, float alpha,
                            uint32_t spp_init, uint32_t spp_batch, uint32_t spp_max, const evrt_render_opts *opts,
                            const evrt_frame_out *out, void *stream)
{
    return guarded(c, [&] {
        need_ctx(c);
        evrt_render_opts o;
        if (opts) o = *opts;
        else evrt_default_opts(&o);
        validate_opts(o);
        if (!c->committed) fail(EVRT_E_STATE, "scene not committed");
        if (n_pairs == 0) fail(EVRT_E_INVALID, "n_pairs must be positive");
        // Counts first: times[] is only read once n_pairs is known to be sane.
        if (n_pairs + 1ull > kMaxBatchFrames) fail(EVRT_E_UNSUPPORTED, "more than 2047 pairs in one batch");
        if ((uint64_t)o.key_base + n_pairs > (1u << 24)) fail(EVRT_E_INVALID, "key_base + n_pairs above 2^24");
        if (!times) fail(EVRT_E_INVALID, "NULL times");
        for (uint32_t k = 0; k < n_pairs + 1; ++k)
            if (!std::isfinite(times[k])) fail(EVRT_E_INVALID, "times must be finite");
        validate_frame_args(o, C, alpha, spp_init, spp_batch, spp_max, out);
        if (o.ref_mode != EVRT_REF_LOCKSTEP) fail(EVRT_E_UNSUPPORTED, "frame batches sample in lock step only");
        if (o.normality_alpha > 0.0f) fail(EVRT_E_UNSUPPORTED, "frame batches do not run the normality pre-test");
        const uint64_t npx = (uint64_t)c->scene.cam.width * c->scene.cam.height;
        if (npx > kPixMask + 1ull) fail(EVRT_E_UNSUPPORTED, "more than 2^21 pixels per frame in a batch");
        if ((n_pairs + 1ull) * npx >= (1ull << 31)) fail(EVRT_E_UNSUPPORTED, "more than 2^31 (frame, pixel) items");
        need_device(c);
        render_batch(c, n_pairs, times, C, alpha, spp_init, spp_batch, spp_max, o, *out,
                     static_cast<hipStream_t>(stream));
    });
}

int evrt_get_frame_stats(const evrt_ctx *c, evrt_frame_stats *out)
{
    if (!c || !out) return EVRT_E_INVALID;
    *out = c->stats;
    return EVRT_OK;
}

int evrt_trace_rays(evrt_ctx *c, double t, uint32_t n, const float *rays, const uint32_t *skip, int any_hit,
                    float *t_out, uint32_t *prim_out, void *stream)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (!c->committed) fail(EVRT_E_STATE, "scene not committed");
        if (!std::isfinite(t)) fail(EVRT_E_INVALID, "t must be finite");
        if (n == 0) return;
        if (n >= (1u << 31)) fail(EVRT_E_INVALID, "too many rays");
        if (!rays || !prim_out || (!any_hit && !t_out)) fail(EVRT_E_INVALID, "NULL ray or output array");
        need_device(c);
        trace_rays(c, t, n, rays, skip, any_hit, t_out, prim_out, static_cast<hipStream_t>(stream));
    });
}

static_assert(EVRT_NOALLOC_MAX_RAYS == kNoAllocRays, "header and library disagree on the no-alloc limit");

int evrt_trace_rays_noalloc(evrt_ctx *c, double t, uint32_t n, const float *rays, const uint32_t *skip,
                            int any_hit, float *t_out, uint32_t *prim_out, void *stream)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (!c->committed) fail(EVRT_E_STATE, "scene not committed");
        if (!std::isfinite(t)) fail(EVRT_E_INVALID, "t must be finite");
        if (n == 0) return;
        if (n > EVRT_NOALLOC_MAX_RAYS)
            fail(EVRT_E_INVALID, "n = " + std::to_string(n) + " rays is above the no-alloc maximum of " +
                                     std::to_string(EVRT_NOALLOC_MAX_RAYS));
        if (!rays || !prim_out || (!any_hit && !t_out)) fail(EVRT_E_INVALID, "NULL ray or output array");
        need_device(c);
        trace_rays_noalloc(c, t, n, rays, skip, any_hit, t_out, prim_out, static_cast<hipStream_t>(stream));
    });
}

int evrt_render_paths(evrt_ctx *c, double t0, double t1, uint32_t n_pixels, const uint32_t *pixels,
                      uint32_t spp, const evrt_render_opts *opts, float *L_out, void *stream)
{
    return guarded(c, [&] {
        need_ctx(c);
        evrt_render_opts o;
        if (opts) o = *opts;
        else evrt_default_opts(&o);
        validate_opts(o);
        if (!c->committed) fail(EVRT_E_STATE, "scene not committed");
        if (!std::isfinite(t0) || !std::isfinite(t1)) fail(EVRT_E_INVALID, "t0 and t1 must be finite");
        if (n_pixels == 0 || spp == 0) return;
        if (!pixels || !L_out) fail(EVRT_E_INVALID, "NULL pixel or output array");
        if (spp > (1u << 24)) fail(EVRT_E_UNSUPPORTED, "spp above 2^24");
        need_device(c);
        render_paths(c, t0, t1, n_pixels, pixels, spp, o, L_out, static_cast<hipStream_t>(stream));
    });
}

int evrt_event_loss_grad(evrt_ctx *c, double t0, double t1, float C, float tau, uint32_t spp,
                         const evrt_render_opts *opts, const evrt_diff_out *out, void *stream)
{
    return guarded(c, [&] {
        need_ctx(c);
        evrt_render_opts o;
        if (opts) o = *opts;
        else evrt_default_opts(&o);
        validate_opts(o);
        if (!c->committed) fail(EVRT_E_STATE, "scene not committed");
        if (!std::isfinite(t0) || !std::isfinite(t1)) fail(EVRT_E_INVALID, "t0 and t1 must be finite");
        if (!std::isfinite(C) || C < 0.0f) fail(EVRT_E_INVALID, "C must be finite and >= 0");
        if (!std::isfinite(tau) || !(tau > 0.0f)) fail(EVRT_E_INVALID, "tau must be finite and > 0");
        if (spp == 0 || spp % o.minibatch != 0) fail(EVRT_E_INVALID, "spp must be a positive multiple of minibatch");
        if (!out || !out->loss || !out->grad) fail(EVRT_E_INVALID, "NULL loss or gradient output");
        if (o.mis) fail(EVRT_E_UNSUPPORTED, "the gradient follows the estimator without MIS");
        if (c->scene.rgb) fail(EVRT_E_UNSUPPORTED, "the gradient follows grey radiance");
        if (c->scene.albedo.size() > 2048) fail(EVRT_E_UNSUPPORTED, "more than 2048 materials");
        const uint64_t npx = (uint64_t)c->scene.cam.width * c->scene.cam.height;
        if (2ull * npx * spp >= (1ull << 31)) fail(EVRT_E_UNSUPPORTED, "more than 2^31 paths");
        need_device(c);
        event_loss_grad(c, t0, t1, C, tau, spp, o, *out, static_cast<hipStream_t>(stream));
    });
}

int evrt_delta_vjp(evrt_ctx *c, double t0, double t1, uint32_t spp, const evrt_render_opts *opts,
                   const double *grad_delta, const evrt_diff_out *out, void *stream)
{
    return guarded(c, [&] {
        need_ctx(c);
        evrt_render_opts o;
        if (opts) o = *opts;
        else evrt_default_opts(&o);
        validate_opts(o);
        if (!c->committed) fail(EVRT_E_STATE, "scene not committed");
        if (!std::isfinite(t0) || !std::isfinite(t1)) fail(EVRT_E_INVALID, "t0 and t1 must be finite");
        if (spp == 0 || spp % o.minibatch != 0) fail(EVRT_E_INVALID, "spp must be a positive multiple of minibatch");
        if (!out) fail(EVRT_E_INVALID, "NULL output");
        if (grad_delta && (!out->loss || !out->grad)) fail(EVRT_E_INVALID, "NULL value or gradient output");
        if (!grad_delta && !out->delta) fail(EVRT_E_INVALID, "NULL delta output (grad_delta NULL computes Delta only)");
        if (o.mis) fail(EVRT_E_UNSUPPORTED, "the gradient follows the estimator without MIS");
        if (c->scene.rgb) fail(EVRT_E_UNSUPPORTED, "the gradient follows grey radiance");
        if (c->scene.albedo.size() > 2048) fail(EVRT_E_UNSUPPORTED, "more than 2048 materials");
        const uint64_t npx = (uint64_t)c->scene.cam.width * c->scene.cam.height;
        if (2ull * npx * spp >= (1ull << 31)) fail(EVRT_E_UNSUPPORTED, "more than 2^31 paths");
        need_device(c);
        evrt_diff_out d = *out;
        if (!grad_delta) {
            d.loss = nullptr;
            d.grad = nullptr;
            d.loss_px = nullptr;
            d.replay_mismatch = nullptr;
        }
        event_loss_grad(c, t0, t1, 0.0f, 1.0f, spp, o, d, static_cast<hipStream_t>(stream), grad_delta,
                        grad_delta == nullptr);
    });
}

int evrt_decide_stats(evrt_ctx *c, const double *x0, const double *x1, uint32_t n_pixels, uint32_t m, float C,
                      float alpha, uint8_t mode, uint8_t df_mode, double *t_out, uint8_t *stop_out,
                      int8_t *polarity_out, double *p_out, void *stream)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (m < 2) fail(EVRT_E_INVALID, "m must be >= 2");
        if (!std::isfinite(C) || C < 0.0f) fail(EVRT_E_INVALID, "C must be finite and >= 0");
        if (!(alpha > 0.0f && alpha < 1.0f)) fail(EVRT_E_INVALID, "alpha must be in (0, 1)");
        if (mode > EVRT_MODE_MEAN_ONLY) fail(EVRT_E_INVALID, "unknown mode");
        if (df_mode > EVRT_DF_WELCH) fail(EVRT_E_INVALID, "unknown df_mode");
        if (n_pixels == 0) return;
        if (!x0 || !x1 || !t_out || !stop_out || !polarity_out) fail(EVRT_E_INVALID, "NULL array");
        need_device(c);
        decide_stats(c, x0, x1, n_pixels, m, C, alpha, mode, df_mode, t_out, stop_out, polarity_out, p_out,
                     static_cast<hipStream_t>(stream));
    });
}

int evrt_scene_info_at(evrt_ctx *c, double t, evrt_scene_info *out)
{
    return guarded(c, [&] {
        need_ctx(c);
        if (!out) fail(EVRT_E_INVALID, "out is NULL");
        if (!c->committed) fail(EVRT_E_STATE, "scene not committed");
        if (!std::isfinite(t)) fail(EVRT_E_INVALID, "t must be finite");
        HostInstant h;
        build_world(c->scene, t, h);
        const float pad = bvh_padding(c->scene, h, h);
        build_bvh(h, (uint32_t)lds_treelet_nodes(), pad);
        std::memset(out, 0, sizeof(*out));
        out->n_tri = (uint32_t)(h.tri.size() / 9);
        out->n_nodes = (uint32_t)(h.nodes.size() / 8);
        out->n_lds = h.n_lds;
        out->depth = h.depth;
        out->n_emit = (uint32_t)h.emit_prim.size();
        out->box_pad = pad;
        out->sah_cost = h.sah_cost;
        const std::string msg = check_bvh(h, pad);
        if (!msg.empty()) fail(EVRT_E_INVALID, "BVH check failed: " + msg);
    });
}

double evrt_t_quantile(double p, uint32_t df) { return t_quantile(p, df); }

}  // extern "C"
#pragma GCC visibility pop
