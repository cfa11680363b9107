"""MI355X (gfx950) adaptive event-camera path tracer: Python binding.

A thin ctypes layer over ``libevrt.so`` (declared in ``include/evrt.h``):
argument marshalling only.  Every step of rendering runs in the library's
HIP kernels; PyTorch provides device memory and the current stream.  There
is no CPU fallback: without the built library (or without a GPU for the
render calls) the calls raise.

Implements "Monte Carlo Path Tracing and Statistical Event Detection for
Event Camera Simulation" (arXiv 2408.07996): per-pixel path tracing at two
instants, mini-batch log-luminance statistics (Eq. 3-4), the one-tailed
t-test of Eq. 7 that stops sampling once "no event" is significant, and the
event rule of Algorithm 1.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

__all__ = ["Renderer", "EvrtError", "default_opts", "load_library", "MODE_ADAPTIVE_1T", "MODE_FIXED",
           "MODE_ADAPTIVE_2T", "MODE_MEAN_ONLY", "DF_STUDENT", "DF_WELCH", "REF_LOCKSTEP", "REF_FULL",
           "event_loss", "log_luminance_delta"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# EVRT_LIBRARY may point at another build of the same library (tuning runs).
LIB_PATH = os.environ.get("EVRT_LIBRARY") or os.path.join(_HERE, "libevrt.so")

EVRT_OK, EVRT_E_INVALID, EVRT_E_NOMEM, EVRT_E_DEVICE, EVRT_E_STATE, EVRT_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
MODE_ADAPTIVE_1T, MODE_FIXED, MODE_ADAPTIVE_2T, MODE_MEAN_ONLY = 0, 1, 2, 3
DF_STUDENT, DF_WELCH = 0, 1
REF_LOCKSTEP, REF_FULL = 0, 1
NO_PRIM = 0xFFFFFFFF

_c_p = ctypes.c_void_p
_u32 = ctypes.c_uint32


class RenderOpts(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64), ("max_depth", _u32), ("rr_start_depth", _u32), ("minibatch", _u32),
        ("log_eps", ctypes.c_double), ("nee", ctypes.c_uint8), ("jitter", ctypes.c_uint8),
        ("mode", ctypes.c_uint8), ("df_mode", ctypes.c_uint8), ("ref_mode", ctypes.c_uint8),
        ("profile", ctypes.c_uint8), ("count_work", ctypes.c_uint8), ("lds_nodes", ctypes.c_uint8),
        ("mis", ctypes.c_uint8), ("ray_batch", _u32), ("key_base", _u32), ("trace_blocks_per_cu", _u32),
        ("replay_retrace", _u32), ("normality_alpha", ctypes.c_float),
    ]


class FrameOut(ctypes.Structure):
    _fields_ = [("polarity", _c_p), ("n_paths", _c_p), ("mean", _c_p), ("var", _c_p),
                ("t_last", _c_p), ("mean_radiance", _c_p), ("flags", _c_p)]


class FrameStats(ctypes.Structure):
    _fields_ = [
        ("camera_rays", ctypes.c_uint64), ("extension_rays", ctypes.c_uint64),
        ("shadow_rays", ctypes.c_uint64), ("node_visits", ctypes.c_uint64),
        ("tri_tests", ctypes.c_uint64), ("node_visits_shadow", ctypes.c_uint64),
        ("tri_tests_shadow", ctypes.c_uint64), ("paths", ctypes.c_uint64), ("rounds", _u32),
        ("pieces", _u32), ("n_closest_launches", _u32), ("n_shadow_launches", _u32),
        ("ms_wall", ctypes.c_double), ("ms_closest", ctypes.c_double), ("ms_shadow", ctypes.c_double),
        ("ms_build", ctypes.c_double), ("active_after_round", _u32 * 64),
    ]


class SceneInfo(ctypes.Structure):
    _fields_ = [("n_tri", _u32), ("n_nodes", _u32), ("n_lds", _u32), ("depth", _u32), ("n_emit", _u32),
                ("box_pad", ctypes.c_float), ("sah_cost", ctypes.c_double)]


class DiffOut(ctypes.Structure):
    _fields_ = [("loss", _c_p), ("grad", _c_p), ("loss_px", _c_p), ("delta", _c_p),
                ("replay_mismatch", _c_p)]


class EvrtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"evrt error {code}: {msg}")
        self.code = code


_lib = None

# (name, restype, argtypes) of every entry point in include/evrt.h
SIGNATURES = [
    ("evrt_abi_version", ctypes.c_int, []),
    ("evrt_create", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_c_p)]),
    ("evrt_destroy", None, [_c_p]),
    ("evrt_last_error", ctypes.c_char_p, [_c_p]),
    ("evrt_scene_set_materials", ctypes.c_int, [_c_p, _c_p, _c_p, _u32]),
    ("evrt_scene_set_materials_rgb", ctypes.c_int, [_c_p, _c_p, _c_p, _u32]),
    ("evrt_scene_set_mesh", ctypes.c_int, [_c_p, _u32, _c_p, _u32, _c_p, _c_p, _u32]),
    ("evrt_scene_set_instance", ctypes.c_int, [_c_p, _u32, _u32, _u32, _c_p, _c_p]),
    ("evrt_scene_set_point_lights", ctypes.c_int, [_c_p, _c_p, _c_p, _u32]),
    ("evrt_scene_set_point_lights_rgb", ctypes.c_int, [_c_p, _c_p, _c_p, _u32]),
    ("evrt_scene_set_camera", ctypes.c_int, [_c_p, _u32, _u32, ctypes.c_double, _u32, _c_p, _c_p]),
    ("evrt_scene_set_environment", ctypes.c_int, [_c_p, _c_p, _u32]),
    ("evrt_scene_set_lens", ctypes.c_int, [_c_p, ctypes.c_float, ctypes.c_float]),
    ("evrt_scene_reset", ctypes.c_int, [_c_p]),
    ("evrt_scene_commit", ctypes.c_int, [_c_p]),
    ("evrt_default_opts", None, [ctypes.POINTER(RenderOpts)]),
    ("evrt_render_event_frame", ctypes.c_int,
     [_c_p, ctypes.c_double, ctypes.c_double, ctypes.c_float, ctypes.c_float, _u32, _u32, _u32,
      ctypes.POINTER(RenderOpts), ctypes.POINTER(FrameOut), _c_p]),
    ("evrt_render_event_video", ctypes.c_int,
     [_c_p, _u32, _c_p, ctypes.c_float, ctypes.c_float, _u32, _u32, _u32, ctypes.POINTER(RenderOpts),
      ctypes.POINTER(FrameOut), _c_p]),
    ("evrt_render_event_batch", ctypes.c_int,
     [_c_p, _u32, _c_p, ctypes.c_float, ctypes.c_float, _u32, _u32, _u32, ctypes.POINTER(RenderOpts),
      ctypes.POINTER(FrameOut), _c_p]),
    ("evrt_get_frame_stats", ctypes.c_int, [_c_p, ctypes.POINTER(FrameStats)]),
    ("evrt_trace_rays", ctypes.c_int, [_c_p, ctypes.c_double, _u32, _c_p, _c_p, ctypes.c_int, _c_p, _c_p, _c_p]),
    ("evrt_trace_rays_noalloc", ctypes.c_int,
     [_c_p, ctypes.c_double, _u32, _c_p, _c_p, ctypes.c_int, _c_p, _c_p, _c_p]),
    ("evrt_render_paths", ctypes.c_int,
     [_c_p, ctypes.c_double, ctypes.c_double, _u32, _c_p, _u32, ctypes.POINTER(RenderOpts), _c_p, _c_p]),
    ("evrt_decide_stats", ctypes.c_int,
     [_c_p, _c_p, _c_p, _u32, _u32, ctypes.c_float, ctypes.c_float, ctypes.c_uint8, ctypes.c_uint8, _c_p, _c_p,
      _c_p, _c_p, _c_p]),
    ("evrt_event_loss_grad", ctypes.c_int,
     [_c_p, ctypes.c_double, ctypes.c_double, ctypes.c_float, ctypes.c_float, _u32, ctypes.POINTER(RenderOpts),
      ctypes.POINTER(DiffOut), _c_p]),
    ("evrt_delta_vjp", ctypes.c_int,
     [_c_p, ctypes.c_double, ctypes.c_double, _u32, ctypes.POINTER(RenderOpts), _c_p, ctypes.POINTER(DiffOut), _c_p]),
    ("evrt_scene_info_at", ctypes.c_int, [_c_p, ctypes.c_double, ctypes.POINTER(SceneInfo)]),
    ("evrt_t_quantile", ctypes.c_double, [ctypes.c_double, _u32]),
]


def load_library():
    """Load libevrt.so, building it with hipcc only when it does not exist."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build
        _build.build()
    # torch brings its own HIP and HSA runtimes; loading them before the
    # library makes the library bind to the same ones (a second copy of the
    # runtime in the process does not see the device).
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def default_opts(**kw) -> RenderOpts:
    o = RenderOpts()
    load_library().evrt_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(f"unknown render option {k!r}")
        setattr(o, k, v)
    return o


def t_quantile(p: float, df: int) -> float:
    return float(load_library().evrt_t_quantile(float(p), int(df)))


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(_c_p) if a.size else None


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t) -> Optional[int]:
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Renderer:
    """One library context on one GPU (``device=-1``: host only, for
    argument validation without a GPU)."""

    def __init__(self, device: int = 0):
        L = load_library()
        if device >= 0:
            # Outputs are torch tensors: bring up torch's device runtime before
            # the library's, which it does not detect when it starts second.
            import torch
            if not torch.cuda.is_available():
                raise EvrtError(EVRT_E_DEVICE, "no visible GPU")
        h = _c_p()
        rc = L.evrt_create(int(device), ctypes.byref(h))
        if rc != EVRT_OK:
            raise EvrtError(rc, L.evrt_last_error(None).decode())
        self._h = h
        self.device = device
        self.scene = None

    def close(self) -> None:
        if getattr(self, "_h", None):
            load_library().evrt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc: int) -> None:
        if rc != EVRT_OK:
            raise EvrtError(rc, load_library().evrt_last_error(self._h).decode())

    # -- scene -----------------------------------------------------------
    def scene_set_materials(self, albedo, emission) -> None:
        a = np.ascontiguousarray(albedo, np.float32)
        e = np.ascontiguousarray(emission, np.float32)
        self._check(load_library().evrt_scene_set_materials(self._h, _np_ptr(a), _np_ptr(e), len(a)))

    def scene_set_materials_rgb(self, albedo_rgb, emission_rgb) -> None:
        a = np.ascontiguousarray(albedo_rgb, np.float32).reshape(-1, 3)
        e = np.ascontiguousarray(emission_rgb, np.float32).reshape(-1, 3)
        if len(a) != len(e):
            raise ValueError("albedo_rgb and emission_rgb differ in length")
        self._check(load_library().evrt_scene_set_materials_rgb(self._h, _np_ptr(a), _np_ptr(e), len(a)))

    def scene_set_mesh(self, mesh_id: int, xyz, tri_idx, tri_mat) -> None:
        v = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
        t = np.ascontiguousarray(tri_idx, np.uint32).reshape(-1, 3)
        m = np.ascontiguousarray(tri_mat, np.uint32).reshape(-1)
        self._check(load_library().evrt_scene_set_mesh(self._h, int(mesh_id), _np_ptr(v), len(v), _np_ptr(t),
                                                       _np_ptr(m), len(t)))

    def scene_set_instance(self, inst_id: int, mesh_id: int, key_t, xform3x4) -> None:
        kt = np.ascontiguousarray(key_t, np.float64).reshape(-1)
        kx = np.ascontiguousarray(xform3x4, np.float64).reshape(-1, 12)
        self._check(load_library().evrt_scene_set_instance(self._h, int(inst_id), int(mesh_id), len(kt),
                                                           _np_ptr(kt), _np_ptr(kx)))

    def scene_set_point_lights(self, pos_xyz, intensity) -> None:
        p = np.ascontiguousarray(pos_xyz, np.float32).reshape(-1, 3)
        i = np.ascontiguousarray(intensity, np.float32).reshape(-1)
        self._check(load_library().evrt_scene_set_point_lights(self._h, _np_ptr(p), _np_ptr(i), len(i)))

    def scene_set_point_lights_rgb(self, pos_xyz, intensity_rgb) -> None:
        p = np.ascontiguousarray(pos_xyz, np.float32).reshape(-1, 3)
        i = np.ascontiguousarray(intensity_rgb, np.float32).reshape(-1, 3)
        if len(p) != len(i):
            raise ValueError("positions and intensities differ in length")
        self._check(load_library().evrt_scene_set_point_lights_rgb(self._h, _np_ptr(p), _np_ptr(i), len(i)))

    def scene_set_camera(self, width: int, height: int, vfov_deg: float, key_t, eye_look_up) -> None:
        kt = np.ascontiguousarray(key_t, np.float64).reshape(-1)
        e = np.ascontiguousarray(eye_look_up, np.float64).reshape(-1, 9)
        self._check(load_library().evrt_scene_set_camera(self._h, int(width), int(height), float(vfov_deg),
                                                         len(kt), _np_ptr(kt), _np_ptr(e)))

    def scene_reset(self) -> None:
        self._check(load_library().evrt_scene_reset(self._h))

    def scene_commit(self) -> None:
        self._check(load_library().evrt_scene_commit(self._h))

    def set_scene(self, sc) -> None:
        """Uploads a ``scenes.Scene`` (flat arrays) mesh by mesh and commits."""
        self.scene_reset()
        if getattr(sc, "albedo_rgb", None) is not None:
            self.scene_set_materials_rgb(sc.albedo_rgb, sc.emission_rgb)
        else:
            self.scene_set_materials(sc.albedo, sc.emission)
        off = sc.mesh_tri_off.astype(np.int64)
        for m in range(len(off) - 1):
            tri = sc.tri_idx[off[m]:off[m + 1]].astype(np.int64)
            if len(tri):
                v0, v1 = int(tri.min()), int(tri.max()) + 1
                self.scene_set_mesh(m, sc.xyz[v0:v1], tri - v0, sc.tri_mat[off[m]:off[m + 1]])
            else:
                self.scene_set_mesh(m, np.zeros((0, 3), np.float32), np.zeros((0, 3), np.uint32),
                                    np.zeros(0, np.uint32))
        koff = sc.inst_key_off.astype(np.int64)
        for i in range(len(sc.inst_mesh)):
            self.scene_set_instance(i, int(sc.inst_mesh[i]), sc.key_t[koff[i]:koff[i + 1]],
                                    sc.key_xform[koff[i]:koff[i + 1]])
        if getattr(sc, "pl_rgb", None) is not None:
            self.scene_set_point_lights_rgb(sc.pl_pos, sc.pl_rgb)
        else:
            self.scene_set_point_lights(sc.pl_pos, sc.pl_intensity)
        self.scene_set_camera(sc.width, sc.height, sc.vfov_deg, sc.cam_t, sc.cam_elu)
        env = getattr(sc, "env", None)
        if env is not None:
            e = np.ascontiguousarray(env, np.float32)
            self._check(load_library().evrt_scene_set_environment(self._h, _np_ptr(e), int(e.shape[-1])))
        else:
            self._check(load_library().evrt_scene_set_environment(self._h, None, 0))
        self._check(load_library().evrt_scene_set_lens(self._h, float(getattr(sc, "lens_radius", 0.0)),
                                                       float(getattr(sc, "focus_dist", 1.0))))
        self.scene_commit()
        self.scene = sc

    def set_materials(self, albedo, emission) -> None:
        """Replaces the materials of the committed scene and commits again
        (geometry is kept; instants are rebuilt on next use)."""
        self.scene_set_materials(albedo, emission)
        self.scene_commit()
        if getattr(self, "scene", None) is not None:
            import dataclasses
            self.scene = dataclasses.replace(self.scene, albedo=np.asarray(albedo, np.float32).copy(),
                                             emission=np.asarray(emission, np.float32).copy())

    def scene_info_at(self, t: float) -> Dict:
        """Host-side BVH build and structural check at time t."""
        info = SceneInfo()
        self._check(load_library().evrt_scene_info_at(self._h, float(t), ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in SceneInfo._fields_}

    # -- rendering ---------------------------------------------------------
    def _opts(self, opts) -> RenderOpts:
        if opts is None:
            return default_opts()
        if isinstance(opts, RenderOpts):
            return opts
        return default_opts(**opts)

    def render_event_frame(self, t0: float, t1: float, C: float, alpha: float, spp_init: int,
                           spp_batch: int, spp_max: int, opts=None, out: Optional[Dict] = None,
                           stream=None, extras: bool = True) -> Dict:
        """Renders one event frame; returns device tensors (see evrt.h)."""
        import torch
        o = self._opts(opts)
        if self.scene is None:
            raise EvrtError(EVRT_E_STATE, "no scene")
        npx = self.scene.width * self.scene.height
        dev = torch.device("cuda", self.device)
        if out is None:
            out = dict(
                polarity=torch.empty(npx, dtype=torch.int8, device=dev),
                n_paths=torch.empty(npx, dtype=torch.int32, device=dev),
                mean=torch.empty(npx, 2, dtype=torch.float64, device=dev),
                var=torch.empty(npx, 2, dtype=torch.float64, device=dev),
            )
            if extras:
                out["t_last"] = torch.empty(npx, dtype=torch.float64, device=dev)
                out["mean_radiance"] = torch.empty(npx, 2, dtype=torch.float64, device=dev)
                out["flags"] = torch.empty(npx, dtype=torch.uint8, device=dev)
        fo = FrameOut(_dptr(out["polarity"]), _dptr(out["n_paths"]), _dptr(out["mean"]), _dptr(out["var"]),
                      _dptr(out.get("t_last")), _dptr(out.get("mean_radiance")), _dptr(out.get("flags")))
        self._check(load_library().evrt_render_event_frame(
            self._h, float(t0), float(t1), float(C), float(alpha), int(spp_init), int(spp_batch),
            int(spp_max), ctypes.byref(o), ctypes.byref(fo), _stream_ptr(stream)))
        return out

    def render_event_video(self, times, C: float, alpha: float, spp_init: int, spp_batch: int, spp_max: int,
                           opts=None, stream=None, extras: bool = True) -> Dict:
        """Sequential event video over frames at `times` (reference carried
        per pixel, replaced at events); device tensors with a leading axis
        of len(times) - 1 frames (see evrt.h)."""
        return self._multi("evrt_render_event_video", times, len(times), C, alpha, spp_init, spp_batch, spp_max,
                           opts, stream, extras)

    def _multi(self, fn, times, n_arg, C, alpha, spp_init, spp_batch, spp_max, opts, stream, extras) -> Dict:
        import torch
        o = self._opts(opts)
        if self.scene is None:
            raise EvrtError(EVRT_E_STATE, "no scene")
        t = np.ascontiguousarray(times, np.float64).reshape(-1)
        n = len(t) - 1
        if n < 1:
            raise EvrtError(EVRT_E_INVALID, "need at least two times")
        npx = self.scene.width * self.scene.height
        dev = torch.device("cuda", self.device)
        out = dict(
            polarity=torch.empty(n, npx, dtype=torch.int8, device=dev),
            n_paths=torch.empty(n, npx, dtype=torch.int32, device=dev),
            mean=torch.empty(n, npx, 2, dtype=torch.float64, device=dev),
            var=torch.empty(n, npx, 2, dtype=torch.float64, device=dev),
        )
        if extras:
            out["t_last"] = torch.empty(n, npx, dtype=torch.float64, device=dev)
            out["mean_radiance"] = torch.empty(n, npx, 2, dtype=torch.float64, device=dev)
            out["flags"] = torch.empty(n, npx, dtype=torch.uint8, device=dev)
        fo = FrameOut(_dptr(out["polarity"]), _dptr(out["n_paths"]), _dptr(out["mean"]), _dptr(out["var"]),
                      _dptr(out.get("t_last")), _dptr(out.get("mean_radiance")), _dptr(out.get("flags")))
        self._check(getattr(load_library(), fn)(
            self._h, int(n_arg), _np_ptr(t), float(C), float(alpha), int(spp_init), int(spp_batch), int(spp_max),
            ctypes.byref(o), ctypes.byref(fo), _stream_ptr(stream)))
        return out

    def render_event_batch(self, times, C: float, alpha: float, spp_init: int, spp_batch: int, spp_max: int,
                           opts=None, stream=None, extras: bool = True) -> Dict:
        """Renders the consecutive pairs (times[k], times[k+1]) at once;
        returns device tensors with a leading pair axis (see evrt.h)."""
        return self._multi("evrt_render_event_batch", times, len(times) - 1, C, alpha, spp_init, spp_batch,
                           spp_max, opts, stream, extras)

    def frame_stats(self) -> Dict:
        s = FrameStats()
        self._check(load_library().evrt_get_frame_stats(self._h, ctypes.byref(s)))
        d = {k: getattr(s, k) for k, _ in FrameStats._fields_ if k != "active_after_round"}
        d["active_after_round"] = list(s.active_after_round)[: s.rounds]
        return d

    def render_paths(self, t0: float, t1: float, pixels, spp: int, opts=None, stream=None):
        """Per-path radiance [n_pixels, 2, spp] (float32 device tensor)."""
        import torch
        o = self._opts(opts)
        dev = torch.device("cuda", self.device)
        px = torch.as_tensor(np.ascontiguousarray(pixels, np.uint32).view(np.int32)).to(dev)
        L = torch.empty(len(px), 2, int(spp), dtype=torch.float32, device=dev)
        self._check(load_library().evrt_render_paths(self._h, float(t0), float(t1), len(px), _dptr(px), int(spp),
                                                     ctypes.byref(o), _dptr(L), _stream_ptr(stream)))
        return L

    def trace_rays(self, t: float, rays, skip=None, any_hit: bool = False, stream=None):
        """rays: float32 [n, 8] = (o, tmin, d, tmax).  Returns (t, prim) or
        the any-hit flags."""
        import torch
        dev = torch.device("cuda", self.device)
        r = torch.as_tensor(rays, dtype=torch.float32).to(dev).contiguous()
        n = r.shape[0]
        sk = None
        if skip is not None:
            sk = torch.as_tensor(np.ascontiguousarray(skip, np.uint32).view(np.int32)).to(dev)
        prim = torch.empty(n, dtype=torch.int32, device=dev)
        tt = None if any_hit else torch.empty(n, dtype=torch.float32, device=dev)
        self._check(load_library().evrt_trace_rays(self._h, float(t), n, _dptr(r), _dptr(sk), int(bool(any_hit)),
                                                   _dptr(tt), _dptr(prim), _stream_ptr(stream)))
        return prim if any_hit else (tt, prim)

    def trace_rays_noalloc(self, t: float, rays, skip, any_hit: bool, t_out, prim_out, stream=None) -> None:
        """evrt_trace_rays_noalloc on caller device tensors (rays float32
        [n, 8], skip uint32/int32 [n] or None, t_out float32 [n] (None with
        any_hit), prim_out int32 [n]): enqueues the query on the stream and
        returns; allocates nothing."""
        n = int(rays.shape[0])
        self._check(load_library().evrt_trace_rays_noalloc(
            self._h, float(t), n, _dptr(rays), _dptr(skip) if skip is not None else None, int(bool(any_hit)),
            _dptr(t_out) if t_out is not None else None, _dptr(prim_out), _stream_ptr(stream)))

    def event_loss_grad(self, t0: float, t1: float, C: float, tau: float, spp: int, opts=None,
                        per_pixel: bool = False, stream=None) -> Dict:
        """Smoothed event loss sum softplus((|Delta| - C) / tau) at spp paths
        per pixel and instant, and its path-replay gradient (float64 device
        tensors): loss [1], grad_albedo [n_mat], grad_emission [n_mat],
        replay_mismatch [1]; with per_pixel also loss_px and delta [H*W].
        The replay re-shades from the forward pass's ray log; opts
        replay_retrace=1 makes it trace its rays again."""
        import torch
        o = self._opts(opts)
        dev = torch.device("cuda", self.device)
        n_mat = len(self.scene.albedo)
        npx = self.scene.width * self.scene.height
        loss = torch.empty(1, dtype=torch.float64, device=dev)
        grad = torch.empty(2 * n_mat, dtype=torch.float64, device=dev)
        mism = torch.empty(1, dtype=torch.int32, device=dev)
        lpx = torch.empty(npx, dtype=torch.float64, device=dev) if per_pixel else None
        dpx = torch.empty(npx, dtype=torch.float64, device=dev) if per_pixel else None
        out = DiffOut(_dptr(loss), _dptr(grad), _dptr(lpx), _dptr(dpx), _dptr(mism))
        self._check(load_library().evrt_event_loss_grad(self._h, float(t0), float(t1), float(C), float(tau),
                                                        int(spp), ctypes.byref(o), ctypes.byref(out),
                                                        _stream_ptr(stream)))
        res = dict(loss=loss, grad_albedo=grad[:n_mat], grad_emission=grad[n_mat:], replay_mismatch=mism)
        if per_pixel:
            res.update(loss_px=lpx, delta=dpx)
        return res

    def delta_vjp(self, t0: float, t1: float, spp: int, grad_delta=None, opts=None, stream=None) -> Dict:
        """The per-pixel log-luminance difference Delta [H*W] at spp paths
        per pixel and instant and, with grad_delta (dL/dDelta per pixel, any
        float tensor or array of H*W values), value = sum g Delta and its
        path-replay gradient: grad_albedo, grad_emission [n_mat],
        replay_mismatch [1] (float64 device tensors).  Without grad_delta
        only Delta is computed (no replay)."""
        import torch
        o = self._opts(opts)
        dev = torch.device("cuda", self.device)
        n_mat = len(self.scene.albedo)
        npx = self.scene.width * self.scene.height
        delta = torch.empty(npx, dtype=torch.float64, device=dev)
        if grad_delta is None:
            out = DiffOut(None, None, None, _dptr(delta), None)
            self._check(load_library().evrt_delta_vjp(self._h, float(t0), float(t1), int(spp), ctypes.byref(o), None,
                                                      ctypes.byref(out), _stream_ptr(stream)))
            return dict(delta=delta)
        g = torch.as_tensor(grad_delta).to(device=dev, dtype=torch.float64).reshape(-1).contiguous()
        if g.numel() != npx:
            raise ValueError(f"grad_delta needs {npx} values, got {g.numel()}")
        val = torch.empty(1, dtype=torch.float64, device=dev)
        grad = torch.empty(2 * n_mat, dtype=torch.float64, device=dev)
        mism = torch.empty(1, dtype=torch.int32, device=dev)
        out = DiffOut(_dptr(val), _dptr(grad), None, _dptr(delta), _dptr(mism))
        self._check(load_library().evrt_delta_vjp(self._h, float(t0), float(t1), int(spp), ctypes.byref(o),
                                                  _dptr(g), ctypes.byref(out), _stream_ptr(stream)))
        return dict(value=val, delta=delta, grad_albedo=grad[:n_mat], grad_emission=grad[n_mat:],
                    replay_mismatch=mism)

    def decide_stats(self, x0, x1, C: float, alpha: float, mode: int = MODE_ADAPTIVE_1T,
                     df_mode: int = DF_STUDENT, want_p: bool = False, stream=None):
        """Decision kernels on caller log-luminance samples [n, m] (float64).
        Returns (t, stop, polarity) and, with want_p, the lower-tail
        probability of t at each pixel's degrees of freedom (device CDF)."""
        import torch
        dev = torch.device("cuda", self.device)
        a = torch.as_tensor(x0, dtype=torch.float64).to(dev).contiguous()
        b = torch.as_tensor(x1, dtype=torch.float64).to(dev).contiguous()
        n, m = a.shape
        t = torch.empty(n, dtype=torch.float64, device=dev)
        stop = torch.empty(n, dtype=torch.uint8, device=dev)
        pol = torch.empty(n, dtype=torch.int8, device=dev)
        p = torch.empty(n, dtype=torch.float64, device=dev) if want_p else None
        self._check(load_library().evrt_decide_stats(self._h, _dptr(a), _dptr(b), n, m, float(C), float(alpha),
                                                     int(mode), int(df_mode), _dptr(t), _dptr(stop), _dptr(pol),
                                                     _dptr(p) if p is not None else None, _stream_ptr(stream)))
        return (t, stop, pol, p) if want_p else (t, stop, pol)


# ---------------------------------------------------------------------------
# Differentiable event loss.

_EVENT_LOSS_FN = None


def _event_loss_function():
    global _EVENT_LOSS_FN
    if _EVENT_LOSS_FN is not None:
        return _EVENT_LOSS_FN
    import torch

    class EventLoss(torch.autograd.Function):
        """loss(albedo, emission) of Renderer.event_loss_grad; the backward
        pass returns the path-replay gradient computed with the forward."""

        @staticmethod
        def forward(ctx, albedo, emission, renderer, t0, t1, C, tau, spp, opts):
            renderer.set_materials(albedo.detach().cpu().numpy(), emission.detach().cpu().numpy())
            r = renderer.event_loss_grad(t0, t1, C, tau, spp, opts)
            ctx.save_for_backward(r["grad_albedo"].to(albedo.device, albedo.dtype),
                                  r["grad_emission"].to(emission.device, emission.dtype))
            return r["loss"][0].to(device=albedo.device, dtype=albedo.dtype)

        @staticmethod
        def backward(ctx, g):
            ga, ge = ctx.saved_tensors
            return g * ga, g * ge, None, None, None, None, None, None, None

    _EVENT_LOSS_FN = EventLoss
    return EventLoss


_DELTA_FN = None


def _delta_function():
    global _DELTA_FN
    if _DELTA_FN is not None:
        return _DELTA_FN
    import torch

    class LogLuminanceDelta(torch.autograd.Function):
        """Delta(albedo, emission) per pixel of Renderer.delta_vjp; the
        backward pass is the path-replay vector-Jacobian product with the
        incoming gradient."""

        @staticmethod
        def forward(ctx, albedo, emission, renderer, t0, t1, spp, opts):
            ctx.mats = (albedo.detach().cpu().numpy(), emission.detach().cpu().numpy())
            renderer.set_materials(*ctx.mats)
            ctx.renderer, ctx.args = renderer, (t0, t1, spp, opts)
            ctx.dev = (albedo.device, albedo.dtype, emission.device, emission.dtype)
            d = renderer.delta_vjp(t0, t1, spp, None, opts)["delta"]
            return d.to(device=albedo.device, dtype=albedo.dtype)

        @staticmethod
        def backward(ctx, g):
            t0, t1, spp, opts = ctx.args
            ctx.renderer.set_materials(*ctx.mats)  # the forward's materials
            r = ctx.renderer.delta_vjp(t0, t1, spp, g.detach(), opts)
            ad, at, ed, et = ctx.dev
            return (r["grad_albedo"].to(ad, at), r["grad_emission"].to(ed, et), None, None, None, None, None)

    _DELTA_FN = LogLuminanceDelta
    return LogLuminanceDelta


def log_luminance_delta(renderer: "Renderer", albedo, emission, t0: float, t1: float, spp: int, opts=None):
    """Differentiable per-pixel difference of mean log-luminance between t1
    and t0 (a flat tensor of H*W values) with the given per-material albedo
    and emission tensors; gradients of any function of it flow to both by
    path replay (the backward pass sets the forward's materials again)."""
    return _delta_function().apply(albedo, emission, renderer, t0, t1, spp, opts)


def event_loss(renderer: "Renderer", albedo, emission, t0: float, t1: float, C: float, tau: float,
               spp: int, opts=None):
    """Differentiable smoothed event loss of the renderer's scene with the
    given per-material albedo and emission tensors (any device and float
    dtype); gradients flow to both."""
    return _event_loss_function().apply(albedo, emission, renderer, t0, t1, C, tau, spp, opts)
