"""CPU oracle for the adaptive event-camera path tracer (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares
no code with the GPU library: the C sources under ``oracle/src`` implement
the written definitions independently (Philox keying, scene at an instant,
camera, watertight intersection, the path estimator, FP64 statistics, the
Student t CDF, and Algorithm 1 of the paper for one pair of instants).

Functions without an independent pin are flagged "parity unpinned" in their
docstrings; see the oracle tests for the pins of the others.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MODE_ADAPTIVE_1T, MODE_FIXED, MODE_ADAPTIVE_2T, MODE_MEAN_ONLY = 0, 1, 2, 3
DF_STUDENT, DF_WELCH = 0, 1
REF_LOCKSTEP, REF_FULL = 0, 1
NO_PRIM = 0xFFFFFFFF

_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def luminance(r: float, g: float, b: float) -> float:
    """The oracle's luminance of linear RGB (Rec. 709), FP32."""
    return float(lib().evo_luminance(float(r), float(g), float(b)))


class _SceneDesc(ctypes.Structure):
    _fields_ = [
        ("n_mat", ctypes.c_uint32), ("albedo", _f32p), ("emission", _f32p),
        ("n_vert", ctypes.c_uint32), ("xyz", _f32p),
        ("n_tri", ctypes.c_uint32), ("tri_idx", _u32p), ("tri_mat", _u32p),
        ("n_mesh", ctypes.c_uint32), ("mesh_tri_off", _u32p),
        ("n_inst", ctypes.c_uint32), ("inst_mesh", _u32p), ("inst_key_off", _u32p),
        ("key_t", _f64p), ("key_xform", _f64p),
        ("n_plight", ctypes.c_uint32), ("pl_pos", _f32p), ("pl_intensity", _f32p),
        ("width", ctypes.c_uint32), ("height", ctypes.c_uint32), ("vfov_deg", ctypes.c_double),
        ("cam_nkeys", ctypes.c_uint32), ("cam_t", _f64p), ("cam_elu", _f64p),
        ("env_res", ctypes.c_uint32), ("env", _f32p),
        ("lens_radius", ctypes.c_float), ("focus_dist", ctypes.c_float),
        ("albedo_rgb", _f32p), ("emission_rgb", _f32p), ("pl_rgb", _f32p),
    ]


class Params(ctypes.Structure):
    _fields_ = [
        ("seed", ctypes.c_uint64),
        ("spp_init", ctypes.c_uint32), ("spp_batch", ctypes.c_uint32), ("spp_max", ctypes.c_uint32),
        ("max_depth", ctypes.c_uint32), ("rr_start_depth", ctypes.c_uint32),
        ("minibatch", ctypes.c_uint32), ("log_eps", ctypes.c_double),
        ("C", ctypes.c_float), ("alpha", ctypes.c_float),
        ("nee", ctypes.c_uint8), ("jitter", ctypes.c_uint8), ("mode", ctypes.c_uint8),
        ("df_mode", ctypes.c_uint8), ("ref_mode", ctypes.c_uint8), ("mis", ctypes.c_uint8),
        ("key_base", ctypes.c_uint32), ("normality_alpha", ctypes.c_float),
    ]


class _PixelOut(ctypes.Structure):
    _fields_ = [
        ("polarity", ctypes.c_int8), ("decided_early", ctypes.c_uint8),
        ("near_crit", ctypes.c_uint8), ("pad", ctypes.c_uint8),
        ("n_paths", ctypes.c_uint32), ("n_paths_ref", ctypes.c_uint32), ("rounds", ctypes.c_uint32),
        ("mean", ctypes.c_double * 2), ("var", ctypes.c_double * 2),
        ("mean_radiance", ctypes.c_double * 2), ("t_last", ctypes.c_double),
        ("crit_margin", ctypes.c_double),
    ]


REC_MAX = 64


class _PathRec(ctypes.Structure):
    _fields_ = [
        ("n_vert", ctypes.c_uint32), ("n_term", ctypes.c_uint32),
        ("vmat", ctypes.c_uint32 * REC_MAX), ("vlb", ctypes.c_float * REC_MAX),
        ("tmat", ctypes.c_uint32 * (2 * REC_MAX)), ("tval", ctypes.c_float * (2 * REC_MAX)),
    ]


def lib():
    """Load liboracle.so (building it with gcc first if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    L = ctypes.CDLL(_LIB_PATH)
    L.evo_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.evo_u01.argtypes = [ctypes.c_uint32]
    L.evo_luminance.argtypes = [ctypes.c_float] * 3
    L.evo_luminance.restype = ctypes.c_float
    L.evo_u01.restype = ctypes.c_float
    for name, nargs in (("evo_t_cdf", 2), ("evo_t_ppf", 2), ("evo_ibeta", 3)):
        fn = getattr(L, name)
        fn.argtypes = [ctypes.c_double] * nargs
        fn.restype = ctypes.c_double
    L.evo_scene_new.argtypes = [ctypes.POINTER(_SceneDesc)]
    L.evo_scene_new.restype = ctypes.c_void_p
    L.evo_scene_free.argtypes = [ctypes.c_void_p]
    L.evo_frame_new.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int]
    L.evo_frame_new.restype = ctypes.c_void_p
    L.evo_frame_free.argtypes = [ctypes.c_void_p]
    L.evo_frame_num_tris.argtypes = [ctypes.c_void_p]
    L.evo_frame_num_tris.restype = ctypes.c_uint32
    L.evo_frame_world_tris.argtypes = [ctypes.c_void_p, ctypes.c_int, _f32p, _u32p]
    L.evo_frame_camera.argtypes = [ctypes.c_void_p, ctypes.c_int, _f32p, _f32p, _f32p, _f32p, _f32p]
    L.evo_closest_hit.argtypes = [ctypes.c_void_p, ctypes.c_int, _f32p, _f32p, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_uint32, ctypes.c_int, _f32p, _u32p]
    L.evo_any_hit.argtypes = [ctypes.c_void_p, ctypes.c_int, _f32p, _f32p, ctypes.c_float,
                              ctypes.c_float, ctypes.c_uint32, ctypes.c_int]
    L.evo_ray_queries.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, _f32p, _f32p, _f32p, _f32p,
                                  _u32p, ctypes.c_int, ctypes.c_int, _f32p, _u32p]
    L.evo_ray_queries.restype = None
    L.evo_path_radiance.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_uint32,
                                    ctypes.c_int, ctypes.c_uint32]
    L.evo_path_radiance.restype = ctypes.c_float
    L.evo_path_radiance_rec.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_uint32,
                                        ctypes.c_int, ctypes.c_uint32, ctypes.POINTER(_PathRec)]
    L.evo_path_radiance_rec.restype = ctypes.c_float
    L.evo_event_loss.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_double,
                                 ctypes.c_double, ctypes.c_uint32, _u32p, ctypes.c_uint32, ctypes.c_int,
                                 _f64p, _f64p, _f64p, _f64p, _f64p]
    L.evo_delta_vjp.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_uint32, _f64p, _u32p,
                                ctypes.c_uint32, ctypes.c_int, _f64p, _f64p, _f64p, _f64p]
    L.evo_paths_batch.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_uint32,
                                  _u32p, _u8p, _u32p, _f32p, ctypes.c_int]
    L.evo_decide.argtypes = [_f64p, ctypes.c_uint32, _f64p, ctypes.c_uint32, ctypes.c_float,
                             ctypes.c_float, ctypes.c_int, ctypes.c_int, _f64p, _f64p, _f64p,
                             ctypes.POINTER(ctypes.c_int), _f64p]
    L.evo_camera_ray.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_uint32, ctypes.c_int,
                                 ctypes.c_uint32, _f32p, _f32p]
    L.evo_env_radiance.restype = ctypes.c_float
    L.evo_env_radiance.argtypes = [ctypes.c_void_p, _f32p]
    L.evo_jarque_bera.restype = ctypes.c_double
    L.evo_jarque_bera.argtypes = [_f64p, ctypes.c_uint32]
    L.evo_crit_margin.restype = ctypes.c_double
    L.evo_crit_margin.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_float, ctypes.c_int]
    L.evo_render.argtypes = [ctypes.c_void_p, ctypes.POINTER(Params), _u32p, ctypes.c_uint32,
                             ctypes.c_int, ctypes.POINTER(_PixelOut)]
    L.evo_render_video.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint32, ctypes.POINTER(Params),
                                   _u32p, ctypes.c_uint32, ctypes.c_int, ctypes.POINTER(_PixelOut)]
    _lib = L
    return L


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# ---------------------------------------------------------------------------
# Small pure functions.

def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 of one 4-word counter under a 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().evo_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def u01(x: int) -> float:
    return float(lib().evo_u01(int(x)))


def t_cdf(t: float, df: float) -> float:
    return float(lib().evo_t_cdf(float(t), float(df)))


def t_ppf(p: float, df: float) -> float:
    return float(lib().evo_t_ppf(float(p), float(df)))


def ibeta(a: float, b: float, x: float) -> float:
    return float(lib().evo_ibeta(float(a), float(b), float(x)))


def decide(x0, x1, C: float, alpha: float, df_mode: int = DF_STUDENT,
           mode: int = MODE_ADAPTIVE_1T) -> Dict[str, float]:
    """t statistic (Eq. 7), lower-tail p-value, degrees of freedom, the
    stop decision and the exemption margin (distance of t from the
    critical value(s) of `mode`) for two sets of log-luminance samples."""
    a = np.ascontiguousarray(x0, dtype=np.float64)
    b = np.ascontiguousarray(x1, dtype=np.float64)
    t = ctypes.c_double()
    p = ctypes.c_double()
    df = ctypes.c_double()
    stop = ctypes.c_int()
    margin = ctypes.c_double()
    rc = lib().evo_decide(_ptr(a, ctypes.c_double), len(a), _ptr(b, ctypes.c_double), len(b),
                          float(C), float(alpha), int(df_mode), int(mode), ctypes.byref(t),
                          ctypes.byref(p), ctypes.byref(df), ctypes.byref(stop), ctypes.byref(margin))
    if rc != 0:
        raise ValueError("decide needs at least two samples per instant")
    return dict(t=t.value, p=p.value, df=df.value, stop=bool(stop.value), margin=margin.value)


def jarque_bera(x) -> float:
    """Jarque-Bera statistic of a sample (normality pre-test)."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().evo_jarque_bera(_ptr(a, ctypes.c_double), len(a)))


def crit_margin(mode: int, t: float, df: float, alpha: float, final_check: bool = False) -> float:
    """Exemption margin of one executed decision (see evo_crit_margin)."""
    return float(lib().evo_crit_margin(int(mode), float(t), float(df), float(alpha), int(final_check)))


def make_params(**kw) -> Params:
    base = dict(seed=0, spp_init=16, spp_batch=16, spp_max=256, max_depth=4, rr_start_depth=2,
                minibatch=4, log_eps=1e-4, C=0.2, alpha=0.01, nee=1, jitter=1, mode=0,
                df_mode=0, ref_mode=0, key_base=0, mis=0, normality_alpha=0.0)
    base.update(kw)
    p = Params()
    for k, v in base.items():
        setattr(p, k, v)
    return p


# ---------------------------------------------------------------------------
# Scene and frame.

class Frame:
    """The scene at the two instants (t0, t1) of one event frame."""

    def __init__(self, scene, t0: float = 0.0, t1: float = 1.0, use_bvh: bool = True):
        L = lib()
        self.scene = scene
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        d = _SceneDesc()
        albedo = arr(scene.albedo, np.float32)
        emission = arr(scene.emission, np.float32)
        xyz = arr(scene.xyz, np.float32)
        tri_idx = arr(scene.tri_idx, np.uint32)
        tri_mat = arr(scene.tri_mat, np.uint32)
        mesh_off = arr(scene.mesh_tri_off, np.uint32)
        inst_mesh = arr(scene.inst_mesh, np.uint32)
        inst_off = arr(scene.inst_key_off, np.uint32)
        key_t = arr(scene.key_t, np.float64)
        key_x = arr(scene.key_xform, np.float64)
        pl_pos = arr(scene.pl_pos, np.float32)
        pl_int = arr(scene.pl_intensity, np.float32)
        cam_t = arr(scene.cam_t, np.float64)
        cam_elu = arr(scene.cam_elu, np.float64)
        d.n_mat = len(albedo)
        d.albedo = _ptr(albedo, ctypes.c_float)
        d.emission = _ptr(emission, ctypes.c_float)
        d.n_vert = len(xyz)
        d.xyz = _ptr(xyz, ctypes.c_float)
        d.n_tri = len(tri_idx)
        d.tri_idx = _ptr(tri_idx, ctypes.c_uint32)
        d.tri_mat = _ptr(tri_mat, ctypes.c_uint32)
        d.n_mesh = len(mesh_off) - 1
        d.mesh_tri_off = _ptr(mesh_off, ctypes.c_uint32)
        d.n_inst = len(inst_mesh)
        d.inst_mesh = _ptr(inst_mesh, ctypes.c_uint32)
        d.inst_key_off = _ptr(inst_off, ctypes.c_uint32)
        d.key_t = _ptr(key_t, ctypes.c_double)
        d.key_xform = _ptr(key_x, ctypes.c_double)
        d.n_plight = len(pl_int)
        d.pl_pos = _ptr(pl_pos, ctypes.c_float)
        d.pl_intensity = _ptr(pl_int, ctypes.c_float)
        d.width = scene.width
        d.height = scene.height
        d.vfov_deg = scene.vfov_deg
        d.cam_nkeys = len(cam_t)
        d.cam_t = _ptr(cam_t, ctypes.c_double)
        env = getattr(scene, "env", None)
        if env is not None:
            env = arr(env, np.float32)
            d.env_res = env.shape[-1]
            d.env = _ptr(env, ctypes.c_float)
        d.lens_radius = float(getattr(scene, "lens_radius", 0.0))
        d.focus_dist = float(getattr(scene, "focus_dist", 1.0))
        d.cam_elu = _ptr(cam_elu, ctypes.c_double)
        alb3 = getattr(scene, "albedo_rgb", None)
        if alb3 is not None:
            alb3 = arr(alb3, np.float32).reshape(-1, 3)
            emi3 = arr(scene.emission_rgb, np.float32).reshape(-1, 3)
            if len(alb3) != len(albedo) or len(emi3) != len(albedo):
                raise ValueError("RGB materials must match the material count")
            d.albedo_rgb = _ptr(alb3, ctypes.c_float)
            d.emission_rgb = _ptr(emi3, ctypes.c_float)
            pl3 = getattr(scene, "pl_rgb", None)
            if pl3 is not None:
                pl3 = arr(pl3, np.float32).reshape(-1, 3)
                if len(pl3) != len(pl_int):
                    raise ValueError("RGB point-light intensities must match the light count")
                d.pl_rgb = _ptr(pl3, ctypes.c_float)
        self._scene = L.evo_scene_new(ctypes.byref(d))
        self._keep = []
        self._frame = L.evo_frame_new(self._scene, float(t0), float(t1), int(bool(use_bvh)))
        self.n_tri = int(L.evo_frame_num_tris(self._frame))

    def close(self) -> None:
        if getattr(self, "_frame", None):
            lib().evo_frame_free(self._frame)
            self._frame = None
        if getattr(self, "_scene", None):
            lib().evo_scene_free(self._scene)
            self._scene = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def world_tris(self, instant: int):
        xyz = np.zeros((self.n_tri, 3, 3), dtype=np.float32)
        mat = np.zeros(self.n_tri, dtype=np.uint32)
        lib().evo_frame_world_tris(self._frame, int(instant), _ptr(xyz, ctypes.c_float),
                                   _ptr(mat, ctypes.c_uint32))
        return xyz, mat

    def camera(self, instant: int):
        bufs = [np.zeros(3, np.float32) for _ in range(4)] + [np.zeros(2, np.float32)]
        lib().evo_frame_camera(self._frame, int(instant), *[_ptr(b, ctypes.c_float) for b in bufs])
        return dict(eye=bufs[0], fwd=bufs[1], right=bufs[2], up=bufs[3], sxy=bufs[4])

    def closest_hit(self, instant, o, d, tmin=1e-4, tmax=np.inf, skip=NO_PRIM, brute=False):
        o = np.ascontiguousarray(o, np.float32)
        d = np.ascontiguousarray(d, np.float32)
        t = ctypes.c_float()
        p = ctypes.c_uint32()
        hit = lib().evo_closest_hit(self._frame, int(instant), _ptr(o, ctypes.c_float),
                                    _ptr(d, ctypes.c_float), float(tmin), float(tmax), int(skip),
                                    int(bool(brute)), ctypes.byref(t), ctypes.byref(p))
        return (bool(hit), np.float32(t.value), int(p.value))

    def any_hit(self, instant, o, d, tmin=1e-4, tmax=np.inf, skip=NO_PRIM, brute=False) -> bool:
        o = np.ascontiguousarray(o, np.float32)
        d = np.ascontiguousarray(d, np.float32)
        return bool(lib().evo_any_hit(self._frame, int(instant), _ptr(o, ctypes.c_float),
                                      _ptr(d, ctypes.c_float), float(tmin), float(tmax), int(skip),
                                      int(bool(brute))))

    def ray_queries(self, instant, o, d, tmin, tmax, skip, any_hit=False, brute=False):
        """closest_hit (t, primitive arrays) or any_hit (0/1 array) for n rays
        at once: o, d [n, 3]; tmin, tmax, skip [n]."""
        o = np.ascontiguousarray(o, np.float32).reshape(-1, 3)
        d = np.ascontiguousarray(d, np.float32).reshape(-1, 3)
        n = len(o)
        tmin = np.ascontiguousarray(np.broadcast_to(np.asarray(tmin, np.float32), (n,)))
        tmax = np.ascontiguousarray(np.broadcast_to(np.asarray(tmax, np.float32), (n,)))
        skip = np.ascontiguousarray(np.broadcast_to(np.asarray(skip, np.uint32), (n,)))
        assert d.shape == o.shape
        t = np.zeros(n, np.float32)
        p = np.zeros(n, np.uint32)
        lib().evo_ray_queries(self._frame, int(instant), n, _ptr(o, ctypes.c_float), _ptr(d, ctypes.c_float),
                              _ptr(tmin, ctypes.c_float), _ptr(tmax, ctypes.c_float), _ptr(skip, ctypes.c_uint32),
                              int(bool(any_hit)), int(bool(brute)), _ptr(t, ctypes.c_float),
                              _ptr(p, ctypes.c_uint32))
        return p if any_hit else (t, p)

    def camera_ray(self, params: Params, pixel: int, instant: int, sample: int):
        """(origin, unit direction) of a path sample's camera ray."""
        o = np.zeros(3, np.float32)
        d = np.zeros(3, np.float32)
        lib().evo_camera_ray(self._frame, ctypes.byref(params), int(pixel), int(instant), int(sample),
                             _ptr(o, ctypes.c_float), _ptr(d, ctypes.c_float))
        return o, d

    def env_radiance(self, d) -> float:
        v = np.ascontiguousarray(d, np.float32)
        return float(lib().evo_env_radiance(self._frame, _ptr(v, ctypes.c_float)))

    def path_radiance(self, params: Params, pixel: int, instant: int, sample: int) -> np.float32:
        return np.float32(lib().evo_path_radiance(self._frame, ctypes.byref(params), int(pixel),
                                                  int(instant), int(sample)))

    def path_record(self, params: Params, pixel: int, instant: int, sample: int):
        """Radiance of one path and its derivative record: (L, [(material,
        radiance before the vertex's light samples)], [(emitter material,
        term value)])."""
        rec = _PathRec()
        L = lib().evo_path_radiance_rec(self._frame, ctypes.byref(params), int(pixel), int(instant),
                                        int(sample), ctypes.byref(rec))
        verts = [(int(rec.vmat[k]), np.float32(rec.vlb[k])) for k in range(rec.n_vert)]
        terms = [(int(rec.tmat[k]), np.float32(rec.tval[k])) for k in range(rec.n_term)]
        return np.float32(L), verts, terms

    def path_gradient(self, params: Params, pixel: int, instant: int, sample: int):
        """dL/d albedo and dL/d emission (per material, FP64) of one path with
        its sampling decisions held fixed."""
        L, verts, terms = self.path_record(params, pixel, instant, sample)
        alb = np.asarray(self.scene.albedo, np.float32)
        emi = np.asarray(self.scene.emission, np.float32)
        ga = np.zeros(len(alb))
        ge = np.zeros(len(emi))
        for m, lb in verts:
            ga[m] += (float(L) - float(lb)) / float(alb[m])
        for m, v in terms:
            ge[m] += float(v) / float(emi[m])
        return L, ga, ge

    def event_loss(self, params: Params, C: float, tau: float, spp: int,
                   pixels: Optional[np.ndarray] = None, threads: int = 0) -> Dict[str, np.ndarray]:
        """Smoothed event loss sum softplus((|Delta| - C) / tau) at a fixed
        count of spp paths per pixel and instant, and its gradient with
        respect to every material's albedo and emission (FP64)."""
        nm = len(self.scene.albedo)
        n = self.scene.width * self.scene.height if pixels is None else len(pixels)
        px = None if pixels is None else np.ascontiguousarray(pixels, np.uint32)
        loss = np.zeros(1)
        ga = np.zeros(nm)
        ge = np.zeros(nm)
        lpx = np.zeros(n)
        dpx = np.zeros(n)
        rc = lib().evo_event_loss(self._frame, ctypes.byref(params), float(C), float(tau), int(spp),
                                  None if px is None else _ptr(px, ctypes.c_uint32), n, int(threads),
                                  _ptr(loss, ctypes.c_double), _ptr(ga, ctypes.c_double),
                                  _ptr(ge, ctypes.c_double), _ptr(lpx, ctypes.c_double),
                                  _ptr(dpx, ctypes.c_double))
        if rc != 0:
            raise ValueError("invalid event-loss parameters")
        return dict(loss=float(loss[0]), grad_albedo=ga, grad_emission=ge, loss_px=lpx, delta=dpx)

    def delta_vjp(self, params: Params, spp: int, g, pixels: Optional[np.ndarray] = None,
                  threads: int = 0) -> Dict[str, np.ndarray]:
        """sum_p g_p Delta_p over the listed pixels (every pixel when None)
        and its gradient with respect to every material's albedo and
        emission (FP64), with Delta the per-pixel log-luminance difference at
        spp paths per pixel and instant."""
        nm = len(self.scene.albedo)
        n = self.scene.width * self.scene.height if pixels is None else len(pixels)
        px = None if pixels is None else np.ascontiguousarray(pixels, np.uint32)
        g = np.ascontiguousarray(g, np.float64)
        assert g.shape == (n,)
        val = np.zeros(1)
        ga = np.zeros(nm)
        ge = np.zeros(nm)
        dpx = np.zeros(n)
        rc = lib().evo_delta_vjp(self._frame, ctypes.byref(params), int(spp), _ptr(g, ctypes.c_double),
                                 None if px is None else _ptr(px, ctypes.c_uint32), n, int(threads),
                                 _ptr(val, ctypes.c_double), _ptr(ga, ctypes.c_double), _ptr(ge, ctypes.c_double),
                                 _ptr(dpx, ctypes.c_double))
        if rc != 0:
            raise ValueError("invalid parameters")
        return dict(value=float(val[0]), grad_albedo=ga, grad_emission=ge, delta=dpx)

    def paths(self, params: Params, pixel, instant, sample, threads: int = 0) -> np.ndarray:
        """Per-path radiance for arrays of (pixel, instant, sample)."""
        px = np.ascontiguousarray(pixel, np.uint32).reshape(-1)
        it = np.ascontiguousarray(np.broadcast_to(instant, px.shape), np.uint8)
        sm = np.ascontiguousarray(np.broadcast_to(sample, px.shape), np.uint32)
        out = np.zeros(px.shape, np.float32)
        lib().evo_paths_batch(self._frame, ctypes.byref(params), len(px), _ptr(px, ctypes.c_uint32),
                              _ptr(it, ctypes.c_uint8), _ptr(sm, ctypes.c_uint32),
                              _ptr(out, ctypes.c_float), int(threads))
        return out

    def render(self, params: Params, pixels: Optional[np.ndarray] = None,
               threads: int = 0) -> Dict[str, np.ndarray]:
        """Algorithm 1 for one pair of instants on a pixel subset (default:
        every pixel).  Returns per-pixel arrays."""
        if pixels is None:
            pixels = np.arange(self.scene.width * self.scene.height, dtype=np.uint32)
        px = np.ascontiguousarray(pixels, np.uint32)
        out = (_PixelOut * max(1, len(px)))()
        rc = lib().evo_render(self._frame, ctypes.byref(params), _ptr(px, ctypes.c_uint32),
                              len(px), int(threads), out)
        if rc != 0:
            raise ValueError("invalid render parameters")
        return _pixel_dict(px, np.ctypeslib.as_array(out)[: len(px)])


def _pixel_dict(px, raw):
    """Per-pixel oracle outputs (structured array) as a dict of arrays."""
    return dict(
        pixels=px.copy(),
        polarity=raw["polarity"].astype(np.int8),
        decided_early=raw["decided_early"].astype(bool),
        near_crit=raw["near_crit"].astype(bool),
        n_paths=raw["n_paths"].astype(np.uint32),
        n_paths_ref=raw["n_paths_ref"].astype(np.uint32),
        rounds=raw["rounds"].astype(np.uint32),
        mean=raw["mean"].astype(np.float64).copy(),
        var=raw["var"].astype(np.float64).copy(),
        mean_radiance=raw["mean_radiance"].astype(np.float64).copy(),
        t_last=raw["t_last"].astype(np.float64),
        crit_margin=raw["crit_margin"].astype(np.float64),
    )


def render_video(scene, times, params: Params, pixels: Optional[np.ndarray] = None,
                 threads: int = 0) -> Dict[str, np.ndarray]:
    """Sequential event video over frames at `times` (Algorithm 1 with the
    reference carried per pixel and replaced at events; frame 0 at the full
    count).  Arrays have a leading axis of len(times) - 1 frames."""
    times = [float(t) for t in times]
    if len(times) < 2:
        raise ValueError("need at least two frames")
    frames = [Frame(scene, times[k - 1], times[k]) for k in range(1, len(times))]
    try:
        if pixels is None:
            pixels = np.arange(scene.width * scene.height, dtype=np.uint32)
        px = np.ascontiguousarray(pixels, np.uint32)
        nf = len(times) - 1
        out = (_PixelOut * max(1, nf * len(px)))()
        ptrs = (ctypes.c_void_p * nf)(*[f._frame for f in frames])
        rc = lib().evo_render_video(ptrs, len(times), ctypes.byref(params), _ptr(px, ctypes.c_uint32), len(px),
                                    int(threads), out)
        if rc != 0:
            raise ValueError("invalid video parameters")
        raw = np.ctypeslib.as_array(out)[: nf * len(px)].reshape(nf, len(px))
        return _pixel_dict(px, raw)
    finally:
        for f in frames:
            f.close()
