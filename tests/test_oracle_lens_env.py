"""Pins of the oracle's environment map and thin-lens camera (the setting of
the paper's failure case, Sec. 5: a background given by an environment map
seen through a lens with depth of field)."""
import math

import numpy as np
import pytest

import oracle
from paper_2408_07996_amd import scenes


def _texel_dir(face, i, j, N, scale=1.0):
    """Direction through the centre of texel (i, j) of a cube-map face: the
    inverse of the face coordinates (sc, tc) of the lookup."""
    sc = 2.0 * (i + 0.5) / N - 1.0
    tc = 2.0 * (j + 0.5) / N - 1.0
    d = {0: (1.0, -tc, -sc), 1: (-1.0, -tc, sc), 2: (sc, 1.0, tc), 3: (sc, -1.0, -tc),
         4: (sc, -tc, 1.0), 5: (-sc, -tc, -1.0)}[face]
    return np.array(d, np.float32) * np.float32(scale)


def _sky_scene(env, width=12, height=8, look=(0.0, 0.0, -1.0)):
    b = scenes.SceneBuilder()
    b.material(0.5)
    b.set_camera(width, height, 60.0, [0.0], [[0, 0, 0, *look, 0, 1, 0]])
    sc = b.build()
    sc.env = env
    return sc


def test_env_lookup_returns_the_texel_of_each_direction():
    N = 6
    env = np.arange(6 * N * N, dtype=np.float32).reshape(6, N, N)
    sc = _sky_scene(env)
    with oracle.Frame(sc, 0, 0) as f:
        for face in range(6):
            for j in range(N):
                for i in range(N):
                    for scale in (1.0, 0.37, 5.0):
                        d = _texel_dir(face, i, j, N, scale)
                        assert f.env_radiance(d) == env[face, j, i], (face, i, j, scale)
        assert f.env_radiance(np.zeros(3)) == 0.0


def test_camera_sees_the_environment():
    """Empty scene, pinhole camera, jitter off: each path's radiance is the
    texel of its pixel's direction."""
    N = 8
    rng = np.random.default_rng(2)
    env = rng.uniform(0.1, 5.0, (6, N, N)).astype(np.float32)
    for look in ((0.0, 0.0, -1.0), (1.0, 0.3, 0.2), (0.1, -1.0, 0.05)):
        sc = _sky_scene(env, look=look)
        p = oracle.make_params(jitter=0)
        with oracle.Frame(sc, 0, 0) as f:
            for px in range(sc.width * sc.height):
                _, d = f.camera_ray(p, px, 0, 0)
                assert f.path_radiance(p, px, 0, 0) == np.float32(f.env_radiance(d))


@pytest.mark.parametrize("D", [1, 2, 5])
def test_plane_under_uniform_sky_is_exact(D):
    """Lambertian plane y = 0 of albedo a under a constant environment L0:
    a camera ray that meets the plane bounces into the open sky, so the path
    carries exactly a L0 (nothing for D = 1); one that misses carries L0."""
    a, L0 = 0.6, 2.5
    b = scenes.SceneBuilder()
    m = b.material(a)
    v, t = scenes.oriented_quad([(-50, 0, -50), (50, 0, -50), (50, 0, 50), (-50, 0, 50)], (0, 1, 0))
    b.static(b.mesh(v, t, m))
    b.set_camera(16, 12, 50.0, [0.0], [[0, 1.5, 3.0, 0, 0.8, 0, 0, 1, 0]])
    sc = b.build()
    sc.env = np.full((6, 4, 4), L0, np.float32)
    p = oracle.make_params(max_depth=D, rr_start_depth=99)
    hit_val = np.float32(0.0) if D == 1 else np.float32(np.float32(a) * np.float32(L0))
    n_hit = 0
    with oracle.Frame(sc, 0, 0) as f:
        for px in range(sc.width * sc.height):
            for s in range(4):
                o, d = f.camera_ray(p, px, 0, s)
                hit, _, _ = f.closest_hit(0, o, d)
                L = f.path_radiance(p, px, 0, s)
                assert L == (hit_val if hit else np.float32(L0)), (px, s, L)
                n_hit += hit
    assert 0 < n_hit < 16 * 12 * 4


def test_thin_lens_rays_pass_through_the_focus_point():
    """Every lens ray of a pixel starts on the aperture disk (radius R, in
    the plane through the eye spanned by right and up) and passes through
    the pinhole ray's point on the plane in focus; the origins cover the
    disk uniformly (mean squared radius R^2 / 2)."""
    R, F = 0.2, 3.0
    sc = scenes.tiny_box(width=16, height=12)
    sc.lens_radius, sc.focus_dist = R, F
    p = oracle.make_params()
    p0 = oracle.make_params(jitter=0)
    r2 = []
    with oracle.Frame(sc, 0, 0) as f:
        cam = f.camera(0)
        eye, fwd, right, up = (cam[k].astype(np.float64) for k in ("eye", "fwd", "right", "up"))
        sx, sy = (float(v) for v in cam["sxy"])
        for px in (0, 37, 95, 191):
            x, y = px % 16, px // 16
            for s in range(200):
                o, d = f.camera_ray(p0, px, 0, s)
                nx = 2.0 * (x + 0.5) / 16 - 1.0
                ny = 1.0 - 2.0 * (y + 0.5) / 12
                d_un = fwd + (nx * sx) * right + (ny * sy) * up
                focus = eye + F * d_un
                off = o.astype(np.float64) - eye
                assert abs(off @ fwd) < 1e-6 and np.linalg.norm(off) <= R * (1 + 1e-6)
                lam = np.linalg.norm(focus - o)
                assert np.linalg.norm(o + lam * d - focus) < 2e-5 * max(1.0, lam)
                r2.append(off @ off)
    assert abs(np.mean(r2) / (R * R / 2) - 1.0) < 0.06
    # Without a lens the origin is the eye.
    sc.lens_radius = 0.0
    with oracle.Frame(sc, 0, 0) as f:
        o, _ = f.camera_ray(p, 5, 0, 3)
        np.testing.assert_array_equal(o, f.camera(0)["eye"])
