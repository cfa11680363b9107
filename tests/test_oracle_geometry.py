"""Pins of the oracle's scene-at-an-instant, camera and ray queries."""
import math

import numpy as np
import pytest

import oracle
from paper_2408_07996_amd import scenes


def _random_rays(rng, n, extent=3.0, targets=None):
    o = rng.uniform(-extent, extent, size=(n, 3)).astype(np.float32)
    if targets is None:
        d = rng.normal(size=(n, 3))
    else:
        d = targets[rng.integers(0, len(targets), n)] - o
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    return o, d


@pytest.mark.parametrize("seed", [0, 1])
def test_bvh_equals_brute_force(seed):
    sc = scenes.triangle_soup(300, seed=seed, moving=True)
    rng = np.random.default_rng(100 + seed)
    with oracle.Frame(sc, 0.0, 1.0) as f:
        for inst in (0, 1):
            tri, _ = f.world_tris(inst)
            # Aim half of the rays exactly at vertices and edge midpoints.
            pts = np.concatenate([tri.reshape(-1, 3), 0.5 * (tri[:, 0] + tri[:, 1])])
            o1, d1 = _random_rays(rng, 1500)
            o2, d2 = _random_rays(rng, 1500, targets=pts)
            for o, d in ((o1, d1), (o2, d2)):
                for k in range(len(o)):
                    skip = int(rng.integers(0, 300)) if k % 3 == 0 else oracle.NO_PRIM
                    a = f.closest_hit(inst, o[k], d[k], skip=skip, brute=True)
                    b = f.closest_hit(inst, o[k], d[k], skip=skip, brute=False)
                    assert a == b
                    tmax = np.float32(rng.uniform(0.5, 6.0))
                    assert (f.any_hit(inst, o[k], d[k], tmax=tmax, skip=skip, brute=True)
                            == f.any_hit(inst, o[k], d[k], tmax=tmax, skip=skip, brute=False))


def test_bvh_equals_brute_force_million_rays():
    """The oracle's BVH against its brute force on 10^6 rays (the batched
    query): 250,000 random and 250,000 aimed at vertices and edge midpoints
    per instant of a moving 300-triangle soup, a third of them skipping a
    primitive; closest hits bit for bit, any-hit answers under random tmax."""
    sc = scenes.triangle_soup(300, seed=7, moving=True)
    rng = np.random.default_rng(107)
    n = 250_000
    with oracle.Frame(sc, 0.0, 1.0) as f:
        for inst in (0, 1):
            tri, _ = f.world_tris(inst)
            pts = np.concatenate([tri.reshape(-1, 3), 0.5 * (tri[:, 0] + tri[:, 1])])
            o1, d1 = _random_rays(rng, n)
            o2, d2 = _random_rays(rng, n, targets=pts)
            o, d = np.concatenate([o1, o2]), np.concatenate([d1, d2])
            skip = np.where(np.arange(2 * n) % 3 == 0, rng.integers(0, 300, 2 * n), oracle.NO_PRIM).astype(np.uint32)
            tmin = np.full(2 * n, 1e-4, np.float32)
            ta, pa = f.ray_queries(inst, o, d, tmin, np.inf, skip, brute=True)
            tb, pb = f.ray_queries(inst, o, d, tmin, np.inf, skip, brute=False)
            np.testing.assert_array_equal(pa, pb)
            np.testing.assert_array_equal(ta.view(np.uint32), tb.view(np.uint32))
            assert 0.1 < (pa != oracle.NO_PRIM).mean() < 0.9
            tmax = rng.uniform(0.5, 6.0, 2 * n).astype(np.float32)
            aa = f.ray_queries(inst, o, d, tmin, tmax, skip, any_hit=True, brute=True)
            ab = f.ray_queries(inst, o, d, tmin, tmax, skip, any_hit=True, brute=False)
            np.testing.assert_array_equal(aa, ab)


def _closed_sphere(subdiv=2):
    b = scenes.SceneBuilder()
    m = b.material(0.5)
    v, t = scenes.icosphere(subdiv)
    b.static(b.mesh(v * 2.0, t, m))
    b.set_camera(8, 8, 40, [0.0], [[0, 0, 0, 0, 0, -1, 0, 1, 0]])
    return b.build()


def test_watertight_closed_mesh():
    """Rays from inside a closed mesh always hit it, also when aimed
    exactly at shared vertices and edges."""
    sc = _closed_sphere()
    rng = np.random.default_rng(4)
    with oracle.Frame(sc, 0, 0, use_bvh=False) as f:
        tri, _ = f.world_tris(0)
        pts = np.concatenate([tri.reshape(-1, 3), 0.5 * (tri[:, 0] + tri[:, 1]),
                              0.5 * (tri[:, 1] + tri[:, 2])])
        for origin in (np.zeros(3), np.array([0.3, -0.2, 0.1])):
            o = origin.astype(np.float32)
            for p in pts:
                d = (p - origin).astype(np.float32)
                hit, t, prim = f.closest_hit(0, o, d, tmin=0.0, brute=True)
                assert hit
            for _ in range(500):
                d = rng.normal(size=3).astype(np.float32)
                assert f.closest_hit(0, o, d, tmin=0.0, brute=True)[0]


def test_single_triangle_against_float64():
    """Hit/miss and distance of one triangle versus an FP64 ray/plane and
    barycentric computation, for rays not grazing an edge."""
    b = scenes.SceneBuilder()
    m = b.material(0.5)
    tri = np.array([[-1.0, -0.5, 0.2], [1.2, -0.7, -0.1], [0.1, 1.1, 0.3]], np.float32)
    b.static(b.mesh(tri, [[0, 1, 2]], m))
    b.set_camera(4, 4, 40, [0.0], [[0, 0, 5, 0, 0, 0, 0, 1, 0]])
    sc = b.build()
    rng = np.random.default_rng(8)
    T = tri.astype(np.float64)
    n = np.cross(T[1] - T[0], T[2] - T[0])
    checked = 0
    with oracle.Frame(sc, 0, 0, use_bvh=False) as f:
        for _ in range(3000):
            o = rng.uniform(-2, 2, 3).astype(np.float32) + np.float32([0, 0, 3])
            d = (rng.uniform(-1.5, 1.5, 3) - o).astype(np.float32)
            od, dd = o.astype(np.float64), d.astype(np.float64)
            denom = n @ dd
            if abs(denom) < 1e-6:
                continue
            t = n @ (T[0] - od) / denom
            p = od + t * dd
            # barycentric coordinates of p
            v0, v1, v2 = T[1] - T[0], T[2] - T[0], p - T[0]
            d00, d01, d11 = v0 @ v0, v0 @ v1, v1 @ v1
            d20, d21 = v2 @ v0, v2 @ v1
            den = d00 * d11 - d01 * d01
            bv = (d11 * d20 - d01 * d21) / den
            bw = (d00 * d21 - d01 * d20) / den
            bu = 1 - bv - bw
            if min(abs(bu), abs(bv), abs(bw)) < 1e-5:
                continue
            inside = bu > 0 and bv > 0 and bw > 0 and t > 1e-4
            hit, th, prim = f.closest_hit(0, o, d, brute=True)
            assert hit == inside
            if inside:
                assert abs(th - t) <= 2e-6 * max(1.0, abs(t))
                assert prim == 0
            checked += 1
    assert checked > 2000


def test_tie_break_lowest_primitive():
    b = scenes.SceneBuilder()
    m = b.material(0.5)
    tri = np.array([[-1, -1, 0], [1, -1, 0], [0, 1, 0]], np.float32)
    b.static(b.mesh(np.concatenate([tri, tri, tri]), [[0, 1, 2], [3, 4, 5], [6, 7, 8]], m))
    b.set_camera(4, 4, 40, [0.0], [[0, 0, 5, 0, 0, 0, 0, 1, 0]])
    with oracle.Frame(b.build(), 0, 0) as f:
        o = np.float32([0.1, 0.0, 2.0])
        d = np.float32([0.0, 0.05, -1.0])
        for brute in (True, False):
            assert f.closest_hit(0, o, d, brute=brute)[2] == 0
            assert f.closest_hit(0, o, d, skip=0, brute=brute)[2] == 1
        # t exactly equal to tmax is outside the open interval.
        hit, t, _ = f.closest_hit(0, o, d, brute=True)
        assert not f.any_hit(0, o, d, tmax=t, brute=True)
        assert not f.closest_hit(0, o, d, tmax=t, brute=True)[0]


def _one_tri_scene(keys_t, xforms):
    b = scenes.SceneBuilder()
    m = b.material(0.5)
    verts = np.array([[0.3, -0.7, 1.25], [1.1, 0.2, -0.4], [-0.6, 0.9, 0.15]], np.float32)
    b.instance(b.mesh(verts, [[0, 1, 2]], m), keys_t, xforms)
    b.set_camera(4, 4, 40, [0.0], [[0, 0, 5, 0, 0, 0, 0, 1, 0]])
    return b.build(), verts


def test_instance_transform_special_cases():
    perm = np.array([[0, 0, 1, 0.0], [0, 1, 0, 0.0], [-1, 0, 0, 0.0]])
    shift = scenes.translation([0.1, -0.25, 0.0])
    sc, v = _one_tri_scene([0.0, 1.0, 2.0], [scenes.identity(), shift, perm])
    with oracle.Frame(sc, 0.0, 2.0) as f:
        w0, _ = f.world_tris(0)
        w2, _ = f.world_tris(1)
    np.testing.assert_array_equal(w0[0], v)                       # identity is exact
    np.testing.assert_array_equal(w2[0], np.stack([v[:, 2], v[:, 1], -v[:, 0]], 1))
    with oracle.Frame(sc, 1.0, 0.5) as f:
        w1, _ = f.world_tris(0)
        wh, _ = f.world_tris(1)
    exp1 = (v.astype(np.float64) + [0.1, -0.25, 0.0]).astype(np.float32)
    np.testing.assert_array_equal(w1[0], exp1)                     # key time: that key
    exph = (v.astype(np.float64) + [0.05, -0.125, 0.0]).astype(np.float32)
    np.testing.assert_allclose(w1[0], exp1)
    assert np.abs(wh[0].astype(np.float64) - exph).max() <= 2 * np.spacing(np.float32(2.0))
    # Outside the key range the end keys hold.
    with oracle.Frame(sc, -5.0, 9.0) as f:
        np.testing.assert_array_equal(f.world_tris(0)[0][0], v)
        np.testing.assert_array_equal(f.world_tris(1)[0][0], w2[0])


def test_pinhole_camera_directions():
    """Jitter off: the ray through pixel (x, y) has direction
    f + nx tan(fov/2) aspect r + ny tan(fov/2) u with nx, ny at the pixel
    centre; checked through the first-hit distance to a wall at z = -4."""
    W, H, fov = 7, 5, 50.0
    b = scenes.SceneBuilder()
    m = b.material(0.0, 1.0)
    v, t = scenes.oriented_quad([(-50, -50, -4), (50, -50, -4), (50, 50, -4), (-50, 50, -4)], (0, 0, 1))
    b.static(b.mesh(v, t, m))
    b.set_camera(W, H, fov, [0.0], [[0, 0, 1, 0, 0, -3, 0, 1, 0]])
    sc = b.build()
    p = oracle.make_params(jitter=0, nee=1, max_depth=1, spp_init=8, spp_batch=8, spp_max=8)
    with oracle.Frame(sc, 0, 0) as f:
        cam = f.camera(0)
        np.testing.assert_allclose(cam["fwd"], [0, 0, -1], atol=0)
        np.testing.assert_allclose(cam["sxy"][1], math.tan(math.radians(fov / 2)), rtol=1e-7)
        np.testing.assert_allclose(cam["sxy"][0], math.tan(math.radians(fov / 2)) * W / H, rtol=1e-7)
        # The emitter (albedo 0) is the first and only hit, so L = Le for every
        # pixel whose ray meets the wall -- all of them.
        for px in range(W * H):
            assert f.path_radiance(p, px, 0, 0) == np.float32(1.0)
        # Centre pixel of an odd-sized image looks straight ahead.
        o = cam["eye"]
        hit, t, _ = f.closest_hit(0, o, np.float32([0, 0, -1]))
        assert hit and abs(t - 5.0) < 1e-6


def test_sensor_scene_variants():
    """scenes.sensor(n_moving=1, sky=s): the same scene at t = 0, at t = 1
    only the first sphere has moved (the floor comes first, then the spheres
    of 1,280 triangles each), and a uniform sky of radiance s."""
    a = scenes.sensor()
    b = scenes.sensor(n_moving=1, sky=2.0)
    assert a.env is None and b.env.shape == (6, 8, 8) and (b.env == 2.0).all()
    floor, sphere = 190 * 190 * 2, 1280
    with oracle.Frame(a, 0.0, 1.0) as fa, oracle.Frame(b, 0.0, 1.0) as fb:
        a0, a1 = fa.world_tris(0)[0], fa.world_tris(1)[0]
        b0, b1 = fb.world_tris(0)[0], fb.world_tris(1)[0]
    np.testing.assert_array_equal(a0, b0)
    np.testing.assert_array_equal(b1[:floor + sphere], a1[:floor + sphere])
    np.testing.assert_array_equal(b1[floor + sphere:], b0[floor + sphere:])
    assert not np.array_equal(a1[floor + sphere:floor + 20 * sphere], a0[floor + sphere:floor + 20 * sphere])
