"""Closed-form pins of the oracle's per-path radiance estimator."""
import math

import numpy as np
import pytest

import oracle
from paper_2408_07996_amd import scenes


def _all_paths(f, p, pixels, spp, instant=0):
    px = np.repeat(np.asarray(pixels, np.uint32), spp)
    sm = np.tile(np.arange(spp, dtype=np.uint32), len(pixels))
    return f.paths(p, px, instant, sm).reshape(len(pixels), spp)


@pytest.mark.parametrize("a,Le,D", [(0.5, 1.0, 4), (0.8, 2.5, 6), (0.3, 10.0, 1)])
def test_white_furnace_nee_off_is_exact(a, Le, D):
    """Closed box, every wall albedo a and emission Le, NEE and roulette
    off: a path gathers Le at each of its D vertices with throughput a^k,
    so L = Le (1 - a^D) / (1 - a) for every path."""
    sc = scenes.furnace(a, Le, 12, 12)
    p = oracle.make_params(nee=0, max_depth=D, rr_start_depth=D + 10)
    expect = Le * (1 - a ** D) / (1 - a)
    with oracle.Frame(sc, 0, 0) as f:
        L = _all_paths(f, p, range(144), 512).astype(np.float64)
    exact = np.abs(L - expect) <= 1e-5 * expect
    # Every other path ended early: it carries the first j terms of the
    # series, 1 <= j < D, which is what a bounce ray that leaves the box
    # through a corner gap returns (test_furnace_corner_gap_lets_a_ray_out).
    # Such a ray must start within the self-intersection offset of an edge,
    # on about 1e-4 of the paths (9 of 73,728 here).
    partial = Le * (1 - a ** np.arange(1, D)) / (1 - a)
    for v in L[~exact]:
        assert np.abs(partial - v).min() <= 1e-5 * expect, v
    assert (~exact).sum() <= 1e-3 * L.size
    if D == 1:
        assert exact.all()


def test_furnace_corner_gap_lets_a_ray_out():
    """The furnace's only loss: a ray that leaves the floor 3e-5 from the
    wall x = 1, heading into it at 45 degrees, meets it at t = 4.2e-5,
    inside the self-intersection offset t_min = 1e-4, so the hit is skipped
    and the ray leaves the box; 3e-2 from the wall it stops there, and with
    t_min = 1e-6 the near hit is found.  BVH and brute force agree."""
    d = np.array([1, 1, 0], np.float32) / np.float32(math.sqrt(2.0))
    near = np.array([1 - 3e-5, -1, 0.1], np.float32)
    far = np.array([1 - 3e-2, -1, 0.1], np.float32)
    with oracle.Frame(scenes.furnace(0.5, 1.0, 4, 4), 0, 0) as f:
        for brute in (True, False):
            assert not f.closest_hit(0, near, d, tmin=1e-4, brute=brute)[0]
            hit, t, _ = f.closest_hit(0, far, d, tmin=1e-4, brute=brute)
            assert hit and t == pytest.approx(3e-2 * math.sqrt(2.0), rel=1e-4)
            hit, t, _ = f.closest_hit(0, near, d, tmin=1e-6, brute=brute)
            assert hit and t == pytest.approx(3e-5 * math.sqrt(2.0), rel=2e-2)


def test_white_furnace_zero_variance_decides_at_spp_init():
    sc = scenes.furnace(0.5, 1.0, 8, 8)
    p = oracle.make_params(nee=0, max_depth=3, rr_start_depth=99, spp_init=16, spp_batch=16,
                           spp_max=256, C=0.2, alpha=0.01)
    expect = 1.0 * (1 - 0.5 ** 3) / 0.5
    with oracle.Frame(sc, 0, 0) as f:
        r = f.render(p)
    exact = np.abs(r["mean_radiance"] - expect).max(axis=1) <= 1e-5 * expect
    # A pixel is inexact only if one of its paths ends early through a corner
    # gap (about 1e-4 of the paths): none of these 64 pixels.
    assert exact.sum() >= exact.size - 1
    assert (r["n_paths"][exact] == 16).all()
    assert (r["var"][exact] == 0).all()
    assert np.isneginf(r["t_last"][exact]).all()
    assert (r["polarity"] == 0).all()
    np.testing.assert_allclose(r["mean"][exact], math.log(float(np.float32(expect)) + 1e-4), rtol=1e-7)


def test_white_furnace_nee_and_roulette_unbiased():
    """With NEE every vertex also gathers a * Le of direct light, so the
    expected radiance is Le (1 - a^(D+1)) / (1 - a); roulette keeps it
    unbiased."""
    a, Le, D = 0.6, 1.5, 4
    sc = scenes.furnace(a, Le, 8, 8)
    expect = Le * (1 - a ** (D + 1)) / (1 - a)
    for rr in (2, 99):
        p = oracle.make_params(nee=1, max_depth=D, rr_start_depth=rr)
        with oracle.Frame(sc, 0, 0) as f:
            L = _all_paths(f, p, range(64), 512).astype(np.float64).reshape(-1)
        se = L.std(ddof=1) / math.sqrt(len(L))
        assert abs(L.mean() - expect) < 4 * se + 1e-3 * expect, (rr, L.mean(), expect, se)


def _pinhole_rays(sc):
    e, look, up = sc.cam_elu[0, :3], sc.cam_elu[0, 3:6], sc.cam_elu[0, 6:9]
    fw = (look - e) / np.linalg.norm(look - e)
    r = np.cross(fw, up)
    r /= np.linalg.norm(r)
    u = np.cross(r, fw)
    th = math.tan(math.radians(sc.vfov_deg) / 2)
    xs, ys = np.meshgrid(np.arange(sc.width), np.arange(sc.height))
    nx = 2 * (xs + 0.5) / sc.width - 1
    ny = 1 - 2 * (ys + 0.5) / sc.height
    d = fw + (nx * th * sc.width / sc.height)[..., None] * r + (ny * th)[..., None] * u
    return e, d.reshape(-1, 3)


@pytest.mark.parametrize("D", [1, 3])
def test_plane_under_point_light_exact(D):
    """Lambertian plane y = 0 and a point light of intensity I at height h:
    L(x) = (a / pi) I cos(theta) / r^2 = (a / pi) I h / r^3, deterministic
    (jitter off; the bounce leaves into empty space)."""
    a, I, h = 0.7, 5.0, 1.5
    sc = scenes.plane_point_light(a, I, h, 24, 16)
    lp = sc.pl_pos[0].astype(np.float64)
    e, d = _pinhole_rays(sc)
    p = oracle.make_params(jitter=0, max_depth=D, spp_init=8, spp_batch=8, spp_max=8)
    n_checked = 0
    with oracle.Frame(sc, 0, 0) as f:
        for px in range(sc.width * sc.height):
            if d[px, 1] >= -1e-3:
                continue
            t = -e[1] / d[px, 1]
            x = e + t * d[px]
            if np.abs(x).max() > 20:
                continue
            r = np.linalg.norm(lp - x)
            expect = a / math.pi * I * (lp[1] - x[1]) / r ** 3
            got = [float(f.path_radiance(p, px, 0, s)) for s in range(3)]
            assert got[0] == got[1] == got[2]
            assert abs(got[0] - expect) <= 2e-5 * expect, (px, got[0], expect)
            n_checked += 1
    assert n_checked > 200


def _polygon_irradiance(x, n, poly, Le):
    """Lambert's polygon formula: E = (Le / 2) sum_i Theta_i (n . Gamma_i)."""
    g = poly - x
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    tot = 0.0
    for i in range(len(poly)):
        a, b = g[i], g[(i + 1) % len(poly)]
        theta = math.acos(np.clip(a @ b, -1, 1))
        c = np.cross(a, b)
        tot += theta * (n @ (c / np.linalg.norm(c)))
    return 0.5 * Le * abs(tot)


@pytest.mark.parametrize("nee", [1, 0])
def test_plane_under_triangle_area_light(nee):
    """Plane under a one-sided triangular emitter: the mean radiance matches
    (a / pi) times the polygon irradiance within 4 standard errors, both for
    next-event estimation and, with NEE off, for cosine-weighted bounces that
    find the emitter (which pins the direction sampling)."""
    a, Le = 0.6, 4.0
    sc = scenes.plane_area_light(a, Le, 8, 8)
    xyz = sc.xyz.astype(np.float64)
    light = xyz[sc.tri_idx[2]]
    e, d = _pinhole_rays(sc)
    p = oracle.make_params(jitter=0, max_depth=1 if nee else 2, nee=nee, spp_init=8,
                           spp_batch=8, spp_max=8)
    n_samples = 20000 if nee else 200000
    checked = 0
    with oracle.Frame(sc, 0, 0) as f:
        for px in (9, 18, 27, 36, 45, 54, 21, 42):
            t = -e[1] / d[px, 1]
            x = e + t * d[px]
            # skip pixels whose camera ray meets the emitter first
            hit, _, prim = f.closest_hit(0, e.astype(np.float32), d[px].astype(np.float32))
            if prim == 2:
                continue
            expect = a / math.pi * _polygon_irradiance(x, np.array([0, 1.0, 0]), light, Le)
            L = _all_paths(f, p, [px], n_samples)[0].astype(np.float64)
            se = L.std(ddof=1) / math.sqrt(len(L))
            assert abs(L.mean() - expect) < 4 * se, (px, L.mean(), expect, se)
            checked += 1
    assert checked >= 6


def test_empty_scene_is_black():
    sc = scenes.empty(6, 5)
    p = oracle.make_params(spp_init=8, spp_batch=8, spp_max=64, C=0.2)
    with oracle.Frame(sc, 0, 1) as f:
        L = _all_paths(f, p, range(30), 16)
        r = f.render(p)
    assert (L == 0).all()
    assert (r["n_paths"] == 8).all() and (r["polarity"] == 0).all()
    np.testing.assert_array_equal(r["mean"], math.log(1e-4))


def test_emitter_is_one_sided():
    """Looking at the back of an emitter (albedo 0) gives zero radiance."""
    b = scenes.SceneBuilder()
    m = b.material(0.0, 3.0)
    v, t = scenes.oriented_quad([(-5, -5, -2), (5, -5, -2), (5, 5, -2), (-5, 5, -2)], (0, 0, 1))
    b.static(b.mesh(v, t, m))
    b.set_camera(4, 4, 30, [0.0], [[0, 0, 0, 0, 0, -1, 0, 1, 0]])
    front = b.build()
    b2 = scenes.SceneBuilder()
    m = b2.material(0.0, 3.0)
    v, t = scenes.oriented_quad([(-5, -5, -2), (5, -5, -2), (5, 5, -2), (-5, 5, -2)], (0, 0, -1))
    b2.static(b2.mesh(v, t, m))
    b2.set_camera(4, 4, 30, [0.0], [[0, 0, 0, 0, 0, -1, 0, 1, 0]])
    back = b2.build()
    p = oracle.make_params()
    with oracle.Frame(front, 0, 0) as f:
        assert (_all_paths(f, p, range(16), 4) == np.float32(3.0)).all()
    with oracle.Frame(back, 0, 0) as f:
        assert (_all_paths(f, p, range(16), 4) == 0).all()


# --------------------------------------------------------------------------
# Multiple importance sampling (power heuristic) of next-event estimation
# and BSDF sampling: unbiased, so the closed forms above hold with it too;
# a wrong light or BSDF pdf would make the two weights not sum to one and
# shift the mean by many standard errors in these scenes, where both
# strategies carry much of the light.

def test_white_furnace_mis_unbiased():
    a, Le, D = 0.6, 1.5, 4
    sc = scenes.furnace(a, Le, 8, 8)
    expect = Le * (1 - a ** (D + 1)) / (1 - a)
    for rr in (2, 99):
        p = oracle.make_params(nee=1, mis=1, max_depth=D, rr_start_depth=rr)
        with oracle.Frame(sc, 0, 0) as f:
            L = _all_paths(f, p, range(64), 512).astype(np.float64).reshape(-1)
        se = L.std(ddof=1) / math.sqrt(len(L))
        assert abs(L.mean() - expect) < 4 * se + 1e-3 * expect, (rr, L.mean(), expect, se)


def _close_quad_light(a=0.6, Le=3.0, h=0.35):
    """Plane y = 0 under a 1.2 x 1.2 emitting quad (two triangles) at height
    h facing down: a large, close light, so that cosine-sampled bounces find
    it as often as light samples do."""
    b = scenes.SceneBuilder()
    m = b.material(a)
    v, t = scenes.oriented_quad([(-50, 0, -50), (50, 0, -50), (50, 0, 50), (-50, 0, 50)], (0, 1, 0))
    b.static(b.mesh(v, t, m))
    lm = b.material(0.0, Le)
    corners = [(-0.6, h, -0.6), (0.6, h, -0.6), (0.6, h, 0.6), (-0.6, h, 0.6)]
    v, t = scenes.oriented_quad(corners, (0, -1, 0))
    b.static(b.mesh(v, t, lm))
    b.set_camera(8, 8, 30.0, [0.0], [[0.0, 2.5, 2.5, 0, 0, 0, 0, 1, 0]])
    return b.build(), np.array(corners, np.float64)


@pytest.mark.parametrize("scene", ["triangle", "close_quad"])
def test_mis_plane_under_area_light(scene):
    """Plane under an area emitter with MIS at depth 2 (light samples at the
    first vertex, cosine-sampled bounces that reach the emitter at the
    second): the mean radiance is (a / pi) times Lambert's polygon
    irradiance within 4 standard errors; per path the estimate differs from
    next-event estimation alone, with the same mean."""
    a, Le = 0.6, (4.0 if scene == "triangle" else 3.0)
    if scene == "triangle":
        sc = scenes.plane_area_light(a, Le, 8, 8)
        poly = sc.xyz.astype(np.float64)[sc.tri_idx[2]]
    else:
        sc, poly = _close_quad_light(a, Le)
    e, d = _pinhole_rays(sc)
    p_mis = oracle.make_params(jitter=0, max_depth=2, nee=1, mis=1, spp_init=8, spp_batch=8, spp_max=8)
    p_nee = oracle.make_params(jitter=0, max_depth=2, nee=1, mis=0, spp_init=8, spp_batch=8, spp_max=8)
    checked = 0
    with oracle.Frame(sc, 0, 0) as f:
        for px in (9, 18, 27, 36, 45, 54, 21, 42):
            t = -e[1] / d[px, 1]
            x = e + t * d[px]
            _, _, prim = f.closest_hit(0, e.astype(np.float32), d[px].astype(np.float32))
            if prim >= 2:
                continue    # the camera ray meets the emitter first
            expect = a / math.pi * _polygon_irradiance(x, np.array([0, 1.0, 0]), poly, Le)
            L = _all_paths(f, p_mis, [px], 40000)[0].astype(np.float64)
            Ln = _all_paths(f, p_nee, [px], 40000)[0].astype(np.float64)
            se = L.std(ddof=1) / math.sqrt(len(L))
            assert abs(L.mean() - expect) < 4 * se, (px, L.mean(), expect, se)
            assert (L != Ln).mean() > 0.05
            checked += 1
    assert checked >= 4
