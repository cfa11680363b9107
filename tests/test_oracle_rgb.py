"""Pins of the oracle's RGB radiance option: closed forms per channel,
reduced to luminance with the Rec. 709 weights (ITU-R BT.709:
Y = 0.2126 R + 0.7152 G + 0.0722 B), and agreement with grey radiance when
the three channels are equal."""
import math

import numpy as np
import pytest

import oracle
from paper_2408_07996_amd import scenes

W709 = np.array([0.2126, 0.7152, 0.0722])


def _all_paths(f, p, pixels, spp, instant=0):
    px = np.repeat(np.asarray(pixels, np.uint32), spp)
    sm = np.tile(np.arange(spp, dtype=np.uint32), len(pixels))
    return f.paths(p, px, instant, sm).reshape(len(pixels), spp)


def _rgb(sc, albedo_rgb, emission_rgb, pl_rgb=None):
    sc.albedo_rgb = np.asarray(albedo_rgb, np.float32).reshape(-1, 3)
    sc.emission_rgb = np.asarray(emission_rgb, np.float32).reshape(-1, 3)
    sc.pl_rgb = None if pl_rgb is None else np.asarray(pl_rgb, np.float32).reshape(-1, 3)
    return sc


def test_luminance_weights():
    """Y of the primaries and of white (the weights sum to one)."""
    assert oracle.luminance(1, 0, 0) == np.float32(0.2126)
    assert oracle.luminance(0, 1, 0) == np.float32(0.7152)
    assert oracle.luminance(0, 0, 1) == np.float32(0.0722)
    assert abs(oracle.luminance(1, 1, 1) - 1.0) <= 1e-7
    assert abs(oracle.luminance(2.0, 3.0, 4.0) - W709 @ [2.0, 3.0, 4.0]) <= 1e-6


@pytest.mark.parametrize("D", [1, 4, 6])
def test_rgb_furnace_nee_off_is_exact(D):
    """Closed box, walls of albedo a_c and emission Le_c per channel, NEE and
    roulette off: every path carries Le_c (1 - a_c^D) / (1 - a_c) in channel
    c, so its luminance is the weighted sum of the three."""
    a = np.array([0.8, 0.5, 0.2])
    Le = np.array([1.0, 2.5, 4.0])
    sc = _rgb(scenes.furnace(0.5, 1.0, 12, 12), [a], [Le])
    p = oracle.make_params(nee=0, max_depth=D, rr_start_depth=D + 10)
    expect = float(W709 @ (Le * (1 - a ** D) / (1 - a)))
    with oracle.Frame(sc, 0, 0) as f:
        L = _all_paths(f, p, range(144), 512).astype(np.float64)
    exact = np.abs(L - expect) <= 1e-5 * expect
    # As for the grey furnace, every other path left the box through a
    # corner gap after j < D vertices and carries the first j terms.
    partial = np.array([float(W709 @ (Le * (1 - a ** j) / (1 - a))) for j in range(1, D)])
    for v in L[~exact]:
        assert np.abs(partial - v).min() <= 1e-5 * expect, v
    assert (~exact).sum() <= 1e-3 * L.size
    if D == 1:
        assert exact.all()


def test_rgb_furnace_nee_and_roulette_unbiased():
    """With NEE each vertex also gathers a_c Le_c of direct light in channel
    c: E[L] = Y(Le_c (1 - a_c^(D+1)) / (1 - a_c)); roulette (survival
    min(1, largest channel of the throughput), every channel divided by it)
    keeps it unbiased."""
    a = np.array([0.7, 0.4, 0.55])
    Le = np.array([2.0, 1.0, 0.5])
    D = 4
    expect = float(W709 @ (Le * (1 - a ** (D + 1)) / (1 - a)))
    for rr in (2, 99):
        sc = _rgb(scenes.furnace(0.5, 1.0, 8, 8), [a], [Le])
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


@pytest.mark.parametrize("grey_light", [False, True])
def test_rgb_plane_under_point_light_exact(grey_light):
    """Plane y = 0 of albedo a_c under a point light of intensity I_c at
    height h: L = Y((a_c / pi) I_c h / r^3), deterministic.  A grey light
    (no per-channel intensity) shines with its intensity in every channel."""
    a = np.array([0.9, 0.3, 0.6])
    I = np.array([5.0, 2.0, 8.0])
    h = 1.5
    sc = scenes.plane_point_light(0.7, 4.0, h, 24, 16)
    if grey_light:
        I = np.full(3, float(sc.pl_intensity[0]))
    _rgb(sc, [a], [[0.0, 0.0, 0.0]], None if grey_light else [I])
    lp = sc.pl_pos[0].astype(np.float64)
    e, d = _pinhole_rays(sc)
    p = oracle.make_params(jitter=0, max_depth=1, spp_init=8, spp_batch=8, spp_max=8)
    n_checked = 0
    with oracle.Frame(sc, 0, 0) as f:
        for px in range(0, sc.width * sc.height, 3):
            if d[px, 1] >= -1e-3:
                continue
            t = -e[1] / d[px, 1]
            x = e + t * d[px]
            if np.abs(x).max() > 20:
                continue
            r = np.linalg.norm(lp - x)
            expect = float(W709 @ (a / math.pi * I * (lp[1] - x[1]) / r ** 3))
            got = float(f.path_radiance(p, px, 0, 0))
            assert abs(got - expect) <= 3e-5 * expect, (px, got, expect)
            n_checked += 1
    assert n_checked > 60


def _polygon_irradiance(x, n, poly, Le):
    g = poly - x
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    tot = 0.0
    for i in range(len(poly)):
        a, b = g[i], g[(i + 1) % len(poly)]
        theta = math.acos(np.clip(a @ b, -1, 1))
        c = np.cross(a, b)
        tot += theta * (n @ (c / np.linalg.norm(c)))
    return 0.5 * Le * abs(tot)


def _two_light_scene(a, Le1, Le2):
    b = scenes.SceneBuilder()
    m = b.material(0.5)
    v, t = scenes.oriented_quad([(-50, 0, -50), (50, 0, -50), (50, 0, 50), (-50, 0, 50)], (0, 1, 0))
    b.static(b.mesh(v, t, m))
    lights = []
    for k, (x0, lm) in enumerate(((-0.7, b.material(0.0, 1.0)), (0.6, b.material(0.0, 1.0)))):
        tri = np.array([[x0 - 0.4, 1.0 + 0.2 * k, -0.3], [x0 + 0.4, 1.0 + 0.2 * k, -0.2],
                        [x0, 1.0 + 0.2 * k, 0.5]], dtype=np.float64)
        if np.cross(tri[1] - tri[0], tri[2] - tri[0])[1] > 0:
            tri = tri[[0, 2, 1]]
        b.static(b.mesh(tri.astype(np.float32), np.array([[0, 1, 2]]), lm))
        lights.append(tri)
    b.set_camera(8, 8, 30.0, [0.0], [[0.0, 2.5, 2.5, 0, 0, 0, 0, 1, 0]])
    sc = b.build()
    _rgb(sc, [a, [0, 0, 0], [0, 0, 0]], [[0, 0, 0], Le1, Le2])
    return sc, lights


def test_rgb_two_coloured_area_lights():
    """Plane under two triangular emitters of different colour: with the
    emitter picked in proportion to A_j Y(Le_j) and the estimate weighted
    to match, the mean of next-event estimates is
    sum_j Y((a_c / pi) E_j,c), E_j,c the polygon irradiance of emitter j in
    channel c (within 4 standard errors)."""
    a = np.array([0.8, 0.5, 0.3])
    Le1 = np.array([6.0, 1.0, 0.5])
    Le2 = np.array([0.5, 2.0, 9.0])
    sc, lights = _two_light_scene(a, Le1, Le2)
    e, d = _pinhole_rays(sc)
    p = oracle.make_params(jitter=0, max_depth=1, nee=1, spp_init=8, spp_batch=8, spp_max=8)
    checked = 0
    with oracle.Frame(sc, 0, 0) as f:
        for px in (9, 18, 27, 36, 45, 54, 21, 42):
            hit, _, prim = f.closest_hit(0, e.astype(np.float32), d[px].astype(np.float32))
            if not hit or prim >= 2:
                continue
            t = -e[1] / d[px, 1]
            x = e + t * d[px]
            n = np.array([0, 1.0, 0])
            E = np.array([[_polygon_irradiance(x, n, L, 1.0) * c for c in Le] for L, Le in
                          zip(lights, (Le1, Le2))])
            expect = float(sum(W709 @ (a / math.pi * E[j]) for j in range(2)))
            L = _all_paths(f, p, [px], 40000)[0].astype(np.float64)
            se = L.std(ddof=1) / math.sqrt(len(L))
            assert abs(L.mean() - expect) < 4 * se, (px, L.mean(), expect, se)
            checked += 1
    assert checked >= 6


@pytest.mark.parametrize("mis", [0, 1])
def test_rgb_equal_channels_match_grey(mis):
    """RGB with the three channels equal to the grey values follows the grey
    paths: every path's luminance agrees with its grey radiance to a few
    FP32 roundings (the luminance weights sum to one)."""
    sc = scenes.tiny_box(width=16, height=12)
    rgb = _rgb(scenes.tiny_box(width=16, height=12),
               np.repeat(np.asarray(sc.albedo, np.float32)[:, None], 3, 1),
               np.repeat(np.asarray(sc.emission, np.float32)[:, None], 3, 1))
    p = oracle.make_params(max_depth=5, rr_start_depth=2, mis=mis)
    with oracle.Frame(sc, 0, 1) as f, oracle.Frame(rgb, 0, 1) as g:
        for inst in (0, 1):
            Lg = _all_paths(f, p, range(0, 192, 5), 16, inst).astype(np.float64)
            Lc = _all_paths(g, p, range(0, 192, 5), 16, inst).astype(np.float64)
            assert (Lg > 0).mean() > 0.2
            np.testing.assert_allclose(Lc, Lg, rtol=2e-6, atol=1e-30)


def test_rgb_gradient_refused():
    sc = scenes.colorize(scenes.tiny_box(width=8, height=8), seed=1)
    with oracle.Frame(sc, 0, 1) as f:
        with pytest.raises(Exception):
            f.event_loss(oracle.make_params(), 0.2, 0.05, 16)


def test_rgb_roulette_survival_is_largest_channel():
    """Furnace, NEE off, depth 3, roulette from vertex 2: a path adds Y(Le)
    and Y(a * Le), then survives with probability q = min(1, max_c a_c)
    and adds Y(a^2 * Le) / q.  So the paths take two values, the larger
    one for a fraction q of them (the rule, not only the mean, is pinned:
    any q gives the same expectation)."""
    a = np.array([0.9, 0.15, 0.05])
    Le = np.array([1.0, 2.0, 3.0])
    q = float(a.max())
    sc = _rgb(scenes.furnace(0.5, 1.0, 8, 8), [a], [Le])
    p = oracle.make_params(nee=0, max_depth=3, rr_start_depth=2)
    low = float(W709 @ Le + W709 @ (a * Le))
    high = low + float(W709 @ (a * a * Le)) / q
    with oracle.Frame(sc, 0, 0) as f:
        L = _all_paths(f, p, range(64), 128).astype(np.float64).reshape(-1)
    is_low = np.abs(L - low) <= 1e-5 * low
    is_high = np.abs(L - high) <= 1e-5 * high
    # Any other path left the box through a corner gap after its first
    # vertex and carries Y(Le) alone (about 1e-4 of the paths).
    gap = np.abs(L - float(W709 @ Le)) <= 1e-5 * low
    assert (is_low | is_high | gap).all()
    assert gap.sum() <= 1e-3 * len(L)
    frac = is_high.sum() / (is_low | is_high).sum()
    assert abs(frac - q) < 4 * math.sqrt(q * (1 - q) / len(L)), frac


@pytest.mark.parametrize("D", [1, 2, 5])
def test_rgb_plane_under_uniform_sky_is_exact(D):
    """Plane of albedo a_c under a constant grey environment L0: a camera ray
    that meets the plane bounces into the open sky and carries
    Y(a_c L0) (nothing for D = 1); one that misses carries Y(L0, L0, L0)."""
    a = np.array([0.2, 0.9, 0.5])
    L0 = 2.5
    b = scenes.SceneBuilder()
    m = b.material(0.6)
    v, t = scenes.oriented_quad([(-50, 0, -50), (50, 0, -50), (50, 0, 50), (-50, 0, 50)], (0, 1, 0))
    b.static(b.mesh(v, t, m))
    b.set_camera(16, 12, 50.0, [0.0], [[0, 1.5, 3.0, 0, 0.8, 0, 0, 1, 0]])
    sc = _rgb(b.build(), [a], [[0.0, 0.0, 0.0]])
    sc.env = np.full((6, 4, 4), L0, np.float32)
    p = oracle.make_params(max_depth=D, rr_start_depth=99)
    n_hit = 0
    with oracle.Frame(sc, 0, 0) as f:
        for px in range(sc.width * sc.height):
            o, d = f.camera_ray(p, px, 0, 0)
            hit, _, _ = f.closest_hit(0, o, d)
            L = float(f.path_radiance(p, px, 0, 0))
            expect = (0.0 if D == 1 else float(W709 @ (a * L0))) if hit else L0
            assert abs(L - expect) <= 2e-6 * max(expect, 1e-30), (px, L, expect)
            n_hit += hit
    assert 0 < n_hit < sc.width * sc.height
