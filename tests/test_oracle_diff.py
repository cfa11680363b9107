"""Pins of the oracle's event-loss gradient (path-replay derivative).

Each path's derivative with its sampling decisions held fixed is pinned by
closed forms (white furnace, plane under a point light); the loss's forward
statistics by the already-pinned fixed-count loop; the whole chain through
ln(Y + eps), the mean and the softplus by central finite differences of the
loss with Russian roulette off and one emitter material (so that no sampling
decision depends on the parameters).
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2408_07996_amd import scenes


def test_furnace_path_derivatives_closed_form():
    # NEE off, RR off: every path returns Le * sum_{k<D} a^k exactly.
    a, Le, D = 0.6, 2.0, 5
    sc = scenes.furnace(a, Le, width=4, height=4)
    P = oracle.make_params(max_depth=D, rr_start_depth=99, nee=0)
    with oracle.Frame(sc, 0.0, 0.0) as f:
        for pixel, sample in ((0, 0), (5, 3), (15, 11)):
            L, ga, ge = f.path_gradient(P, pixel, 0, sample)
            a32 = float(np.float32(a))
            assert L == pytest.approx(Le * sum(a32 ** k for k in range(D)), rel=1e-6)
            assert ga[0] == pytest.approx(Le * sum(k * a32 ** (k - 1) for k in range(1, D)), rel=1e-5)
            assert ge[0] == pytest.approx(sum(a32 ** k for k in range(D)), rel=1e-6)


def test_plane_point_light_derivative_is_l_over_a():
    a = 0.7
    sc = scenes.plane_point_light(albedo=a)
    P = oracle.make_params(max_depth=3, jitter=0)
    with oracle.Frame(sc, 0.0, 0.0) as f:
        for pixel in (0, 37, 200, 383):
            L, ga, ge = f.path_gradient(P, pixel, 0, 0)
            assert L > 0
            assert ga[0] == pytest.approx(float(L) / float(np.float32(a)), rel=1e-7)
            assert not ge.any()


def test_emission_derivative_is_homogeneous():
    # Without point lights every term is proportional to one emitted
    # radiance: sum_e Le_e dL/dLe_e = L for every path.
    sc = scenes.diff_scene(width=16, height=16)
    assert (np.asarray(sc.emission) > 0).sum() == 4
    P = oracle.make_params(max_depth=5)
    with oracle.Frame(sc, 0.0, 1.0) as f:
        checked = 0
        for pixel in range(0, 256, 7):
            for inst in (0, 1):
                L, ga, ge = f.path_gradient(P, pixel, inst, pixel % 7)
                s = float(np.dot(np.asarray(sc.emission, np.float64), ge))
                assert s == pytest.approx(float(L), rel=1e-5, abs=1e-7)
                checked += L > 0
        assert checked > 20


def test_loss_statistics_match_fixed_count_loop():
    sc = scenes.tiny_box(width=12, height=10)
    spp = 32
    P = oracle.make_params(spp_init=spp, spp_max=spp, mode=oracle.MODE_FIXED)
    with oracle.Frame(sc, 0.0, 1.0) as f:
        r = f.event_loss(P, 0.2, 0.05, spp)
        fx = f.render(P)
    delta = fx["mean"][:, 1] - fx["mean"][:, 0]
    np.testing.assert_allclose(r["delta"], delta, rtol=0, atol=1e-12)
    z = (np.abs(delta) - 0.2) / 0.05
    np.testing.assert_allclose(r["loss_px"], np.logaddexp(0.0, z), rtol=1e-12)
    assert r["loss"] == pytest.approx(float(np.logaddexp(0.0, z).sum()), rel=1e-12)


def _fd(sc, P, C, tau, spp, field, m, h):
    vals = []
    for sgn in (1, -1):
        arr = np.array(getattr(sc, field), np.float32)
        arr[m] = np.float32(arr[m] + sgn * h)
        vals.append((arr[m], dataclasses.replace(sc, **{field: arr})))
    out = []
    for _, s in vals:
        with oracle.Frame(s, 0.0, 1.0) as f:
            out.append(f.event_loss(P, C, tau, spp)["loss"])
    return (out[0] - out[1]) / (float(vals[0][0]) - float(vals[1][0]))


def test_loss_gradient_matches_central_differences():
    sc = scenes.tiny_box(width=16, height=12)
    P = oracle.make_params(max_depth=3, rr_start_depth=99)
    C, tau, spp = 0.2, 0.05, 32
    with oracle.Frame(sc, 0.0, 1.0) as f:
        g = f.event_loss(P, C, tau, spp)
    emitters = np.nonzero(np.asarray(sc.emission) > 0)[0]
    assert len(emitters) == 1
    scale = np.abs(g["grad_albedo"]).max()
    for m in range(len(sc.albedo)):
        if sc.albedo[m] <= 0:
            continue
        fd = _fd(sc, P, C, tau, spp, "albedo", m, 1e-3)
        assert g["grad_albedo"][m] == pytest.approx(fd, rel=1e-2, abs=1e-3 * scale), m

    # The emission gradient: with one emitter and no other light every path
    # is proportional to Le and Delta depends on Le only through eps, too
    # weakly for FP32 paths; a point light (not a parameter) makes Le shift
    # the balance of the light.
    scp = dataclasses.replace(sc, pl_pos=np.array([[0.4, 1.6, 0.3]], np.float32),
                              pl_intensity=np.array([4.0], np.float32))
    with oracle.Frame(scp, 0.0, 1.0) as f:
        gp = f.event_loss(P, C, tau, spp)
    e = int(emitters[0])
    fd = _fd(scp, P, C, tau, spp, "emission", e, 1e-3)
    assert abs(gp["grad_emission"][e]) > 0.5
    assert gp["grad_emission"][e] == pytest.approx(fd, rel=1e-2)


def test_gradient_matches_central_differences_on_the_diff_workload():
    """The differentiation workload (256x256, 9,648 triangles, 36 materials,
    4 emitters) on every 8th pixel in x and y, Russian roulette off:
    the path-replay gradient of the oracle against central differences of
    its loss with h = 1e-3, for the six albedos with the largest gradient.
    With the roulette off no sampling decision depends on an albedo, so the
    difference quotient at fixed random numbers measures the same
    derivative.  (Emission is checked on a scene with one area emitter: with
    several, the emitter-pick distribution is proportional to area times
    emission, so at fixed random numbers a change of one emission moves
    every pick boundary and switches some paths to another emitter, jumps
    that a difference quotient amplifies by 1 / 2h; the gradient holds
    those decisions fixed.)  The loss
    is computed from FP32 paths and FP64 statistics: rounding of a path is a
    deterministic function of the parameters, and with h = 1e-3 its effect
    on the difference quotient stays far below the 1 % bar (the quotients
    below agree with the gradient to a few 1e-3 relative)."""
    sc = scenes.diff_scene()
    P = oracle.make_params(max_depth=4, rr_start_depth=99)
    C, tau, spp, h = 0.2, 0.05, 64, 1e-3
    px = scenes.subset_every(sc.width, sc.height, 8)

    def loss_of(s):
        with oracle.Frame(s, 0.0, 1.0) as f:
            return f.event_loss(P, C, tau, spp, pixels=px)

    g = loss_of(sc)
    albedo_ids = np.argsort(-np.abs(g["grad_albedo"]))[:6]
    scale = np.abs(g["grad_albedo"]).max()
    for m in albedo_ids:
        vals = []
        for sgn in (1, -1):
            arr = np.array(sc.albedo, np.float32)
            arr[m] = np.float32(arr[m] + sgn * h)
            vals.append((float(arr[m]), loss_of(dataclasses.replace(sc, albedo=arr))["loss"]))
        fd = (vals[0][1] - vals[1][1]) / (vals[0][0] - vals[1][0])
        assert g["grad_albedo"][m] == pytest.approx(fd, rel=1e-2, abs=1e-3 * scale), (m, g["grad_albedo"][m], fd)


def test_delta_vjp_matches_central_differences_and_the_loss_gradient():
    """The vector-Jacobian product through the per-pixel log-luminance
    difference: value = sum_p g_p Delta_p for seeded weights g; its albedo
    gradient against central differences of the value (h = 1e-3, roulette
    off, one emitter), its Delta equal to the loss's Delta, and with g the
    loss's own dL/dDelta it reproduces the loss gradient."""
    sc = scenes.tiny_box(width=16, height=12)
    P = oracle.make_params(max_depth=3, rr_start_depth=99)
    spp = 32
    n = sc.width * sc.height
    g = np.random.default_rng(5).normal(size=n)
    with oracle.Frame(sc, 0.0, 1.0) as f:
        v = f.delta_vjp(P, spp, g)
        lo = f.event_loss(P, 0.2, 0.05, spp)
    np.testing.assert_array_equal(v["delta"], lo["delta"])
    assert v["value"] == pytest.approx(float(np.dot(g, v["delta"])), rel=1e-12)
    scale = np.abs(v["grad_albedo"]).max()
    assert scale > 0
    for m in range(len(sc.albedo)):
        if sc.albedo[m] <= 0:
            continue
        vals = []
        for sgn in (1, -1):
            arr = np.array(sc.albedo, np.float32)
            arr[m] = np.float32(arr[m] + sgn * 1e-3)
            with oracle.Frame(dataclasses.replace(sc, albedo=arr), 0.0, 1.0) as f:
                vals.append((float(arr[m]), f.delta_vjp(P, spp, g)["value"]))
        fd = (vals[0][1] - vals[1][1]) / (vals[0][0] - vals[1][0])
        assert v["grad_albedo"][m] == pytest.approx(fd, rel=1e-2, abs=1e-3 * scale), m
    # The loss's own weights: sigmoid((|Delta| - C) / tau) / tau * sign(Delta).
    d = lo["delta"]
    z = (np.abs(d) - 0.2) / 0.05
    w = 1.0 / (1.0 + np.exp(-z)) / 0.05 * np.sign(d)
    with oracle.Frame(sc, 0.0, 1.0) as f:
        v2 = f.delta_vjp(P, spp, w)
    np.testing.assert_allclose(v2["grad_albedo"], lo["grad_albedo"], rtol=1e-9, atol=1e-12 * scale)
    np.testing.assert_allclose(v2["grad_emission"], lo["grad_emission"], rtol=1e-9,
                               atol=1e-12 * np.abs(lo["grad_emission"]).max())
