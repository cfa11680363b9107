"""GPU parity of the event-loss gradient (path-replay adjoint) with the
oracle, finite differences through the autograd function, and the full
differentiation workload."""
import time

import numpy as np
import pytest

import oracle
import paper_2408_07996_amd as ev
from paper_2408_07996_amd import scenes

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _opts(P):
    o = dict(seed=P.get("seed", 0), max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
             minibatch=P["minibatch"], log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"])
    for k in ("ray_batch", "lds_nodes", "replay_retrace"):
        if k in P:
            o[k] = P[k]
    return o


def _oracle_params(P):
    return oracle.make_params(seed=P.get("seed", 0), max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
                              minibatch=P["minibatch"], log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"])


def _compare(sc, P, t0=0.0, t1=1.0, threads=0):
    rend = ev.Renderer(0)
    rend.set_scene(sc)
    _say(f"gpu event loss {sc.width}x{sc.height} spp {P['spp']}")
    t = time.time()
    g = rend.event_loss_grad(t0, t1, P["C"], P["tau"], P["spp"], _opts(P), per_pixel=True)
    gl = float(g["loss"].cpu()[0])
    _say(f"  gpu {time.time() - t:.2f}s loss {gl:.6f} mismatch {int(g['replay_mismatch'].cpu()[0])}")
    t = time.time()
    # The ABI takes C and tau in FP32: the oracle gets the same values.
    C32, tau32 = float(np.float32(P["C"])), float(np.float32(P["tau"]))
    with oracle.Frame(sc, t0, t1) as f:
        r = f.event_loss(_oracle_params(P), C32, tau32, P["spp"], threads=threads)
    _say(f"  oracle {time.time() - t:.2f}s loss {r['loss']:.6f}")
    assert int(g["replay_mismatch"].cpu()[0]) == 0
    np.testing.assert_allclose(g["delta"].cpu().numpy(), r["delta"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(g["loss_px"].cpu().numpy(), r["loss_px"], rtol=1e-12, atol=1e-14)
    assert gl == pytest.approx(r["loss"], rel=1e-12)
    for k in ("grad_albedo", "grad_emission"):
        a = g[k].cpu().numpy()
        b = r[k]
        scale = max(np.abs(b).max(), 1e-300)
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * scale, err_msg=k)
    return g, r


def test_event_loss_gradient_matches_oracle_small():
    P = dict(scenes.DIFF_PARAMS, spp=32)
    g, r = _compare(scenes.diff_scene(width=32, height=24), P)
    assert np.abs(r["grad_albedo"]).max() > 0 and np.abs(r["grad_emission"]).max() > 0


@pytest.mark.parametrize("variant", ["pieces", "lds_treelet", "no_nee", "retrace"])
def test_event_loss_gradient_variants(variant):
    """The replay in several pieces per pass (small ray batch: the shadow
    entries' weights and the ray log are per piece), with the LDS treelet
    (closest hits logged, shadow rays traced again), without next-event
    estimation (emission differentiated at every hit), and with every ray
    of the replay traced again instead of read from the log."""
    P = dict(scenes.DIFF_PARAMS, spp=32)
    if variant == "pieces":
        P["ray_batch"] = 4096
    elif variant == "lds_treelet":
        P["lds_nodes"] = 32
    elif variant == "retrace":
        P["replay_retrace"] = 1
    else:
        P["nee"] = 0
    g, r = _compare(scenes.diff_scene(width=24, height=20), P)
    assert np.abs(r["grad_emission"]).max() > 0


def test_event_loss_gradient_matches_oracle_point_lights_mb8():
    sc = scenes.tiny_box(width=20, height=16)
    import dataclasses
    sc = dataclasses.replace(sc, pl_pos=np.array([[0.4, 1.6, 0.3], [-0.5, 1.2, 0.6]], np.float32),
                             pl_intensity=np.array([4.0, 2.0], np.float32))
    P = dict(scenes.DIFF_PARAMS, spp=64, minibatch=8, max_depth=5)
    _compare(sc, P)


def test_event_loss_gradient_many_point_lights():
    # 40 point lights: 41 shadow slots per vertex, more than a visibility
    # mask holds, so the replay reads the logged closest hits and traces its
    # shadow rays again.
    sc = scenes.tiny_box(width=16, height=12)
    import dataclasses
    rng = np.random.default_rng(5)
    pos = np.stack([rng.uniform(-0.8, 0.8, 40), rng.uniform(0.6, 1.8, 40), rng.uniform(-0.8, 0.8, 40)], 1)
    sc = dataclasses.replace(sc, pl_pos=pos.astype(np.float32),
                             pl_intensity=rng.uniform(0.05, 0.2, 40).astype(np.float32))
    P = dict(scenes.DIFF_PARAMS, spp=16, max_depth=3)
    _compare(sc, P)


def test_autograd_matches_central_differences():
    import torch
    sc = scenes.tiny_box(width=16, height=12)
    P = dict(scenes.DIFF_PARAMS, spp=32, max_depth=3, rr_start_depth=99)
    rend = ev.Renderer(0)
    rend.set_scene(sc)
    a = torch.tensor(np.asarray(sc.albedo), dtype=torch.float64, requires_grad=True)
    e = torch.tensor(np.asarray(sc.emission), dtype=torch.float64, requires_grad=True)
    loss = ev.event_loss(rend, a, e, 0.0, 1.0, P["C"], P["tau"], P["spp"], _opts(P))
    loss.backward()
    ga = a.grad.numpy()
    scale = np.abs(ga).max()
    assert scale > 0
    base_a = np.asarray(sc.albedo, np.float32)
    for m in np.nonzero(base_a > 0)[0][:3]:
        vals = []
        for sgn in (1, -1):
            aa = base_a.copy()
            aa[m] = np.float32(aa[m] + sgn * 1e-3)
            vals.append((float(aa[m]), float(ev.event_loss(rend, torch.tensor(aa, dtype=torch.float64),
                                                            torch.tensor(np.asarray(sc.emission)), 0.0, 1.0,
                                                            P["C"], P["tau"], P["spp"], _opts(P)))))
        fd = (vals[0][1] - vals[1][1]) / (vals[0][0] - vals[1][0])
        assert ga[m] == pytest.approx(fd, rel=1e-2, abs=1e-3 * scale), m


@pytest.mark.parametrize("variant", ["default", "retrace"])
def test_delta_vjp_matches_oracle(variant):
    """The product through the per-pixel log-luminance difference with
    seeded weights g: Delta, sum g Delta and its gradient against the
    oracle's; Delta alone (no replay) equal to it."""
    import torch
    sc = scenes.diff_scene(width=32, height=24)
    P = dict(scenes.DIFF_PARAMS, spp=32)
    if variant == "retrace":
        P["replay_retrace"] = 1
    rend = ev.Renderer(0)
    rend.set_scene(sc)
    g = np.random.default_rng(9).normal(size=sc.width * sc.height)
    _say(f"gpu delta vjp {variant}")
    r = rend.delta_vjp(0.0, 1.0, P["spp"], torch.tensor(g), _opts(P))
    d_only = rend.delta_vjp(0.0, 1.0, P["spp"], None, _opts(P))["delta"].cpu().numpy()
    with oracle.Frame(sc, 0.0, 1.0) as f:
        o = f.delta_vjp(_oracle_params(P), P["spp"], g)
    assert int(r["replay_mismatch"].cpu()[0]) == 0
    np.testing.assert_allclose(r["delta"].cpu().numpy(), o["delta"], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(d_only, r["delta"].cpu().numpy())
    assert float(r["value"].cpu()[0]) == pytest.approx(o["value"], rel=1e-10, abs=1e-12)
    for k in ("grad_albedo", "grad_emission"):
        a, b = r[k].cpu().numpy(), o[k]
        scale = max(np.abs(b).max(), 1e-300)
        assert scale > 1e-300
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * scale, err_msg=k)


def test_log_luminance_delta_autograd():
    """log_luminance_delta through torch.autograd: the gradient of a
    quadratic function of Delta equals the library's product with its
    derivative 2 Delta, and the first entries against central differences
    of the function (roulette off)."""
    import torch
    sc = scenes.tiny_box(width=16, height=12)
    P = dict(scenes.DIFF_PARAMS, spp=32, max_depth=3, rr_start_depth=99)
    rend = ev.Renderer(0)
    rend.set_scene(sc)
    a = torch.tensor(np.asarray(sc.albedo), dtype=torch.float64, requires_grad=True)
    e = torch.tensor(np.asarray(sc.emission), dtype=torch.float64, requires_grad=True)
    d = ev.log_luminance_delta(rend, a, e, 0.0, 1.0, P["spp"], _opts(P))
    (d * d).sum().backward()
    r = rend.delta_vjp(0.0, 1.0, P["spp"], 2.0 * d.detach(), _opts(P))
    np.testing.assert_allclose(a.grad.numpy(), r["grad_albedo"].cpu().numpy(), rtol=1e-12)
    np.testing.assert_allclose(e.grad.numpy(), r["grad_emission"].cpu().numpy(), rtol=1e-12)
    ga = a.grad.numpy()
    scale = np.abs(ga).max()
    assert scale > 0
    base_a = np.asarray(sc.albedo, np.float32)
    for m in np.nonzero(base_a > 0)[0][:3]:
        vals = []
        for sgn in (1, -1):
            aa = base_a.copy()
            aa[m] = np.float32(aa[m] + sgn * 1e-3)
            dd = ev.log_luminance_delta(rend, torch.tensor(aa, dtype=torch.float64),
                                        torch.tensor(np.asarray(sc.emission)), 0.0, 1.0, P["spp"], _opts(P))
            vals.append((float(aa[m]), float((dd * dd).sum())))
        fd = (vals[0][1] - vals[1][1]) / (vals[0][0] - vals[1][0])
        assert ga[m] == pytest.approx(fd, rel=1e-2, abs=1e-3 * scale), m


@pytest.mark.slow
def test_event_loss_gradient_full_workload():
    # 256x256, 9,648 triangles, 32 albedos, 4 emitters, 256 paths per pixel
    # and instant: the GPU gradient against the oracle's full-image gradient.
    _compare(scenes.diff_scene(), dict(scenes.DIFF_PARAMS), threads=16)


def test_material_update_builds_nothing_and_matches_a_fresh_scene():
    """A material-only update (each step of an optimization through the
    autograd function) keeps the cached geometry and BVHs: the next gradient
    builds nothing (ms_build == 0) and equals the gradient of a renderer
    given the new materials from scratch (per-pixel terms and frames bit for
    bit, sums over blocks to rounding).  The update changes
    the set of emitters too (a sphere material starts emitting)."""
    import dataclasses
    import torch
    sc = scenes.diff_scene(width=48, height=40)
    P = dict(scenes.DIFF_PARAMS, spp=32)
    rend = ev.Renderer(0)
    rend.set_scene(sc)
    rend.event_loss_grad(0.0, 1.0, P["C"], P["tau"], P["spp"], _opts(P))
    assert rend.frame_stats()["ms_build"] > 0.0
    rng = np.random.default_rng(3)
    alb = np.asarray(sc.albedo, np.float32).copy()
    emi = np.asarray(sc.emission, np.float32).copy()
    lit = alb > 0
    alb[lit] = np.clip(alb[lit] * rng.uniform(0.8, 1.2, lit.sum()), 0.05, 0.95).astype(np.float32)
    emi[emi > 0] = (emi[emi > 0] * rng.uniform(0.5, 2.0, (emi > 0).sum())).astype(np.float32)
    emi[20] = np.float32(2.5)   # a sphere material becomes an emitter
    for step in range(2):
        rend.set_materials(alb, emi)
        g1 = rend.event_loss_grad(0.0, 1.0, P["C"], P["tau"], P["spp"], _opts(P), per_pixel=True)
        assert rend.frame_stats()["ms_build"] == 0.0
        f1 = rend.render_event_frame(0.0, 1.0, 0.2, 0.01, 16, 16, 128, _opts(P))
        assert rend.frame_stats()["ms_build"] == 0.0
        fresh = ev.Renderer(0)
        fresh.set_scene(dataclasses.replace(sc, albedo=alb.copy(), emission=emi.copy()))
        g2 = fresh.event_loss_grad(0.0, 1.0, P["C"], P["tau"], P["spp"], _opts(P), per_pixel=True)
        f2 = fresh.render_event_frame(0.0, 1.0, 0.2, 0.01, 16, 16, 128, _opts(P))
        fresh.close()
        # Per-pixel terms bit for bit; the sums over blocks (FP64 atomics,
        # any order) to rounding.
        for k in ("loss_px", "delta"):
            assert torch.equal(g1[k], g2[k]), (step, k)
        for k in ("loss", "grad_albedo", "grad_emission"):
            a, b = g1[k].cpu().numpy(), g2[k].cpu().numpy()
            np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max(), err_msg=f"{step} {k}")
        for k in f1:
            assert torch.equal(f1[k], f2[k]), (step, k)
        emi = emi.copy()
        emi[20] = np.float32(0.0)  # and back: the emitter set shrinks again
    rend.close()


def test_gradient_refuses_mis():
    """The gradient follows the estimator without MIS: asking for MIS is
    refused before any device work."""
    sc = scenes.diff_scene(width=16, height=12)
    rend = ev.Renderer(0)
    rend.set_scene(sc)
    P = dict(scenes.DIFF_PARAMS, spp=8)
    with pytest.raises(ev.EvrtError) as e:
        rend.event_loss_grad(0.0, 1.0, P["C"], P["tau"], P["spp"], dict(_opts(P), mis=1))
    assert e.value.code == ev.EVRT_E_UNSUPPORTED
    rend.close()
