"""Frame batches: many consecutive pairs in one call, the frame shared by
two pairs sampled once.  Each pair must equal the single-pair renderer with
the batch's frame keys bit for bit, and the oracle within the parity bars."""
import numpy as np
import pytest

import oracle
import paper_2408_07996_amd as ev
from paper_2408_07996_amd import scenes

pytestmark = pytest.mark.gpu

KEYS = ("polarity", "n_paths", "mean", "var", "t_last", "mean_radiance", "flags")


def _say(msg):
    print(msg, flush=True)


def _opts(P, **kw):
    d = dict(seed=P["seed"], max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
             minibatch=P["minibatch"], log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"])
    d.update(kw)
    return d


@pytest.fixture(scope="module")
def rend():
    import torch
    assert torch.cuda.is_available()
    r = ev.Renderer(0)
    yield r
    r.close()


def _batch_vs_pairs(rend, sc, P, times, **kw):
    rend.set_scene(sc)
    o = _opts(P, **kw)
    b = rend.render_event_batch(times, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], o)
    bst = rend.frame_stats()
    paths_batch = bst["camera_rays"]
    paths_pairs = 0
    for k in range(len(times) - 1):
        f = rend.render_event_frame(times[k], times[k + 1], P["C"], P["alpha"], P["spp_init"], P["spp_batch"],
                                    P["spp_max"], dict(o, key_base=o.get("key_base", 0) + k))
        paths_pairs += rend.frame_stats()["camera_rays"]
        for key in KEYS:
            np.testing.assert_array_equal(b[key][k].cpu().numpy(), f[key].cpu().numpy(), err_msg=f"pair {k} {key}")
    return b, paths_batch, paths_pairs


@pytest.mark.parametrize("variant", ["default", "small_pieces", "split_samples", "fixed", "two_tailed", "mb8",
                                     "key_base", "rgb"])
def test_batch_equals_single_pairs(rend, variant):
    P = dict(scenes.TINY_PARAMS)
    kw = {}
    if variant == "small_pieces":
        kw = dict(ray_batch=1 << 14)
    elif variant == "split_samples":
        kw = dict(ray_batch=512)
    elif variant == "fixed":
        kw = dict(mode=ev.MODE_FIXED)
    elif variant == "two_tailed":
        kw = dict(mode=ev.MODE_ADAPTIVE_2T)
    elif variant == "mb8":
        P.update(minibatch=8, spp_init=32, spp_batch=32)
    elif variant == "key_base":
        kw = dict(key_base=300)
    sc = scenes.panning(scenes.tiny_box(width=32, height=24), 5, 2.0)
    if variant == "rgb":
        sc = scenes.colorize(sc, seed=9)
    _say(f"batch variant {variant}")
    b, pb, pp = _batch_vs_pairs(rend, sc, P, [0.0, 1.0, 2.0, 3.0, 4.0], **kw)
    # shared frames are traced once: fewer camera rays than the pairs
    assert pb < pp


def test_batch_matches_oracle(rend):
    P = dict(scenes.TINY_PARAMS)
    sc = scenes.panning(scenes.tiny_box(width=24, height=20), 4, 3.0)
    rend.set_scene(sc)
    times = [0.0, 1.0, 2.0, 3.0]
    b = rend.render_event_batch(times, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], _opts(P))
    for k in range(3):
        with oracle.Frame(sc, times[k], times[k + 1]) as f:
            r = f.render(oracle.make_params(**P, key_base=k))
        ok = ~r["near_crit"]
        _say(f"  pair {k}: {int((~ok).sum())} of {ok.size} pixels exempt")
        assert (~ok).sum() <= 0.01 * ok.size
        np.testing.assert_array_equal(b["polarity"][k].cpu().numpy()[ok], r["polarity"][ok])
        np.testing.assert_array_equal(b["n_paths"][k].cpu().numpy()[ok], r["n_paths"][ok])
        m = b["mean"][k].cpu().numpy()
        assert (np.abs(m - r["mean"]) <= 1e-4 * np.maximum(1.0, np.abs(r["mean"]))).all()


@pytest.mark.slow
def test_batch_workload_subset_matches_oracle(rend):
    """The frame-batch workload at full size (1280x720, 977,290 triangles,
    camera panning 0.5 degrees per frame, 16/16/2048, depth 8): a batch of
    two pairs against the oracle on every 32nd pixel in x and y."""
    P = dict(scenes.BATCH_PARAMS)
    sc = scenes.batch_scene(n_frames=3)
    rend.set_scene(sc)
    times = [0.0, 1.0, 2.0]
    _say("batch workload: 2 pairs at 1280x720")
    b = rend.render_event_batch(times, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], _opts(P))
    px = scenes.subset_every(sc.width, sc.height, 32)
    for k in range(2):
        with oracle.Frame(sc, times[k], times[k + 1]) as f:
            r = f.render(oracle.make_params(**P, key_base=k), px)
        g = {key: b[key][k].cpu().numpy()[px] for key in KEYS}
        ok = ~r["near_crit"]
        _say(f"  pair {k}: {int((~ok).sum())} of {ok.size} pixels exempt, {int((r['polarity'] != 0).sum())} events")
        assert (~ok).sum() <= 0.01 * ok.size
        np.testing.assert_array_equal(g["polarity"][ok], r["polarity"][ok])
        np.testing.assert_array_equal(g["n_paths"][ok], r["n_paths"][ok])
        same = g["n_paths"] == r["n_paths"]
        for key in ("mean", "var", "mean_radiance"):
            err = np.abs(g[key][same] - r[key][same]) / np.maximum(1.0, np.abs(r[key][same]))
            assert err.max(initial=0.0) <= 1e-4, key
        tg, tr = g["t_last"][same], r["t_last"][same]
        fin = np.isfinite(tr)
        assert (tg[~fin] == tr[~fin]).all()
        assert (np.abs(tg[fin] - tr[fin]) <= 1e-4 * np.maximum(1.0, np.abs(tr[fin]))).all()


@pytest.mark.slow
def test_city_batch_subset_matches_oracle(rend):
    """The stress workload at full size (1920x1080, 4.32M triangles, 16
    area lights, 50 moving boxes, moving camera, depth 12, 64/64/4096,
    alpha = 0.001): a batch of two pairs (three frames, each with its own
    geometry) against the oracle on every 96th pixel in x and y."""
    P = dict(scenes.CITY_PARAMS)
    sc = scenes.city(n_frames=3)
    rend.set_scene(sc)
    times = [0.0, 1.0, 2.0]
    _say("city batch: 2 pairs at 1920x1080")
    b = rend.render_event_batch(times, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], _opts(P))
    st = rend.frame_stats()
    _say(f"  gpu rounds {st['rounds']} build {st['ms_build']:.0f} ms wall {st['ms_wall']:.0f} ms")
    px = scenes.subset_every(sc.width, sc.height, 96)
    for k in range(2):
        with oracle.Frame(sc, times[k], times[k + 1]) as f:
            r = f.render(oracle.make_params(**P, key_base=k), px)
        g = {key: b[key][k].cpu().numpy()[px] for key in KEYS}
        ok = ~r["near_crit"]
        _say(f"  pair {k}: {int((~ok).sum())} of {ok.size} exempt, {int((r['polarity'] != 0).sum())} events, "
             f"{r['n_paths'].mean():.0f} paths per pixel")
        assert (~ok).sum() <= 0.01 * ok.size
        np.testing.assert_array_equal(g["polarity"][ok], r["polarity"][ok])
        np.testing.assert_array_equal(g["n_paths"][ok], r["n_paths"][ok])
        same = g["n_paths"] == r["n_paths"]
        for key in ("mean", "var", "mean_radiance"):
            err = np.abs(g[key][same] - r[key][same]) / np.maximum(1.0, np.abs(r[key][same]))
            assert err.max(initial=0.0) <= 1e-4, key


def test_single_frame_key_base_matches_oracle(rend):
    P = dict(scenes.TINY_PARAMS)
    sc = scenes.tiny_box(width=24, height=20)
    rend.set_scene(sc)
    g = rend.render_event_frame(0.0, 1.0, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"],
                                _opts(P, key_base=257))
    with oracle.Frame(sc, 0.0, 1.0) as f:
        r = f.render(oracle.make_params(**P, key_base=257))
        r0 = f.render(oracle.make_params(**P))
    ok = ~r["near_crit"]
    np.testing.assert_array_equal(g["n_paths"].cpu().numpy()[ok], r["n_paths"][ok])
    m = g["mean"].cpu().numpy()
    assert (np.abs(m - r["mean"]) <= 1e-4 * np.maximum(1.0, np.abs(r["mean"]))).all()
    assert not np.array_equal(r["mean"], r0["mean"])


@pytest.mark.parametrize("variant", ["default", "small_pieces", "split_samples", "two_tailed", "fixed"])
def test_moving_batch_equals_single_pairs(rend, variant):
    """Geometry and camera both change every frame: each frame's items are
    traced with its own instant, and every pair equals the single-pair
    renderer with the batch's keys, bit for bit."""
    P = dict(scenes.TINY_PARAMS)
    kw = {}
    if variant == "small_pieces":
        kw = dict(ray_batch=1 << 14)
    elif variant == "split_samples":
        kw = dict(ray_batch=512)
    elif variant == "two_tailed":
        kw = dict(mode=ev.MODE_ADAPTIVE_2T)
    elif variant == "fixed":
        kw = dict(mode=ev.MODE_FIXED)
    sc = scenes.moving_panning(32, 24, 5)
    _say(f"moving batch variant {variant}")
    b, pb, pp = _batch_vs_pairs(rend, sc, P, [0.0, 1.0, 2.0, 3.0, 4.0], **kw)
    assert pb < pp
    assert rend.frame_stats()["rounds"] >= 1


@pytest.mark.parametrize("rgb", [False, True])
def test_moving_batch_matches_oracle(rend, rgb):
    P = dict(scenes.TINY_PARAMS)
    sc = scenes.moving_panning(24, 20, 4)
    if rgb:
        sc = scenes.colorize(sc, seed=11)
    rend.set_scene(sc)
    times = [0.0, 1.0, 2.0, 3.0]
    b = rend.render_event_batch(times, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], _opts(P))
    for k in range(3):
        with oracle.Frame(sc, times[k], times[k + 1]) as f:
            r = f.render(oracle.make_params(**P, key_base=k))
        ok = ~r["near_crit"]
        _say(f"  pair {k}: {int((~ok).sum())} of {ok.size} pixels exempt")
        assert (~ok).sum() <= 0.01 * ok.size
        np.testing.assert_array_equal(b["polarity"][k].cpu().numpy()[ok], r["polarity"][ok])
        np.testing.assert_array_equal(b["n_paths"][k].cpu().numpy()[ok], r["n_paths"][ok])
        m = b["mean"][k].cpu().numpy()
        assert (np.abs(m - r["mean"]) <= 1e-4 * np.maximum(1.0, np.abs(r["mean"]))).all()
        assert (r["polarity"] != 0).any()


def test_batch_rejects_ref_full_and_normality(rend):
    P = dict(scenes.TINY_PARAMS)
    rend.set_scene(scenes.panning(scenes.tiny_box(width=8, height=8), 3, 1.0))
    with pytest.raises(ev.EvrtError) as e:
        rend.render_event_batch([0.0, 1.0, 2.0], P["C"], P["alpha"], 16, 16, 64,
                                _opts(P, ref_mode=ev.REF_FULL))
    assert e.value.code == ev.EVRT_E_UNSUPPORTED
    with pytest.raises(ev.EvrtError) as e:
        rend.render_event_batch([0.0, 1.0, 2.0], P["C"], P["alpha"], 16, 16, 64,
                                _opts(P, normality_alpha=0.05))
    assert e.value.code == ev.EVRT_E_UNSUPPORTED
