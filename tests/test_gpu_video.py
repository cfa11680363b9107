"""Sequential event video on the GPU: the reference carried per pixel and
replaced at events, against the oracle's video and the single-pair renderer."""
import numpy as np
import pytest

import oracle
import paper_2408_07996_amd as ev
from paper_2408_07996_amd import scenes

pytestmark = pytest.mark.gpu

TIMES = [0.0, 0.25, 0.5, 0.75, 1.0]
KEYS = ("polarity", "n_paths", "mean", "var", "t_last", "mean_radiance", "flags")


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


def test_video_matches_oracle(rend):
    P = dict(scenes.TINY_PARAMS)
    sc = scenes.tiny_box(width=24, height=20)
    rend.set_scene(sc)
    g = rend.render_event_video(TIMES, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], _opts(P))
    v = oracle.render_video(sc, TIMES, oracle.make_params(**P))
    # A decision inside the exemption band may go either way and then
    # changes the pixel's reference: compare each pixel up to that frame.
    ok = ~np.logical_or.accumulate(v["near_crit"], axis=0)
    assert ok[-1].mean() > 0.8
    pol = g["polarity"].cpu().numpy()
    npth = g["n_paths"].cpu().numpy()
    mean = g["mean"].cpu().numpy()
    np.testing.assert_array_equal(pol[ok], v["polarity"][ok])
    np.testing.assert_array_equal(npth[ok], v["n_paths"][ok])
    err = np.abs(mean - v["mean"])
    assert (err[ok] <= 1e-4 * np.maximum(1.0, np.abs(v["mean"][ok]))).all()
    assert (pol != 0).any()


def test_first_frame_equals_reference_full_pair(rend):
    P = dict(scenes.TINY_PARAMS)
    sc = scenes.tiny_box(width=20, height=16)
    rend.set_scene(sc)
    g = rend.render_event_video(TIMES[:3], P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"],
                                _opts(P))
    f = rend.render_event_frame(TIMES[0], TIMES[1], P["C"], P["alpha"], P["spp_init"], P["spp_batch"],
                                P["spp_max"], _opts(P, ref_mode=ev.REF_FULL))
    for k in KEYS:
        np.testing.assert_array_equal(g[k][0].cpu().numpy(), f[k].cpu().numpy(), err_msg=k)


def test_reference_carried_on_gpu(rend):
    P = dict(scenes.TINY_PARAMS)
    sc = scenes.tiny_box(width=20, height=16)
    rend.set_scene(sc)
    g = rend.render_event_video(TIMES, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], _opts(P))
    pol = g["polarity"].cpu().numpy()
    mean = g["mean"].cpu().numpy()
    evk = pol != 0
    assert evk[:-1].any()
    for k in range(1, len(TIMES) - 1):
        np.testing.assert_array_equal(mean[k][evk[k - 1], 0], mean[k - 1][evk[k - 1], 1])
        np.testing.assert_array_equal(mean[k][~evk[k - 1], 0], mean[k - 1][~evk[k - 1], 0])
