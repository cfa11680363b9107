"""Pins of the oracle's sequential event video (Algorithm 1 over frames:
the reference of each pixel is frame 0 at the full count, carried and
replaced only where an event fires)."""
import numpy as np

import oracle
from paper_2408_07996_amd import scenes

TIMES = [0.0, 0.25, 0.5, 0.75, 1.0]


def _video(C=None, **kw):
    sc = scenes.tiny_box(width=16, height=12)
    P = dict(scenes.TINY_PARAMS, **kw)
    if C is not None:
        P["C"] = C
    return sc, P, oracle.render_video(sc, TIMES, oracle.make_params(**P))


def test_first_video_frame_is_the_reference_full_pair():
    sc, P, v = _video()
    with oracle.Frame(sc, TIMES[0], TIMES[1]) as f:
        r = f.render(oracle.make_params(**dict(P, ref_mode=oracle.REF_FULL)))
    for k in ("polarity", "n_paths", "n_paths_ref", "mean", "var", "t_last", "mean_radiance"):
        np.testing.assert_array_equal(v[k][0], r[k], err_msg=k)


def test_reference_is_replaced_only_at_events():
    sc, P, v = _video()
    ev = v["polarity"] != 0
    assert ev[:-1].any(), "the moving cube must fire events"
    for k in range(1, len(TIMES) - 1):
        ref = v["mean"][k][:, 0]
        np.testing.assert_array_equal(ref[ev[k - 1]], v["mean"][k - 1][ev[k - 1], 1])
        np.testing.assert_array_equal(ref[~ev[k - 1]], v["mean"][k - 1][~ev[k - 1], 0])
        np.testing.assert_array_equal(v["var"][k][ev[k - 1], 0], v["var"][k - 1][ev[k - 1], 1])
    # events only at the full count; the reference always holds it
    assert (v["n_paths"][ev] == P["spp_max"]).all()
    assert (v["n_paths_ref"] == P["spp_max"]).all()


def test_no_events_keep_frame_zero_as_reference():
    sc, P, v = _video(C=50.0)
    assert not (v["polarity"] != 0).any()
    for k in range(1, len(TIMES) - 1):
        np.testing.assert_array_equal(v["mean"][k][:, 0], v["mean"][0][:, 0])
