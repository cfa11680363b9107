import math

import numpy as np
import pytest

from paper_2408_07996_amd import metrics


def test_identical_maps():
    a = np.array([[1, 0, -1, 0], [0, 0, 1, -1]], np.int8)
    s = metrics.video_scores(a, a)
    assert s["f1"] == 1.0 and s["rmse"] == 0.0 and s["psnr"] == math.inf


def test_no_events_anywhere():
    z = np.zeros(10, np.int8)
    assert metrics.polarity_f1(z, z) == 1.0


def test_f1_counts_wrong_polarity_as_miss_and_false_event():
    ref = np.array([1, 1, -1, 0, 0], np.int8)
    pred = np.array([1, -1, 0, 1, 0], np.int8)
    # tp = 1; false events: the -1 at 1 and the +1 at 3; misses: 1 and 2
    assert metrics.polarity_f1(pred, ref) == pytest.approx(2 * 1 / (2 * 1 + 2 + 2))


def test_rmse_and_psnr_of_single_differences():
    n = 16
    ref = np.zeros(n, np.int8)
    one = ref.copy()
    one[3] = 1          # image differs by 0.5 at one pixel
    assert metrics.rmse(one, ref) == pytest.approx(0.5 / math.sqrt(n))
    assert metrics.psnr(one, ref) == pytest.approx(20 * math.log10(math.sqrt(n) / 0.5))
    flip = ref.copy()
    flip[0], ref2 = -1, ref.copy()
    ref2[0] = 1         # opposite polarity: difference 1
    assert metrics.rmse(flip, ref2) == pytest.approx(1 / math.sqrt(n))


def test_autotune_calibration_spp():
    """The calibration frame holds at least four batches of the largest
    paths in flight (clamped to [32, 512], a multiple of the mini-batch)."""
    from paper_2408_07996_amd.autotune import calibration_spp
    for w, h in ((1280, 720), (640, 480), (37, 23)):
        spp = calibration_spp(w, h)
        assert spp % 4 == 0 and 32 <= spp <= 512
        assert spp == 512 or 2 * w * h * spp >= 4 * (1 << 26)
    assert calibration_spp(1280, 720) == 148
    assert calibration_spp(8, 8, minibatch=8) % 8 == 0


def test_autotune_prefers_more_work_in_flight_on_ties(monkeypatch):
    """Shapes within 2 % of the fastest count as tied; the tie goes to the
    larger batch, then the more blocks per CU.  The fake renderer advances a
    virtual clock that the tuner reads, so the test does not depend on how
    precisely the host sleeps."""
    import types
    import sys

    import paper_2408_07996_amd.autotune as at

    clock = [0.0]

    class FakeRenderer:
        scene = None

        def render_event_frame(self, t0, t1, C, a, s0, s1, s2, o, extras=False):
            clock[0] += times.get((o.get("ray_batch"), o.get("trace_blocks_per_cu")), 0.0)

    times = {(1 << 24, 4): 0.140, (1 << 25, 4): 0.120, (1 << 26, 4): 0.100, (1 << 26, 8): 0.1005,
             (1 << 24, 8): 0.150, (1 << 25, 8): 0.130}
    monkeypatch.setattr(at.time, "perf_counter", lambda: clock[0])
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(synchronize=lambda: None))
    monkeypatch.setitem(sys.modules, "torch", fake_torch)
    r = at.autotune(FakeRenderer(), 0.0, 1.0, {}, spp=32, ray_batch=(1 << 24, 1 << 25, 1 << 26),
                    blocks_per_cu=(4, 8), repeats=2)
    assert (r["opts"]["ray_batch"], r["opts"]["trace_blocks_per_cu"]) == (1 << 26, 8)
    assert [round(t, 4) for _, _, t in r["table"]] == [0.14, 0.15, 0.12, 0.13, 0.1, 0.1005]
    # Outside the tie band the fastest shape wins.
    times[(1 << 26, 8)] = 0.103
    r = at.autotune(FakeRenderer(), 0.0, 1.0, {}, spp=32, ray_batch=(1 << 24, 1 << 25, 1 << 26),
                    blocks_per_cu=(4, 8), repeats=2)
    assert (r["opts"]["ray_batch"], r["opts"]["trace_blocks_per_cu"]) == (1 << 26, 4)
