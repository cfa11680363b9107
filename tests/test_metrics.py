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
