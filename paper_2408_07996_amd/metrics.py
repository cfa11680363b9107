"""Quality of event maps and event videos as the paper evaluates them
(Sec. 4): the polarity-aware F1 of event pixels, and the RMSE and PSNR of
event frames drawn as images with 0 for a negative event, 0.5 for none and
1 for a positive one (peak value 1).  Videos are scored over all (frame,
pixel) entries together."""
from __future__ import annotations

import math
from typing import Dict

import numpy as np


def polarity_f1(pred, ref) -> float:
    """F1 of event pixels where a predicted event counts as a true positive
    only with the reference's polarity; 1 when neither map has events."""
    p = np.asarray(pred).reshape(-1)
    r = np.asarray(ref).reshape(-1)
    tp = int(((p != 0) & (p == r)).sum())
    fp = int(((p != 0) & (p != r)).sum())
    fn = int(((r != 0) & (p != r)).sum())
    return 1.0 if tp + fp + fn == 0 else 2.0 * tp / (2.0 * tp + fp + fn)


def event_image(polarity) -> np.ndarray:
    """Event map as an image: 0 (negative), 0.5 (none), 1 (positive)."""
    return 0.5 + 0.5 * np.asarray(polarity, dtype=np.float64)


def rmse(pred, ref) -> float:
    d = event_image(pred) - event_image(ref)
    return float(math.sqrt(float(np.mean(d * d)))) if d.size else 0.0


def psnr(pred, ref, peak: float = 1.0) -> float:
    e = rmse(pred, ref)
    return math.inf if e == 0.0 else 20.0 * math.log10(peak / e)


def video_scores(pred, ref) -> Dict[str, float]:
    """F1, RMSE and PSNR of an event video [frames, pixels] against a
    reference video of the same shape."""
    return dict(f1=polarity_f1(pred, ref), rmse=rmse(pred, ref), psnr=psnr(pred, ref))
