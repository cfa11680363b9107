"""Launch-shape autotuner: paths in flight per wavefront piece (the depth of
the ray queues) and traversal blocks per CU (the waves each CU keeps in
flight), chosen by timing calibration frames of the caller's scene.

The calibration frame is a FIXED-mode frame over the whole image, which has
the ray mix of a real frame (every bounce, shadow rays) at a fraction of its
cost.  Its path count is at least four batches of the largest paths in
flight tried, so that every shape runs whole pieces in steady state rather
than one launch tail (with a single round of ~60 M paths the timings of the
shapes differ by less than their noise).  Results do not depend on the
chosen shape: every (pixel, sample) is keyed, so only the time changes.
"""
from __future__ import annotations

import itertools
import time
from typing import Dict, Iterable, Optional, Sequence

DEFAULT_RAY_BATCH = (1 << 24, 1 << 25, 1 << 26)
DEFAULT_BLOCKS_PER_CU = (4, 6, 8)
TIE = 0.02  # relative timing difference below which two shapes count as equal


def calibration_spp(width: int, height: int, ray_batch: Sequence[int] = DEFAULT_RAY_BATCH,
                    minibatch: int = 4, lo: int = 32, hi: int = 512) -> int:
    """Paths per pixel and instant of the calibration frame: enough for four
    batches of the largest paths in flight, within [lo, hi], a multiple of
    the mini-batch."""
    need = -(-4 * max(ray_batch) // (2 * width * height))
    spp = min(hi, max(lo, need))
    return max(2 * minibatch, -(-spp // minibatch) * minibatch)


def autotune(renderer, t0: float, t1: float, opts: Optional[Dict] = None, spp: Optional[int] = None,
             ray_batch: Sequence[int] = DEFAULT_RAY_BATCH,
             blocks_per_cu: Sequence[int] = DEFAULT_BLOCKS_PER_CU, repeats: int = 2) -> Dict:
    """Times every (ray_batch, trace_blocks_per_cu) on a FIXED frame of spp
    paths per pixel and instant (default: calibration_spp of the renderer's
    scene) and returns {"opts": best options (dict), "table": [(ray_batch,
    blocks, seconds)], "best_s": seconds, "spp": spp}."""
    import torch
    import paper_2408_07996_amd as ev
    base = dict(opts or {})
    base["mode"] = ev.MODE_FIXED
    mb = base.get("minibatch", 4)
    if spp is None:
        sc = renderer.scene
        spp = calibration_spp(sc.width, sc.height, ray_batch, mb) if sc is not None else 32
    spp = max(2 * mb, spp - spp % mb)
    table = []
    # One untimed frame builds the geometry and the buffers.
    renderer.render_event_frame(t0, t1, 0.1, 0.01, spp, spp, spp, base, extras=False)
    torch.cuda.synchronize()
    for rb, bc in itertools.product(ray_batch, blocks_per_cu):
        o = dict(base, ray_batch=int(rb), trace_blocks_per_cu=int(bc))
        renderer.render_event_frame(t0, t1, 0.1, 0.01, spp, spp, spp, o, extras=False)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(repeats):
            t = time.perf_counter()
            renderer.render_event_frame(t0, t1, 0.1, 0.01, spp, spp, spp, o, extras=False)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        table.append((int(rb), int(bc), best))
    # Shapes within TIE of the fastest are not told apart by the calibration
    # (its repeat-to-repeat spread is about 1 %); among them take the most
    # work in flight (larger batches, then more blocks per CU), which the
    # small late rounds of an adaptive render favor.  On the 977k-triangle
    # batch workload 64 M x 4 and 64 M x 8 calibrate within 0.4 % of each
    # other, while 64 pairs take 65.5 / 124.0 s (batch / single-pair loop)
    # at 64 M x 4 and 64.1 / 115.0 s at 64 M x 8.
    fastest = min(r[2] for r in table)
    rb, bc, sec = max((r for r in table if r[2] <= fastest * (1.0 + TIE)), key=lambda r: (r[0], r[1]))
    out = dict(opts or {})
    out.update(ray_batch=rb, trace_blocks_per_cu=bc)
    return dict(opts=out, table=table, best_s=sec, spp=spp)
