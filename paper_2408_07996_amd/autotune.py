"""Launch-shape autotuner: paths in flight per wavefront piece (the depth of
the ray queues) and traversal blocks per CU (the waves each CU keeps in
flight), chosen by timing calibration frames of the caller's scene.

The calibration frame is a FIXED-mode frame at a small path count over the
whole image, which has the ray mix of a real frame (every bounce, shadow
rays) at a fraction of its cost.  Results do not depend on the chosen
shape: every (pixel, sample) is keyed, so only the time changes.
"""
from __future__ import annotations

import itertools
import time
from typing import Dict, Iterable, Optional, Sequence

DEFAULT_RAY_BATCH = (1 << 24, 1 << 25, 1 << 26)
DEFAULT_BLOCKS_PER_CU = (4, 6, 8)


def autotune(renderer, t0: float, t1: float, opts: Optional[Dict] = None, spp: int = 32,
             ray_batch: Sequence[int] = DEFAULT_RAY_BATCH,
             blocks_per_cu: Sequence[int] = DEFAULT_BLOCKS_PER_CU, repeats: int = 2) -> Dict:
    """Times every (ray_batch, trace_blocks_per_cu) on a FIXED frame of spp
    paths per pixel and instant and returns {"opts": best options (dict),
    "table": [(ray_batch, blocks, seconds)], "best_s": seconds}."""
    import torch
    import paper_2408_07996_amd as ev
    base = dict(opts or {})
    base["mode"] = ev.MODE_FIXED
    mb = base.get("minibatch", 4)
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
    rb, bc, sec = min(table, key=lambda r: r[2])
    out = dict(opts or {})
    out.update(ray_batch=rb, trace_blocks_per_cu=bc)
    return dict(opts=out, table=table, best_s=sec)
