"""Benchmark of the adaptive event renderer on one MI355X.

A step is one event frame of the sensor workload (640x480, ~98k
triangles, 20 rigidly moving icospheres on a displaced floor, 3 area
lights, max depth 8, schedule 64 + 16k up to 1024 paths per instant,
C = 0.15, alpha = 0.01): every pixel path traced at t0 = 0 and t1 = 1 until
the one-tailed t-test stops it or it reaches 1024 paths, then the event
rule.  Prints one JSON line.

Reported next to the headline (event frames/s):
  * rays/s (camera + extension + shadow rays counted on the device);
  * the same library in FIXED mode at 1024 paths (the paper's baseline) and
    the speed-up over it; the speed-up over the cheapest fixed count whose
    event map has at least the adaptive map's polarity F1 against a
    4096-path reference;
  * roofline of the dominant kernel (closest-hit BVH traversal): FP32
    lane-operations of its box and triangle tests per launch over the
    launch time measured with HIP events on the render stream;
  * the CPU oracle timed on a bounded pixel sample.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# FP32 VALU lane-operations of the intended math per unit of traversal work
# (counted from the kernel's gfx950 ISA for the box and triangle tests).
OPS_PER_NODE = 62.0   # 4-wide node: four slab tests (6 FMA, 6 min/max, 1 compare each) + 4-key sort (10)
OPS_PER_TRI = 52.0    # watertight test: translate, permute, shear, 3 edge functions, signs
# Peak FP32 VALU issue of MI355X without packed math: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz.
PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9

# From rocprofv3 counter passes over one frame of this workload (summaries
# in profiles/): HBM bytes per closest-hit launch (FETCH_SIZE and WRITE_SIZE
# summed over the frame's launches, scaled by what the same counters read
# for a 256 MiB device copy, x1.9997 and x1.0000, divided by the launches),
# and the VALU busy fraction (SQ_ACTIVE_INST_VALU x 4 cycles over 1024 SIMDs
# and the dispatches' GRBM_GUI_ACTIVE, which sums the 8 XCDs) and VALU lane
# utilization (SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU)) of the
# traversal kernels.  They hold for the kernel sources and build flags they
# were taken with and are reported as null for any others.
TRAFFIC = {"sources_sha256": "05cdcfa7b1ef8436525e1bb15435d32d097feb3725fd1b84c2c38949a92ff974",
           "bytes_per_launch": 526307510.5,
           "counters": {"k_trace_closest": {"valu_busy": 0.874, "valu_lane_utilization": 0.601}, "k_trace_shadow": {"valu_busy": 0.713, "valu_lane_utilization": 0.602}, "k_shade": {"valu_busy": 0.504, "valu_lane_utilization": 0.634}}}


def kernel_sources_digest() -> str:
    """Digest of the kernel sources and of the build script (its compiler
    flags change the kernels too)."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2408_07996_amd", "csrc", "*")))
    for f in files + [os.path.join(ROOT, "paper_2408_07996_amd", "build.py")]:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


from paper_2408_07996_amd.metrics import polarity_f1, video_scores  # noqa: E402

# The paper's own per-frame figure (Table 2, "Cup of water" row; also the
# teaser): 200x200 pixels, up to 4096 paths per pixel, on the hardware the
# paper lists.  Context only: another scene, machine and renderer.
PAPER_CONTEXT = {"scene": "Cup of water, 200x200 pixels, up to 4096 paths per pixel, one-tailed test alpha 0.05",
                 "s_per_frame_fixed_4096": 40.81, "s_per_frame_adaptive": 4.55, "speedup": 8.98,
                 "hardware": "Intel Core i9-13900K (24 cores) + NVIDIA RTX A6000, 128 GB RAM; the paper does "
                             "not say which device ran its pbrt-v4-based renderer",
                 "source": "Table 2"}

# Host CPUs one GPU's share of the benchmark box may use for worker pools.
HOST_SHARE_THREADS = 16


def host_cpu() -> dict:
    """CPU model, online CPUs and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return dict(model=model, nproc=os.cpu_count(), allowed=allowed)


def stop_evidence(n_paths, polarity, spp_init: int, spp_max: int) -> dict:
    """Where the adaptive frame spends its paths: the event fraction f_e
    (events run to spp_max by definition), the non-event pixels that never
    stop before spp_max, a histogram of paths per pixel, and the bound on
    the speed-up over fixed spp_max that these imply,
    S <= 1 / (f_e + (1 - f_e) nbar / spp_max), nbar = mean paths of the
    non-event pixels (time taken as proportional to paths)."""
    n = np.asarray(n_paths, np.int64)
    ev = np.asarray(polarity) != 0
    f_e = float(ev.mean())
    nbar = float(n[~ev].mean()) if (~ev).any() else 0.0
    edges = [spp_init, 2 * spp_init, 4 * spp_init, spp_max // 2, spp_max, spp_max + 1]
    edges = sorted(set(e for e in edges if spp_init <= e <= spp_max + 1))
    hist, _ = np.histogram(n, bins=edges)
    return dict(event_fraction=f_e, never_stopped_non_event_fraction=float(((n >= spp_max) & ~ev).mean()),
                stopped_at_first_test_fraction=float((n == spp_init).mean()),
                mean_paths_non_event=nbar,
                paths_histogram={f"[{edges[i]},{edges[i + 1]})": int(h) for i, h in enumerate(hist)},
                speedup_bound=1.0 / (f_e + (1.0 - f_e) * nbar / spp_max))


def bench_diff(ev, scenes, steps: int = 3) -> dict:
    """Event-loss gradient of the differentiation workload (256x256, 9,648
    triangles, 36 materials, 256 paths per pixel and instant): forward
    paths, per-pixel statistics and the path-replay adjoint per call."""
    import torch
    P = scenes.DIFF_PARAMS
    sc = scenes.diff_scene()
    r = ev.Renderer(0)
    r.set_scene(sc)
    o = dict(seed=P["seed"], max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
             minibatch=P["minibatch"], log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"])
    print("[bench] differentiation workload", file=sys.stderr, flush=True)
    g = r.event_loss_grad(0.0, 1.0, P["C"], P["tau"], P["spp"], o)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        g = r.event_loss_grad(0.0, 1.0, P["C"], P["tau"], P["spp"], o)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    # The product through the per-pixel difference (seeded weights), and
    # the difference alone (the forward half of autograd).
    w = torch.tensor(np.random.default_rng(0).normal(size=sc.width * sc.height), dtype=torch.float64)
    v = r.delta_vjp(0.0, 1.0, P["spp"], w, o)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        v = r.delta_vjp(0.0, 1.0, P["spp"], w, o)
    torch.cuda.synchronize()
    dv = (time.perf_counter() - t) / steps
    t = time.perf_counter()
    for _ in range(steps):
        r.delta_vjp(0.0, 1.0, P["spp"], None, o)
    torch.cuda.synchronize()
    dd = (time.perf_counter() - t) / steps
    paths = 2 * 2 * sc.width * sc.height * P["spp"]
    out = dict(workload=f"{sc.width}x{sc.height}, {sc.n_tri_world} triangles, {len(sc.albedo)} materials, "
                        f"{P['spp']} paths per pixel and instant, depth {P['max_depth']}",
               grad_evals_per_s=1.0 / dt, ms_per_grad=1000.0 * dt, path_evals_per_s=paths / dt,
               loss=float(g["loss"].cpu()[0]), replay_mismatch=int(g["replay_mismatch"].cpu()[0]),
               ms_per_delta_vjp=1000.0 * dv, ms_per_delta_forward=1000.0 * dd,
               delta_vjp_replay_mismatch=int(v["replay_mismatch"].cpu()[0]))
    r.close()
    return out


def bench_video(ev, scenes) -> dict:
    """Sequential event video of the sensor scene over 5 frames (t = 0, 0.25,
    ..., 1; reference carried per pixel, replaced at events), scored by F1,
    RMSE and PSNR against the same video at a fixed 4096 paths."""
    import torch
    P = scenes.SENSOR_PARAMS
    sc = scenes.sensor()
    r = ev.Renderer(0)
    r.set_scene(sc)
    o = dict(seed=P["seed"], max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
             minibatch=P["minibatch"], log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"])
    times = [0.0, 0.25, 0.5, 0.75, 1.0]
    print("[bench] sequential video", file=sys.stderr, flush=True)
    r.render_event_video(times[:2], P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], o,
                         extras=False)
    torch.cuda.synchronize()
    t = time.perf_counter()
    v = r.render_event_video(times, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], o,
                             extras=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    ref = r.render_event_video(times, P["C"], P["alpha"], 4 * P["spp_max"], 16, 4 * P["spp_max"],
                               dict(o, mode=ev.MODE_FIXED), extras=False)
    pol = v["polarity"].cpu().numpy()
    out = dict(workload=f"sensor scene, {len(times)} frames t = 0 ... 1, spp {P['spp_init']}/{P['spp_batch']}/"
                        f"{P['spp_max']}, C {P['C']}, reference video at a fixed {4 * P['spp_max']} paths",
               seconds=dt, frames_per_s=(len(times) - 1) / dt,
               mean_paths_per_pixel=float(v["n_paths"].cpu().numpy().mean()),
               events_per_frame=[int(x) for x in (pol != 0).sum(axis=1)],
               quality=video_scores(pol, ref["polarity"].cpu().numpy()))
    r.close()
    return out


def bench_rgb(ev, scenes, steps: int = 3) -> dict:
    """The sensor workload with RGB radiance (materials and lights coloured
    per channel by scenes.colorize): adaptive event frames/s and rays/s,
    next to the grey frame of the headline."""
    import torch
    P = scenes.SENSOR_PARAMS
    sc = scenes.colorize(scenes.sensor(), seed=1)
    r = ev.Renderer(0)
    r.set_scene(sc)
    o = dict(seed=P["seed"], max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
             minibatch=P["minibatch"], log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"])
    print("[bench] RGB sensor frame", file=sys.stderr, flush=True)

    def frame():
        return r.render_event_frame(0.0, 1.0, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], o,
                                    extras=False)
    frame()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        out = frame()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    st = r.frame_stats()
    rays = st["camera_rays"] + st["extension_rays"] + st["shadow_rays"]
    res = dict(workload="sensor workload with RGB materials and lights", frames_per_s=1.0 / dt,
               ms_per_frame=1000.0 * dt, rays_per_s=rays / dt, rounds=st["rounds"],
               mean_paths_per_pixel=float(out["n_paths"].cpu().numpy().mean()),
               events=int((out["polarity"].cpu().numpy() != 0).sum()))
    r.close()
    return res


def bench_tiny(ev, scenes, steps: int = 20) -> dict:
    """The tiny workload (64x64, 24 triangles, depth 4, schedule 16/16/256,
    C = 0.2, alpha = 0.01): adaptive event frames/s on the GPU, where launch
    latency and the per-round readback dominate."""
    import torch
    P = scenes.TINY_PARAMS
    sc = scenes.tiny_box()
    r = ev.Renderer(0)
    r.set_scene(sc)
    o = dict(seed=P["seed"], max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
             minibatch=P["minibatch"], log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"])
    print("[bench] tiny workload", file=sys.stderr, flush=True)

    def run(mode):
        for _ in range(3):
            out = r.render_event_frame(0.0, 1.0, P["C"], P["alpha"], P["spp_init"], P["spp_batch"],
                                       P["spp_max"], dict(o, mode=mode), extras=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            out = r.render_event_frame(0.0, 1.0, P["C"], P["alpha"], P["spp_init"], P["spp_batch"],
                                       P["spp_max"], dict(o, mode=mode), extras=False)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps, out, r.frame_stats()

    dt, out, st = run(ev.MODE_ADAPTIVE_1T)
    dtf, _, _ = run(ev.MODE_FIXED)
    # The timed frame against the oracle's full frame.
    import oracle
    with oracle.Frame(sc, 0.0, 1.0) as f:
        ro = f.render(oracle.make_params(**P), threads=min(HOST_SHARE_THREADS, os.cpu_count() or 1))
    ok = ~ro["near_crit"]
    g_pol = out["polarity"].cpu().numpy()
    g_n = out["n_paths"].cpu().numpy()
    match = dict(pixels=int(sc.n_pixels), exempt=int((~ok).sum()),
                 polarity_mismatch=int((g_pol[ok] != ro["polarity"][ok]).sum()),
                 n_paths_mismatch=int((g_n[ok] != ro["n_paths"][ok]).sum()))
    rays = st["camera_rays"] + st["extension_rays"] + st["shadow_rays"]
    res = dict(workload=f"tiny: {sc.width}x{sc.height}, {sc.n_tri_world} triangles, depth {P['max_depth']}, "
                        f"spp {P['spp_init']}/{P['spp_batch']}/{P['spp_max']}, C {P['C']}",
               frames_per_s=1.0 / dt, ms_per_frame=1000.0 * dt, rounds=st["rounds"], rays_per_s=rays / dt,
               fixed_frames_per_s=1.0 / dtf, speedup_vs_fixed_spp_max=dtf / dt,
               stop_evidence=stop_evidence(out["n_paths"].cpu().numpy(), out["polarity"].cpu().numpy(),
                                           P["spp_init"], P["spp_max"]),
               oracle_match=match)
    r.close()
    return res


def bench_sensitivity(ev, scenes, C: float = 0.15) -> dict:
    """How the speed-up over fixed spp_max depends on readings the paper
    leaves open: the paths per log-luminance sample (mini-batch 1, 2, 4, 8)
    and the significance (alpha 0.01, the workload's, and 0.05, the
    paper's).  Per setting: adaptive frame time, mean paths per pixel, the
    stop evidence and its bound, and the equal-quality speed-up against the
    fixed count whose polarity F1 (vs a 4096-path fixed reference of the
    same mini-batch) reaches the adaptive map's."""
    import torch
    P = scenes.SENSOR_PARAMS
    sc = scenes.sensor()
    r = ev.Renderer(0)
    r.set_scene(sc)
    base = dict(seed=P["seed"], max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
                log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"])

    def timed(opts, alpha, spp_max, reps=2):
        out = r.render_event_frame(0.0, 1.0, C, alpha, min(P["spp_init"], spp_max), P["spp_batch"], spp_max,
                                   opts, extras=False)
        torch.cuda.synchronize()
        if reps == 0:
            return 0.0, out
        t = time.perf_counter()
        for _ in range(reps):
            out = r.render_event_frame(0.0, 1.0, C, alpha, min(P["spp_init"], spp_max), P["spp_batch"],
                                       spp_max, opts, extras=False)
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, out

    rows = []
    for mb in (1, 2, 4, 8):
        o = dict(base, minibatch=mb)
        t_fixed, _ = timed(dict(o, mode=ev.MODE_FIXED), 0.01, P["spp_max"])
        _, ref = timed(dict(o, mode=ev.MODE_FIXED), 0.01, 4 * P["spp_max"], reps=0)
        ref_map = ref["polarity"].cpu().numpy()
        ladder = {}
        for n in (64, 128, 256, 512, 1024, 2048):
            tn, fo = timed(dict(o, mode=ev.MODE_FIXED), 0.01, n, reps=1)
            ladder[n] = (tn, polarity_f1(fo["polarity"].cpu().numpy(), ref_map))
        for alpha in (0.01, 0.05):
            print(f"[bench] sensitivity minibatch {mb} alpha {alpha}", file=sys.stderr, flush=True)
            ta, out = timed(dict(o, mode=ev.MODE_ADAPTIVE_1T), alpha, P["spp_max"])
            amap = out["polarity"].cpu().numpy()
            f1 = polarity_f1(amap, ref_map)
            n_eq = next((n for n in sorted(ladder) if ladder[n][1] >= f1), None)
            ev_ = stop_evidence(out["n_paths"].cpu().numpy(), amap, P["spp_init"], P["spp_max"])
            rows.append(dict(minibatch=mb, alpha=alpha, ms_adaptive=1000 * ta, ms_fixed_spp_max=1000 * t_fixed,
                             speedup_vs_fixed_spp_max=t_fixed / ta, f1_adaptive=f1, n_eq=n_eq,
                             speedup_equal_quality=(ladder[n_eq][0] / ta) if n_eq else None,
                             mean_paths_per_pixel=float(out["n_paths"].cpu().numpy().mean()),
                             speedup_bound=ev_["speedup_bound"], event_fraction=ev_["event_fraction"],
                             never_stopped_non_event_fraction=ev_["never_stopped_non_event_fraction"]))
    r.close()
    return dict(workload=f"sensor, C {C}, spp {P['spp_init']}/{P['spp_batch']}/{P['spp_max']}", rows=rows)


SCENE_VARIANTS = (("twenty moving spheres", {}), ("one moving sphere", dict(n_moving=1)), ("sky 1.0", dict(sky=1.0)),
                  ("one moving sphere, sky 1.0", dict(n_moving=1, sky=1.0)),
                  ("one moving sphere, sky 3.0", dict(n_moving=1, sky=3.0)))


def bench_scene_variants(ev, scenes, C: float = 0.15, names=None) -> dict:
    """Where the equal-quality speed-up comes from: the sensor workload and
    variants of it with one moving sphere instead of twenty and with a
    uniform grey sky as extra light (fewer dark, noisy pixels).  Per
    variant: adaptive and fixed spp_max frame times, S_paper, polarity F1
    of the adaptive map against a 4 x spp_max fixed reference, N_eq and
    S_eq, and the stop evidence with its bound."""
    import torch
    P = scenes.SENSOR_PARAMS
    base = dict(seed=P["seed"], max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
                log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"])
    rows = []
    for name, kw in SCENE_VARIANTS:
        if names is not None and name not in names:
            continue
        print(f"[bench] scene variant: {name}", file=sys.stderr, flush=True)
        r = ev.Renderer(0)
        r.set_scene(scenes.sensor(**kw))

        def timed(mode, spp_max, reps=2):
            args = (0.0, 1.0, C, P["alpha"], min(P["spp_init"], spp_max), P["spp_batch"], spp_max,
                    dict(base, mode=mode))
            out = r.render_event_frame(*args, extras=False)
            torch.cuda.synchronize()
            if reps == 0:
                return 0.0, out
            t = time.perf_counter()
            for _ in range(reps):
                out = r.render_event_frame(*args, extras=False)
            torch.cuda.synchronize()
            return (time.perf_counter() - t) / reps, out

        ta, out = timed(ev.MODE_ADAPTIVE_1T, P["spp_max"], reps=3)
        tf, _ = timed(ev.MODE_FIXED, P["spp_max"])
        _, ref = timed(ev.MODE_FIXED, 4 * P["spp_max"], reps=0)
        ref_map = ref["polarity"].cpu().numpy()
        amap = out["polarity"].cpu().numpy()
        f1 = polarity_f1(amap, ref_map)
        ladder, n_eq = {}, None
        for n in (64, 128, 256, 512, 1024, 2048):
            tn, fo = timed(ev.MODE_FIXED, n, reps=1)
            ladder[n] = (tn, polarity_f1(fo["polarity"].cpu().numpy(), ref_map))
            if ladder[n][1] >= f1:
                n_eq = n
                break
        se = stop_evidence(out["n_paths"].cpu().numpy().astype(np.int64), amap, P["spp_init"], P["spp_max"])
        rows.append(dict(variant=name, ms_adaptive=1000 * ta, ms_fixed_spp_max=1000 * tf,
                         speedup_vs_fixed_spp_max=tf / ta, f1_adaptive=f1, reference_events=int((ref_map != 0).sum()), n_eq=n_eq,
                         speedup_equal_quality=(ladder[n_eq][0] / ta) if n_eq else None,
                         f1_fixed={str(k): v[1] for k, v in ladder.items()}, stop_evidence=se))
        r.close()
    return dict(workload=f"sensor and variants, C {C}, spp {P['spp_init']}/{P['spp_batch']}/{P['spp_max']}",
                rows=rows)


def bench_batch(ev, scenes, args) -> dict:
    """Frame-batch workload (1280x720, 977,290 triangles, camera panning
    0.5 degrees per frame, schedule 16/16/2048, depth 8): K consecutive pairs
    in one batch call against the loop of K single-pair calls with the same
    frame keys, whose outputs it must equal."""
    import numpy as np
    import torch
    from paper_2408_07996_amd import autotune
    P = scenes.BATCH_PARAMS
    K = args.batch_pairs
    sc = scenes.batch_scene(n_frames=max(65, K + 1))
    r = ev.Renderer(0)
    r.set_scene(sc)
    o = dict(seed=P["seed"], max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
             minibatch=P["minibatch"], log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"])
    tuned = None
    if not args.no_autotune:
        print("[bench] autotuning the launch shape", file=sys.stderr, flush=True)
        at = autotune.autotune(r, 0.0, 1.0, o)
        o = at["opts"]
        tuned = dict(ray_batch=o["ray_batch"], trace_blocks_per_cu=o["trace_blocks_per_cu"],
                     calibration_spp=at["spp"], table=[list(x) for x in at["table"]])
    times = [float(k) for k in range(K + 1)]
    print(f"[bench] batch of {K} pairs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    b = r.render_event_batch(times, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], o,
                             extras=False)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    st = r.frame_stats()
    rays_b = st["camera_rays"] + st["extension_rays"] + st["shadow_rays"]
    print(f"[bench] {K} single-pair calls", file=sys.stderr, flush=True)
    same = True
    rays_p = 0
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(K):
        f = r.render_event_frame(times[k], times[k + 1], P["C"], P["alpha"], P["spp_init"], P["spp_batch"],
                                 P["spp_max"], dict(o, key_base=k), extras=False)
        s2 = r.frame_stats()
        rays_p += s2["camera_rays"] + s2["extension_rays"] + s2["shadow_rays"]
        same = same and bool(torch.equal(f["polarity"], b["polarity"][k])) and \
            bool(torch.equal(f["n_paths"], b["n_paths"][k]))
        if (k + 1) % 8 == 0:
            print(f"[bench]   {k + 1} of {K} pairs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    npth = b["n_paths"].cpu().numpy()
    out = dict(workload=f"{sc.width}x{sc.height}, {sc.n_tri_world} triangles, {K} consecutive pairs, camera "
                        f"panning 0.5 deg/frame, spp {P['spp_init']}/{P['spp_batch']}/{P['spp_max']}, "
                        f"depth {P['max_depth']}, C {P['C']}",
               pairs=K, batch_s=tb, pair_loop_s=tp, speedup=tp / tb, identical_to_pair_loop=same,
               batch_pairs_per_s=K / tb, batch_rays_per_s=rays_b / tb, pair_loop_rays_per_s=rays_p / tp,
               sample_share_bound=2.0 * K / (K + 1),
               # The work the sharing saves: a shared frame is traced to the
               # larger of its two pairs' counts, so fewer rays than 2K/(K+1).
               loop_over_batch_rays=rays_p / max(1.0, float(rays_b)),
               mean_paths_per_pixel=float(npth.mean()),
               events_per_pair=float((b["polarity"].cpu().numpy() != 0).sum(axis=1).mean()), autotune=tuned)
    r.close()
    return out


def bench_stress(ev, scenes, args) -> dict:
    """Stress workload (1920x1080 city of 4.32M triangles, camera flying and
    50 boxes moving every frame, depth 12, schedule 64/64/4096, C = 0.2,
    alpha = 0.001): K consecutive pairs in one batch call (one geometry
    instant per frame, built on host threads), with the per-pair figures
    and the host build time."""
    import torch
    P = scenes.CITY_PARAMS
    K = args.stress_pairs
    sc = scenes.city(n_frames=max(K + 1, 2))
    r = ev.Renderer(0)
    r.set_scene(sc)
    o = dict(seed=P["seed"], max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
             minibatch=P["minibatch"], log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"])
    times = [float(k) for k in range(K + 1)]
    print(f"[bench] stress batch of {K} pairs", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    b = r.render_event_batch(times, P["C"], P["alpha"], P["spp_init"], P["spp_batch"], P["spp_max"], o,
                             extras=False)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    st = r.frame_stats()
    rays = st["camera_rays"] + st["extension_rays"] + st["shadow_rays"]
    npth = b["n_paths"].cpu().numpy()
    out = dict(workload=f"city: {sc.width}x{sc.height}, {sc.n_tri_world} triangles, {K} consecutive pairs, "
                        f"moving camera and 50 moving boxes, spp {P['spp_init']}/{P['spp_batch']}/{P['spp_max']}, "
                        f"depth {P['max_depth']}, C {P['C']}, alpha {P['alpha']}",
               pairs=K, batch_s=tb, s_per_pair=tb / K, pairs_per_s=K / tb, rays_per_s=rays / tb,
               host_build_s=st["ms_build"] / 1000.0, rounds=st["rounds"], paths=st["paths"],
               mean_paths_per_pixel=float(npth.mean()),
               events_per_pair=float((b["polarity"].cpu().numpy() != 0).sum(axis=1).mean()))
    r.close()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--C", type=float, default=0.15)
    ap.add_argument("--no-quality", action="store_true", help="skip the equal-quality fixed-spp ladder")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-step", type=int, default=2, help="oracle sample: every n-th pixel in x and y")
    ap.add_argument("--kernel-only", action="store_true",
                    help="run only the timed adaptive frames (for profiler runs)")
    ap.add_argument("--ray-batch", type=int, default=0, help="paths in flight per piece (0: library default)")
    ap.add_argument("--lds-nodes", type=int, default=0, help="top BVH nodes staged in LDS")
    ap.add_argument("--trace-blocks", type=int, default=0,
                    help="traversal blocks per CU of the sensor frame (0: occupancy max)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB on the device (counter calibration)")
    ap.add_argument("--stress-pairs", type=int, default=8, help="pairs of the stress workload (--only stress)")
    ap.add_argument("--only", choices=("all", "frame", "diff", "batch", "video", "tiny", "sensitivity", "stress",
                                       "rgb", "variants"),
                    default="all",
                    help="which workloads to run (the headline is the frame workload)")
    ap.add_argument("--batch-pairs", type=int, default=64, help="pairs of the frame-batch workload")
    ap.add_argument("--no-autotune", action="store_true", help="skip the launch-shape autotuner")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); every pixel and sample is "
              "independent, so a multi-GPU run would shard pixels, which this renderer does not do.",
              file=sys.stderr)
        return 2

    import torch
    import paper_2408_07996_amd as ev
    from paper_2408_07996_amd import scenes

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    if args.copy_mib:
        src = torch.ones(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only in ("diff", "batch", "video", "tiny", "sensitivity", "stress", "rgb", "variants"):
        res = {"metric": "next-row workloads", "next_rows": {}}
        if args.only == "variants":
            res["scene_variants"] = bench_scene_variants(ev, scenes, args.C)
        elif args.only == "rgb":
            res["next_rows"]["rgb_frame"] = bench_rgb(ev, scenes)
        elif args.only == "stress":
            res["next_rows"]["stress"] = bench_stress(ev, scenes, args)
        elif args.only == "sensitivity":
            res["sensitivity"] = bench_sensitivity(ev, scenes, args.C)
        elif args.only == "diff":
            res["next_rows"]["differentiation"] = bench_diff(ev, scenes)
        elif args.only == "tiny":
            res["tiny"] = bench_tiny(ev, scenes)
        elif args.only == "video":
            res["next_rows"]["sequential_video"] = bench_video(ev, scenes)
        else:
            res["next_rows"]["batching"] = bench_batch(ev, scenes, args)
        print(json.dumps(res), flush=True)
        return 0
    sc = scenes.sensor()
    P = dict(scenes.SENSOR_PARAMS, C=args.C)
    base_opts = dict(seed=P["seed"], max_depth=P["max_depth"], rr_start_depth=P["rr_start_depth"],
                     minibatch=P["minibatch"], log_eps=P["log_eps"], nee=P["nee"], jitter=P["jitter"],
                     ray_batch=args.ray_batch, lds_nodes=args.lds_nodes,
                     trace_blocks_per_cu=args.trace_blocks)
    r = ev.Renderer(0)
    t_build = time.perf_counter()
    r.set_scene(sc)
    info = r.scene_info_at(0.0)

    def frame(mode=ev.MODE_ADAPTIVE_1T, spp_max=P["spp_max"], spp_init=P["spp_init"], C=P["C"], **kw):
        o = dict(base_opts, mode=mode, **kw)
        out = r.render_event_frame(0.0, 1.0, C, P["alpha"], min(spp_init, spp_max), P["spp_batch"],
                                   spp_max, opts=o, extras=False)
        return out, r.frame_stats()

    print(f"[bench] warmup {args.warmup} frames", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        frame(profile=1)
    build_ms = time.perf_counter() - t_build

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rays = 0
    ms_closest = 0.0
    n_closest = 0
    ms_shadow = 0.0
    n_shadow = 0
    out = None
    stats = None
    step_ms = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        out, stats = frame(profile=1)
        # The call returns after its last round's readback: the device is
        # idle here, so the host interval is the frame's.
        step_ms.append(1000.0 * (time.perf_counter() - ts))
        rays += stats["camera_rays"] + stats["extension_rays"] + stats["shadow_rays"]
        ms_closest += stats["ms_closest"]
        n_closest += stats["n_closest_launches"]
        ms_shadow += stats["ms_shadow"]
        n_shadow += stats["n_shadow_launches"]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    fps = args.steps / elapsed
    print(f"[bench] adaptive {1000 * elapsed / args.steps:.1f} ms/frame", file=sys.stderr, flush=True)
    if args.kernel_only:
        # The last frame's schedule, for reading a kernel trace of this run.
        nr = min(64, stats["rounds"])
        print(json.dumps(dict(frames_per_s=fps, ms_per_step=1000 * elapsed / args.steps,
                              rounds=stats["rounds"], active_after_round=list(stats["active_after_round"][:nr]),
                              paths=stats["paths"], camera_rays=stats["camera_rays"],
                              extension_rays=stats["extension_rays"], shadow_rays=stats["shadow_rays"])))
        return 0

    # Work counts of the same (deterministic) frame for the roofline.
    _, cst = frame(count_work=1)
    ops_closest = cst["node_visits"] * OPS_PER_NODE + cst["tri_tests"] * OPS_PER_TRI
    ms_per_closest = ms_closest / max(1, n_closest)
    launches_per_frame = n_closest / args.steps
    ops_per_launch = ops_closest / max(1.0, launches_per_frame)
    achieved = ops_per_launch / (ms_per_closest * 1e-3) if ms_per_closest > 0 else 0.0
    ops_shadow = cst["node_visits_shadow"] * OPS_PER_NODE + cst["tri_tests_shadow"] * OPS_PER_TRI
    ms_per_shadow = ms_shadow / max(1, n_shadow)
    shadow_launches_per_frame = n_shadow / args.steps
    achieved_shadow = (ops_shadow / max(1.0, shadow_launches_per_frame) / (ms_per_shadow * 1e-3)
                       if ms_per_shadow > 0 else 0.0)
    closest_rays_per_launch = (cst["camera_rays"] + cst["extension_rays"]) / max(1.0, launches_per_frame)
    shadow_rays_per_launch = cst["shadow_rays"] / max(1.0, shadow_launches_per_frame)

    measured = kernel_sources_digest() == TRAFFIC["sources_sha256"]
    traffic = TRAFFIC["bytes_per_launch"] if measured else None
    counters = TRAFFIC.get("counters") if measured else None
    # Both traversal kernels over the frame: their algorithmic lane-ops per
    # frame over the frame time (the two lanes run concurrently, so the
    # per-launch figure above counts each launch's time shared with the
    # other lane's kernels).
    ops_frame = ops_closest + cst["node_visits_shadow"] * OPS_PER_NODE + cst["tri_tests_shadow"] * OPS_PER_TRI
    frame_frac = ops_frame / (elapsed / args.steps) / PEAK_LANE_OPS

    adaptive_map = out["polarity"].cpu().numpy()
    adaptive_paths = out["n_paths"].cpu().numpy().astype(np.int64)

    # Fixed-count comparator (the paper's baseline: spp_max everywhere).
    print("[bench] fixed-spp comparator", file=sys.stderr, flush=True)
    frame(mode=ev.MODE_FIXED)
    torch.cuda.synchronize()
    tf = time.perf_counter()
    nf = 2
    for _ in range(nf):
        fout, fst = frame(mode=ev.MODE_FIXED)
    torch.cuda.synchronize()
    t_fixed = (time.perf_counter() - tf) / nf
    t_adapt = elapsed / args.steps
    # Paths per second: the ones the outputs use (n_paths at both instants)
    # and all traced (a round traces past a pixel's stop).
    # Rays per path differ between the two: the pixels that stop first are
    # the cheap ones (no hit, or black), so the paths left to the adaptive
    # rounds carry more rays; rays/s compares the renderers' efficiency.
    used_adapt = 2.0 * float(adaptive_paths.sum())
    rays_adapt = stats["camera_rays"] + stats["extension_rays"] + stats["shadow_rays"]
    rays_fixed = fst["camera_rays"] + fst["extension_rays"] + fst["shadow_rays"]
    throughput = dict(adaptive_used_paths_per_s=used_adapt / t_adapt,
                      adaptive_traced_paths_per_s=stats["paths"] / t_adapt,
                      traced_past_stop_fraction=1.0 - used_adapt / max(1.0, float(stats["paths"])),
                      fixed_paths_per_s=fst["paths"] / t_fixed,
                      adaptive_over_fixed_used=(used_adapt / t_adapt) / (fst["paths"] / t_fixed),
                      adaptive_rays_per_s=rays_adapt / t_adapt, fixed_rays_per_s=rays_fixed / t_fixed,
                      adaptive_rays_per_traced_path=rays_adapt / max(1.0, float(stats["paths"])),
                      fixed_rays_per_path=rays_fixed / max(1.0, float(fst["paths"])),
                      ray_weighted_speedup_bound=rays_fixed / max(1.0, rays_adapt * used_adapt / max(1.0, float(stats["paths"]))))

    def quality(C, adapt_map, t_ad):
        """Polarity F1 of the adaptive map and of fixed counts against a
        4 x spp_max reference at threshold C; N_eq and S_eq."""
        ref, _ = frame(mode=ev.MODE_FIXED, spp_max=4 * P["spp_max"], C=C)
        ref_map = ref["polarity"].cpu().numpy()
        f1_adapt = polarity_f1(adapt_map, ref_map)
        q = dict(reference_spp=4 * P["spp_max"], f1_adaptive=f1_adapt, f1_fixed={},
                 ref_events=int((ref_map != 0).sum()))
        n_eq = None
        for n in (64, 128, 256, 512, 1024, 2048):
            fo, _ = frame(mode=ev.MODE_FIXED, spp_max=n, C=C)
            f1 = polarity_f1(fo["polarity"].cpu().numpy(), ref_map)
            q["f1_fixed"][str(n)] = f1
            if f1 >= f1_adapt:
                n_eq = n
                break
        s = None
        if n_eq is not None:
            frame(mode=ev.MODE_FIXED, spp_max=n_eq, C=C)
            torch.cuda.synchronize()
            te = time.perf_counter()
            frame(mode=ev.MODE_FIXED, spp_max=n_eq, C=C)
            torch.cuda.synchronize()
            s = (time.perf_counter() - te) / t_ad
            q["n_eq"] = n_eq
        return q, s

    quality_main, s_eq = ({}, None)
    second = None
    if not args.no_quality:
        print("[bench] equal-quality ladder", file=sys.stderr, flush=True)
        quality_main, s_eq = quality(P["C"], adaptive_map, t_adapt)
        # The second threshold of the workload: its own timing and ladder.
        C2 = 0.3 if abs(P["C"] - 0.3) > 1e-6 else 0.15
        print(f"[bench] threshold C = {C2}", file=sys.stderr, flush=True)
        frame(C=C2)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for _ in range(3):
            o2, s2 = frame(C=C2)
        torch.cuda.synchronize()
        t_ad2 = (time.perf_counter() - t2) / 3
        map2 = o2["polarity"].cpu().numpy()
        q2, s_eq2 = quality(C2, map2, t_ad2)
        second = dict(C=C2, frames_per_s=1.0 / t_ad2, ms_per_step=1000.0 * t_ad2,
                      mean_paths_per_pixel=float(o2["n_paths"].cpu().numpy().mean()),
                      stop_evidence=stop_evidence(o2["n_paths"].cpu().numpy().astype(np.int64), map2,
                                                  P["spp_init"], P["spp_max"]),
                      events=int((map2 != 0).sum()), speedup_vs_fixed_spp_max=t_fixed / t_ad2,
                      speedup_equal_quality=s_eq2, quality=q2)

    cpu = None
    oracle_match = None
    if not args.no_cpu:
        import oracle
        host = host_cpu()
        # Every CPU the process may use, up to one GPU's host share of the box.
        threads = max(1, min(HOST_SHARE_THREADS, host["allowed"]))
        px = scenes.subset_every(sc.width, sc.height, args.cpu_step)
        print(f"[bench] CPU oracle on {len(px)} pixels, {threads} threads", file=sys.stderr, flush=True)
        with oracle.Frame(sc, 0.0, 1.0) as f:
            tc = time.perf_counter()
            ro = f.render(oracle.make_params(**P), px, threads=threads)
            t_cpu = time.perf_counter() - tc
        # The timed frame against the oracle on the same pixels: decisions
        # within the exemption band of a critical value may go either way.
        ok = ~ro["near_crit"]
        g_pol = adaptive_map.reshape(-1)[px]
        g_n = adaptive_paths.reshape(-1)[px]
        g_mean = out["mean"].cpu().numpy().reshape(-1, 2)[px]
        same_n = g_n == ro["n_paths"]
        mean_err = np.abs(g_mean[same_n] - ro["mean"][same_n]) / np.maximum(1.0, np.abs(ro["mean"][same_n]))
        oracle_match = dict(pixels=int(len(px)), exempt=int((~ok).sum()),
                            polarity_mismatch=int((g_pol[ok] != ro["polarity"][ok]).sum()),
                            n_paths_mismatch=int((g_n[ok] != ro["n_paths"][ok]).sum()),
                            max_mean_rel_err=float(mean_err.max(initial=0.0)))
        s_per_frame = t_cpu * sc.n_pixels / len(px)
        # The tiny workload's full frame, not extrapolated.
        tiny = scenes.tiny_box()
        with oracle.Frame(tiny, 0.0, 1.0) as f:
            tc = time.perf_counter()
            f.render(oracle.make_params(**scenes.TINY_PARAMS), threads=threads)
            t_tiny = time.perf_counter() - tc
        cpu = dict(value=1.0 / s_per_frame, unit="event frames/s", cores=threads, kind="oracle",
                   sample=f"every pixel whose x and y are multiples of {args.cpu_step} ({len(px)} of {sc.n_pixels} pixels, "
                          f"adaptive, both instants), {t_cpu:.1f} s, scaled by {sc.n_pixels / len(px):.0f}",
                   cpu_model=host["model"], nproc=host["nproc"], cpus_allowed=host["allowed"],
                   threads_rule=f"all CPUs the process may use, at most {HOST_SHARE_THREADS} (one GPU's host share)",
                   tiny_full_frame_s=t_tiny, tiny_frames_per_s=1.0 / t_tiny)

    res = {
        "metric": "event frames/s + rays/s at oracle-matched events; speedup vs fixed-spp GPU",
        "value": fps,
        "unit": "event frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "median_ms_per_step": float(np.median(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "sensor: 640x480, 97,806 triangles (displaced floor + 20 moving icospheres), "
                               "3 area lights, depth 8, NEE+RR, 4-path logL, spp 64/16/1024, t0=0 t1=1",
                   "C": P["C"], "alpha": P["alpha"], "width": sc.width, "height": sc.height,
                   "triangles": info["n_tri"], "spp_init": P["spp_init"], "spp_batch": P["spp_batch"],
                   "spp_max": P["spp_max"], "max_depth": P["max_depth"], "parallelism": "1 GPU"},
        "rays_per_s": rays / elapsed,
        "mean_paths_per_pixel": float(adaptive_paths.mean()),
        "events": int((adaptive_map != 0).sum()),
        "rounds": stats["rounds"],
        "throughput": throughput,
        "stop_evidence": stop_evidence(adaptive_paths, adaptive_map, P["spp_init"], P["spp_max"]),
        "fixed_frames_per_s": 1.0 / t_fixed,
        "speedup_vs_fixed_spp_max": t_fixed / t_adapt,
        "speedup_equal_quality": s_eq,
        "f1_vs_fixed_spp_max": polarity_f1(adaptive_map, fout["polarity"].cpu().numpy()),
        "quality": quality_main,
        "second_threshold": second,
        "roofline": {
            "kernel": "k_trace_closest",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_LANE_OPS / 1e12,
            "unit": "Tlane-op/s",
            "frac": achieved / PEAK_LANE_OPS,
            "traffic": traffic,
            "traffic_unit": "bytes per launch",
            "ms_per_launch": ms_per_closest,
            "launches_per_frame": launches_per_frame,
            "node_visits_per_frame": cst["node_visits"],
            "tri_tests_per_frame": cst["tri_tests"],
            "closest_rays_per_launch": closest_rays_per_launch,
            "shadow_frac": achieved_shadow / PEAK_LANE_OPS,
            "shadow_rays_per_launch": shadow_rays_per_launch,
            "shadow_ms_per_launch": ms_shadow / max(1, n_shadow),
            "closest_ms_per_frame": ms_closest / args.steps,
            "shadow_ms_per_frame": ms_shadow / args.steps,
            "traversal_frac_over_frame": frame_frac,
            "counters": counters,
        },
        "cpu_baseline": cpu,
        "oracle_match": oracle_match,
        "paper_context": PAPER_CONTEXT,
        "scene_build_and_warmup_s": build_ms,
    }
    if args.only == "all":
        r.close()
        res["tiny"] = bench_tiny(ev, scenes)
        res["next_rows"] = {"differentiation": bench_diff(ev, scenes),
                            "batching": bench_batch(ev, scenes, args),
                            "sequential_video": bench_video(ev, scenes),
                            "rgb_frame": bench_rgb(ev, scenes)}
        # Where the equal-quality ceiling comes from (all five variants:
        # --only variants).
        res["scene_variants"] = bench_scene_variants(ev, scenes, P["C"], names=("one moving sphere", "sky 1.0"))
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
