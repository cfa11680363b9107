"""Invariants of the oracle's Algorithm 1 loop on the tiny box workload."""
import math

import numpy as np
import pytest

import oracle
from paper_2408_07996_amd import scenes


@pytest.fixture(scope="module")
def tiny():
    sc = scenes.tiny_box()
    f = oracle.Frame(sc, 0.0, 1.0)
    p = oracle.make_params(**scenes.TINY_PARAMS)
    r = f.render(p)
    yield sc, f, p, r
    f.close()


def test_schedule_and_decision_invariants(tiny):
    sc, f, p, r = tiny
    n = r["n_paths"]
    C = float(np.float32(p.C))
    gap = r["mean"][:, 1] - r["mean"][:, 0]
    # sample counts follow the schedule 16, 32, ..., 256
    assert set(np.unique(n)) <= set(range(16, 257, 16))
    # decided early => no event, and |gap| < C (Sec. 3.2)
    early = r["decided_early"]
    assert early.any()
    assert (r["polarity"][early] == 0).all()
    assert (np.abs(gap[early]) < C).all()
    assert (n[early] < 256).all()
    # an event pixel always runs to the maximum count
    assert (n[r["polarity"] != 0] == 256).all()
    # pixels that did not stop early ran to the maximum
    assert (n[~early] == 256).all()
    # the event rule: strict |gap| > C, polarity = sign(gap)
    ev = np.abs(gap) > C
    np.testing.assert_array_equal(r["polarity"], np.where(ev, np.sign(gap), 0).astype(np.int8))
    # lock step: both instants have the same count
    np.testing.assert_array_equal(r["n_paths_ref"], n)
    assert (r["rounds"] == n // 16).all()


def test_jensen_inequality(tiny):
    """ln E[Y] >= E[ln Y] (Eq. 5), per pixel and instant."""
    _, _, p, r = tiny
    lhs = np.log(r["mean_radiance"] + p.log_eps)
    assert (lhs >= r["mean"] - 1e-12).all()


def test_zero_threshold_never_stops_and_equals_fixed(tiny):
    """C = 0 makes t >= 0, so nothing stops early and the result is the
    fixed-count result bit for bit."""
    sc, f, p, _ = tiny
    px = np.arange(0, 4096, 97, dtype=np.uint32)
    a = f.render(oracle.make_params(**{**scenes.TINY_PARAMS, "C": 0.0}), px)
    b = f.render(oracle.make_params(**{**scenes.TINY_PARAMS, "C": 0.0, "mode": oracle.MODE_FIXED}), px)
    assert (a["n_paths"] == 256).all() and not a["decided_early"].any()
    for k in ("polarity", "n_paths", "mean", "var", "mean_radiance", "t_last"):
        np.testing.assert_array_equal(a[k], b[k])


def test_statistics_equal_fixed_count_at_the_stop(tiny):
    """The statistics after stopping at n equal a fixed-count render at n."""
    sc, f, p, r = tiny
    for n_stop in (16, 48, 112):
        px = r["pixels"][r["n_paths"] == n_stop][:25]
        if len(px) == 0:
            continue
        fx = f.render(oracle.make_params(**{**scenes.TINY_PARAMS, "mode": oracle.MODE_FIXED,
                                            "spp_max": n_stop}), px)
        sel = np.searchsorted(r["pixels"], px)
        np.testing.assert_array_equal(fx["mean"], r["mean"][sel])
        np.testing.assert_array_equal(fx["var"], r["var"][sel])


def test_subset_and_thread_count_do_not_change_results(tiny):
    sc, f, p, r = tiny
    px = np.array([5, 77, 1024, 2047, 4095, 3000, 1], dtype=np.uint32)
    a = f.render(p, px, threads=1)
    sel = px
    for k in ("polarity", "n_paths", "mean", "var", "t_last"):
        np.testing.assert_array_equal(a[k], r[k][sel])


def test_fixed_mode_and_reference_full(tiny):
    sc, f, p, r = tiny
    px = np.arange(0, 4096, 131, dtype=np.uint32)
    fx = f.render(oracle.make_params(**{**scenes.TINY_PARAMS, "mode": oracle.MODE_FIXED}), px)
    assert (fx["n_paths"] == 256).all() and (fx["rounds"] == 1).all()
    rf = f.render(oracle.make_params(**{**scenes.TINY_PARAMS, "ref_mode": oracle.REF_FULL}), px)
    assert (rf["n_paths_ref"] == 256).all()
    np.testing.assert_array_equal(rf["mean"][:, 0], fx["mean"][:, 0])
    assert (rf["n_paths"] <= 256).all()


def test_pixel_event_map_is_local_to_the_moving_cube(tiny):
    """Events appear only where the cube (or its shadow) changes; a static
    scene (t0 = t1 geometry) gives almost none."""
    sc, f, p, r = tiny
    assert 0 < (r["polarity"] != 0).sum() < 0.2 * sc.n_pixels
    with oracle.Frame(sc, 0.0, 0.0) as g:
        s = g.render(p, np.arange(0, 4096, 5, dtype=np.uint32))
    assert (s["polarity"] != 0).mean() < (r["polarity"] != 0).mean()


def test_invalid_parameters_rejected():
    sc = scenes.empty(4, 4)
    with oracle.Frame(sc, 0, 1) as f:
        for bad in (dict(spp_init=6), dict(spp_init=4, minibatch=4), dict(spp_init=512),
                    dict(minibatch=3, spp_init=12, spp_batch=12, spp_max=48)):
            with pytest.raises(ValueError):
                f.render(oracle.make_params(**bad))
        with pytest.raises(ValueError):
            f.render(oracle.make_params(), np.array([16], np.uint32))


def test_same_instant_key_gives_identical_statistics():
    """Invariant (vi): an instant's random numbers are keyed by its frame
    q = key_base + instant, so at equal times instant 1 of a render with
    key_base k and instant 0 of one with key_base k + 1 sample identical
    paths: bitwise equal means, variances and radiance (fixed count), and
    Delta = 0 exactly between them; with distinct keys they differ."""
    sc = scenes.tiny_box(width=24, height=20)
    P = dict(scenes.TINY_PARAMS, mode=oracle.MODE_FIXED, spp_max=64)
    with oracle.Frame(sc, 0.5, 0.5) as f:
        a = f.render(oracle.make_params(**P, key_base=3))
        b = f.render(oracle.make_params(**P, key_base=4))
    for k in ("mean", "var", "mean_radiance"):
        np.testing.assert_array_equal(a[k][:, 1], b[k][:, 0])
    assert ((a["mean"][:, 1] - b["mean"][:, 0]) == 0).all()
    assert (a["mean"][:, 0] != a["mean"][:, 1]).mean() > 0.5
