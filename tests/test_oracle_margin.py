"""Pins of the oracle's decision boundaries: the exemption margin that
excuses pixels from bit-exact comparison, the two-tailed alpha/2 split,
the mean-only rule's boundary, and the per-pixel stopping loop of
Algorithm 1 (pair and sequential video), each checked against scipy's
t distribution and two-sample t-tests or against a plain Python rerun of
the loop on the oracle's own path radiances (Eq. 7, Sec. 3.2, Alg. 1)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2408_07996_amd import scenes

F32 = np.float32

# Zero-variance pixels (all-black mini-batches) are part of the data.
pytestmark = pytest.mark.filterwarnings("ignore:Precision loss occurred")


# --------------------------------------------------------------------------
# Margin of one decision against scipy's quantiles.

@pytest.mark.parametrize("df", [6.0, 30.0, 126.0, 17.37, 510.0])
def test_crit_margin_matches_scipy_quantiles(df):
    rng = np.random.default_rng(int(df * 100))
    for alpha in (0.01, 0.05, 0.001):
        a = float(F32(alpha))
        for t in rng.uniform(-6.0, 6.0, 40):
            m1 = oracle.crit_margin(oracle.MODE_ADAPTIVE_1T, t, df, alpha)
            assert abs(m1 - abs(t - stats.t.ppf(a, df))) < 1e-9
            m2 = oracle.crit_margin(oracle.MODE_ADAPTIVE_2T, t, df, alpha)
            ref2 = min(abs(t - stats.t.ppf(0.5 * a, df)), abs(t - stats.t.ppf(1.0 - 0.5 * a, df)))
            assert abs(m2 - ref2) < 1e-9
            # Mean-only stops at |gap| <= C, i.e. t <= 0; the final event rule
            # |gap| > C is t > 0: both have the boundary t = 0.
            assert oracle.crit_margin(oracle.MODE_MEAN_ONLY, t, df, alpha) == abs(t)
            assert oracle.crit_margin(oracle.MODE_ADAPTIVE_1T, t, df, alpha, final_check=True) == abs(t)
            assert oracle.crit_margin(oracle.MODE_FIXED, t, df, alpha) == math.inf


def _placed(target_t, m, C, seed=7):
    """Two sample sets whose Eq. 7 statistic is target_t: x1 is x0 shifted by
    g = C + target_t * sqrt(2 s^2 / m), so both have the same variance."""
    rng = np.random.default_rng(seed)
    x0 = rng.normal(0.0, 0.05, m)
    s2 = x0.var(ddof=1)
    g = float(C) + target_t * math.sqrt(2.0 * s2 / m)
    return x0, x0 + g


@pytest.mark.parametrize("offset", [-2e-4, -5e-5, 5e-5, 2e-4])
@pytest.mark.parametrize("mode", [oracle.MODE_ADAPTIVE_1T, oracle.MODE_ADAPTIVE_2T])
def test_margin_band_around_the_critical_value(offset, mode):
    """t placed 5e-5 and 2e-4 on either side of the critical value: the
    margin equals the offset, the band of 1e-4 covers only the inner pair,
    and the stop decision flips across the boundary."""
    m, C, alpha = 16, F32(0.2), F32(0.01)
    df = 2 * m - 2
    bounds = [stats.t.ppf(float(alpha), df)]
    if mode == oracle.MODE_ADAPTIVE_2T:
        bounds = [stats.t.ppf(0.5 * float(alpha), df), stats.t.ppf(1.0 - 0.5 * float(alpha), df)]
    for crit in bounds:
        x0, x1 = _placed(crit + offset, m, C)
        r = oracle.decide(x0, x1, C, alpha, mode=mode)
        assert abs(r["t"] - (crit + offset)) < 1e-9
        assert abs(r["margin"] - abs(offset)) < 1e-8
        assert (r["margin"] < 1e-4) == (abs(offset) < 1e-4)
        if crit < 0:
            assert r["stop"] == (offset < 0)   # below the lower critical value: stop
        else:
            assert r["stop"] == (offset > 0)   # above the upper one (two-tailed): stop


# --------------------------------------------------------------------------
# Two-tailed rule: alpha / 2 in each tail is scipy's two-sided test at alpha.

def test_two_tailed_rule_is_scipy_two_sided_test():
    m, C, alpha = 16, F32(0.2), F32(0.01)
    a = float(alpha)
    df = 2 * m - 2
    lo2, lo1 = stats.t.ppf(0.5 * a, df), stats.t.ppf(a, df)
    hi1, hi2 = stats.t.ppf(1.0 - a, df), stats.t.ppf(1.0 - 0.5 * a, df)
    # t values on both sides of every boundary, including the bands
    # (t_{alpha/2}, t_alpha) and (t_{1-alpha}, t_{1-alpha/2}) where a split
    # of alpha instead of alpha / 2 would decide differently.
    targets = np.concatenate([np.linspace(lo2 - 0.5, hi2 + 0.5, 61),
                              [0.5 * (lo2 + lo1), 0.5 * (hi1 + hi2), lo2 - 1e-3, lo2 + 1e-3, hi2 - 1e-3,
                               hi2 + 1e-3]])
    seen_band = 0
    for i, tt in enumerate(targets):
        x0, x1 = _placed(tt, m, C, seed=100 + i)
        r2 = oracle.decide(x0, x1, C, alpha, mode=oracle.MODE_ADAPTIVE_2T)
        r1 = oracle.decide(x0, x1, C, alpha, mode=oracle.MODE_ADAPTIVE_1T)
        d = x1.mean() - x0.mean()
        sa, sb = (x1 - float(C), x0) if d >= 0 else (x0 - float(C), x1)
        two = stats.ttest_ind(sa, sb, equal_var=True, alternative="two-sided")
        assert r2["stop"] == (two.pvalue < a), (tt, two.pvalue)
        if lo2 + 1e-6 < tt < lo1 - 1e-6:
            seen_band += 1
            assert r1["stop"] and not r2["stop"]
        if hi1 + 1e-6 < tt < hi2 - 1e-6:
            seen_band += 1
            assert not r1["stop"] and not r2["stop"]
    assert seen_band >= 2


# --------------------------------------------------------------------------
# Mean-only rule: stop once |gap| <= C (the boundary itself stops).

def test_mean_only_boundary_is_inclusive():
    x0 = np.array([0.0, 0.5, 0.25, 0.75])       # dyadic: sums and means exact
    C = 0.25
    x1 = x0 + C                                  # gap exactly C
    assert x1.mean() - x0.mean() == C
    r = oracle.decide(x0, x1, C, 0.01, mode=oracle.MODE_MEAN_ONLY)
    assert r["stop"] and r["t"] == 0.0 and r["margin"] == 0.0
    assert not oracle.decide(x0, x1 + 2.0 ** -20, C, 0.01, mode=oracle.MODE_MEAN_ONLY)["stop"]
    assert oracle.decide(x0, x1 - 2.0 ** -20, C, 0.01, mode=oracle.MODE_MEAN_ONLY)["stop"]
    assert oracle.decide(x1, x0, C, 0.01, mode=oracle.MODE_MEAN_ONLY)["stop"]   # gap = -C


# --------------------------------------------------------------------------
# Normality pre-test (Jarque-Bera).

def test_jarque_bera_matches_scipy_and_closed_form():
    rng = np.random.default_rng(8)
    for m in (4, 16, 64, 1000):
        for draw in (rng.normal(0, 1, m), rng.exponential(1.0, m), np.log(rng.uniform(0, 1, m) + 1e-4)):
            ref = stats.jarque_bera(draw).statistic
            assert oracle.jarque_bera(draw) == pytest.approx(ref, rel=1e-10, abs=1e-12)
    # Two-point data +-1: m2 = 1, m3 = 0, m4 = 1, excess kurtosis -2, JB = m / 6.
    for m in (2, 10, 64):
        x = np.tile([-1.0, 1.0], m // 2)
        assert oracle.jarque_bera(x) == pytest.approx(len(x) / 6.0, rel=1e-15)
    assert oracle.jarque_bera(np.full(8, 0.75)) == 0.0


# --------------------------------------------------------------------------
# Algorithm 1 per pixel, rerun in Python on the oracle's path radiances.

def _mb_logs(L, mb, eps):
    """Mini-batch means in FP32 by the pairwise order of the estimator
    (((L0 + L1) + (L2 + L3)) * 0.25 for 4) and their FP64 logs."""
    L = np.asarray(L, F32).reshape(-1, mb)
    while L.shape[1] > 1:
        L = (L[:, 0::2] + L[:, 1::2]).astype(F32)
    Y = (L[:, 0] * F32(1.0 / mb)).astype(F32)
    return np.log(Y.astype(np.float64) + eps)


def _eq7(x0, x1, C):
    """Eq. 7 with N = the count at the second instant."""
    gap = abs(x1.mean() - x0.mean()) - C
    S = x0.var(ddof=1) + x1.var(ddof=1)
    if S == 0.0:
        return -math.inf if gap < 0 else (math.inf if gap > 0 else 0.0)
    return gap / math.sqrt(S / len(x1))


def _test(x0, x1, C, alpha, mode, welch):
    """(t, stop, margin) at one checkpoint before the last count.  With
    equal counts t and p come from scipy's two-sample t-test of
    H0: |mu1 - mu0| = C; otherwise t is Eq. 7 and p scipy's t distribution
    at the pooled df m0 + m1 - 2."""
    d = x1.mean() - x0.mean()
    if len(x0) == len(x1):
        sa, sb = (x1 - C, x0) if d >= 0 else (x0 - C, x1)
        r = stats.ttest_ind(sa, sb, equal_var=not welch, alternative="less")
        t, df, p = float(r.statistic), float(r.df), float(r.pvalue)
        if not np.isfinite(t):
            t = _eq7(x0, x1, C)
            df = len(x0) + len(x1) - 2.0
            p = stats.t.cdf(t, df)
    else:
        assert not welch
        t = _eq7(x0, x1, C)
        df = len(x0) + len(x1) - 2.0
        p = stats.t.cdf(t, df)
    if mode == oracle.MODE_ADAPTIVE_1T:
        return t, p < alpha, abs(t - stats.t.ppf(alpha, df))
    if mode == oracle.MODE_ADAPTIVE_2T:
        up = stats.t.sf(t, df)
        margin = min(abs(t - stats.t.ppf(0.5 * alpha, df)), abs(t - stats.t.ppf(1.0 - 0.5 * alpha, df)))
        return t, (p < 0.5 * alpha) or (up < 0.5 * alpha), margin
    return t, abs(d) <= C, abs(t)


def _normal_ok(x, a):
    """Normality not rejected at level a (Jarque-Bera, chi^2 with 2 df)."""
    return not (math.exp(-0.5 * stats.jarque_bera(x).statistic) < a)


def _pixel_loop(x_ref, x_cur_full, P, mode, welch, m_ref_fixed=None):
    """One pixel of one pair: x_ref holds the first instant's logs (all of
    them in lock step, or a fixed reference of m_ref_fixed samples);
    returns (paths at the second instant, stopped early, margin, polarity)."""
    mb, spp_max = P["minibatch"], P["spp_max"]
    C, alpha = float(F32(P["C"])), float(F32(P["alpha"]))
    n = P["spp_init"]
    margin = math.inf
    while True:
        m1 = n // mb
        x0 = x_ref[:m_ref_fixed] if m_ref_fixed else x_ref[:m1]
        x1 = x_cur_full[:m1]
        if n >= spp_max:
            t = _eq7(x0, x1, C)
            margin = min(margin, abs(t))
            stop = False
            break
        t, stop, mg = _test(x0, x1, C, alpha, mode, welch)
        margin = min(margin, mg)
        a_n = float(F32(P.get("normality_alpha", 0.0)))
        if stop and a_n > 0 and not (_normal_ok(x0, a_n) and _normal_ok(x1, a_n)):
            stop = False
        if stop:
            break
        n = min(n + P["spp_batch"], spp_max)
    gap = x1.mean() - x0.mean()
    pol = (1 if gap > 0 else -1) if abs(gap) > C else 0
    return n, stop, margin, pol, x1


def _all_logs(f, params, P, pixels, instant):
    spp = P["spp_max"]
    px = np.repeat(pixels, spp)
    sm = np.tile(np.arange(spp, dtype=np.uint32), len(pixels))
    L = f.paths(params, px, instant, sm).reshape(len(pixels), spp)
    return [_mb_logs(L[i], P["minibatch"], P["log_eps"]) for i in range(len(pixels))]


@pytest.mark.parametrize("variant", ["1t", "welch", "2t", "mean_only", "ref_full", "normality"])
def test_render_loop_and_margin_match_python_rerun(variant):
    """Sample counts, early stops, polarity and the exemption margin of
    every pixel of a 16x12 frame equal a Python rerun of Algorithm 1 with
    scipy's tests on the same path radiances."""
    sc = scenes.tiny_box(width=16, height=12)
    mode = {"2t": oracle.MODE_ADAPTIVE_2T, "mean_only": oracle.MODE_MEAN_ONLY}.get(variant, oracle.MODE_ADAPTIVE_1T)
    welch = variant == "welch"
    P = dict(scenes.TINY_PARAMS, spp_max=128, mode=mode, df_mode=int(welch),
             ref_mode=oracle.REF_FULL if variant == "ref_full" else oracle.REF_LOCKSTEP,
             normality_alpha=0.05 if variant == "normality" else 0.0)
    params = oracle.make_params(**P)
    pixels = np.arange(16 * 12, dtype=np.uint32)
    with oracle.Frame(sc, 0.0, 1.0) as f:
        out = f.render(params, pixels)
        x0s = _all_logs(f, params, P, pixels, 0)
        x1s = _all_logs(f, params, P, pixels, 1)
    m_ref = P["spp_max"] // P["minibatch"] if variant == "ref_full" else None
    stops = 0
    for i in range(len(pixels)):
        n, stop, margin, pol, _ = _pixel_loop(x0s[i], x1s[i], P, mode, welch, m_ref)
        got = out["crit_margin"][i]
        assert got == margin or abs(got - margin) <= 1e-8 * max(1.0, margin), (i, got, margin)
        if variant != "normality":
            assert out["near_crit"][i] == (out["crit_margin"][i] < 1e-4)
        if out["near_crit"][i]:
            continue
        if margin < 1e-6:
            continue   # both answers are legitimate within rounding of the boundary
        assert out["n_paths"][i] == n and out["decided_early"][i] == stop and out["polarity"][i] == pol, i
        stops += stop
    assert stops > 0
    if variant == "normality":
        # the pre-test holds back some stops the t-test alone would make
        plain = dict(P, normality_alpha=0.0)
        with oracle.Frame(sc, 0.0, 1.0) as f:
            ref = f.render(oracle.make_params(**plain), pixels)
        assert out["decided_early"].sum() < ref["decided_early"].sum()
        assert (out["n_paths"] >= ref["n_paths"]).all()


def test_two_tailed_video_carries_reference_counts():
    """Sequential video with the two-tailed rule: an upper-tail stop fires an
    event before spp_max and the reference then holds that frame's samples
    up to its stop; every later frame is tested against that count (df =
    m_ref + m - 2).  Checked against a Python rerun on the oracle's paths."""
    sc = scenes.tiny_box(width=16, height=12)
    times = [0.0, 1.0, 2.0, 3.0]   # the cube keeps its last key position after t = 1
    P = dict(scenes.TINY_PARAMS, spp_max=128, mode=oracle.MODE_ADAPTIVE_2T, C=0.05)
    params = oracle.make_params(**P)
    pixels = np.arange(16 * 12, dtype=np.uint32)
    v = oracle.render_video(sc, times, params, pixels)
    mb = P["minibatch"]
    # Frame logs: frame q is instant 1 of pair q (keys key_base + q), frame 0
    # is instant 0 of pair 1.
    logs = []
    for q in range(len(times)):
        k = max(q, 1)
        with oracle.Frame(sc, times[k - 1], times[k]) as f:
            pk = oracle.make_params(**dict(P, key_base=k - 1))
            logs.append(_all_logs(f, pk, P, pixels, 0 if q == 0 else 1))
    early_events = 0
    for i in range(len(pixels)):
        ref = logs[0][i]
        m_ref = P["spp_max"] // mb
        for k in range(1, len(times)):
            n, stop, margin, pol, x1 = _pixel_loop(ref, logs[k][i], P, oracle.MODE_ADAPTIVE_2T, False, m_ref)
            o = {key: v[key][k - 1][i] for key in ("n_paths", "n_paths_ref", "polarity", "near_crit")}
            if o["near_crit"] or margin < 1e-6:
                break   # from here on the reference may legitimately differ
            assert o["n_paths_ref"] == m_ref * mb
            assert o["n_paths"] == n and o["polarity"] == pol, (i, k)
            if pol != 0:
                early_events += n < P["spp_max"]
                ref, m_ref = x1, n // mb
    assert early_events > 0, "the scene must produce upper-tail events before spp_max"
