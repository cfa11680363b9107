"""Pins of the oracle's Student t distribution and the decision of Eq. 7."""
import math

import numpy as np
import pytest
from scipy import special, stats

import oracle

DFS = [1, 2, 3, 6, 14, 30, 126, 510, 2046]


@pytest.mark.parametrize("df", DFS)
def test_t_cdf_matches_scipy(df):
    ts = np.concatenate([np.linspace(-40, 40, 161), [-3.1427, -2.3563, -1e-9, 0.0, 1e-9, 1e6, -1e6]])
    for t in ts:
        assert abs(oracle.t_cdf(t, df) - stats.t.cdf(t, df)) < 1e-12, (t, df)


def test_t_cdf_closed_forms():
    for t in np.linspace(-25, 25, 101):
        # df = 1 is the Cauchy distribution; df = 2 has an algebraic CDF.
        assert abs(oracle.t_cdf(t, 1) - (0.5 + math.atan(t) / math.pi)) < 1e-13
        assert abs(oracle.t_cdf(t, 2) - (0.5 + t / (2.0 * math.sqrt(2.0 + t * t)))) < 1e-13
    for t in np.linspace(-6, 6, 49):
        # Large df tends to the standard normal.
        phi = 0.5 * math.erfc(-t / math.sqrt(2.0))
        assert abs(oracle.t_cdf(t, 1e8) - phi) < 1e-7


def test_t_cdf_limits_and_symmetry():
    assert oracle.t_cdf(-math.inf, 10) == 0.0
    assert oracle.t_cdf(math.inf, 10) == 1.0
    assert oracle.t_cdf(0.0, 7) == 0.5
    for t in (0.3, 1.7, 4.0):
        assert abs(oracle.t_cdf(t, 9) + oracle.t_cdf(-t, 9) - 1.0) < 1e-14
    assert math.isnan(oracle.t_cdf(math.nan, 3))


@pytest.mark.parametrize("df", DFS)
@pytest.mark.parametrize("p", [1e-4, 0.001, 0.005, 0.01, 0.05, 0.3, 0.99])
def test_t_ppf_matches_scipy(df, p):
    q = oracle.t_ppf(p, df)
    ref = stats.t.ppf(p, df)
    assert abs(q - ref) <= 1e-9 * max(1.0, abs(ref))


def test_t_ppf_sanity_values():
    # Critical values used by the tiny and sensor schedules.
    assert abs(oracle.t_ppf(0.99, 6) - 3.1427) < 1e-4
    assert abs(oracle.t_ppf(0.99, 126) - 2.3563) < 1e-4
    assert abs(oracle.t_ppf(0.999, 6) - 5.2076) < 1e-4
    assert abs(oracle.t_ppf(0.95, 510) - 1.6478) < 1e-4


def test_ibeta_matches_scipy():
    rng = np.random.default_rng(3)
    for _ in range(300):
        a = float(rng.uniform(0.3, 1500))
        b = float(rng.choice([0.5, rng.uniform(0.2, 50)]))
        x = float(rng.uniform(0, 1))
        assert abs(oracle.ibeta(a, b, x) - special.betainc(a, b, x)) < 1e-11
    assert oracle.ibeta(2, 3, 0.0) == 0.0 and oracle.ibeta(2, 3, 1.0) == 1.0


# --------------------------------------------------------------------------
# The decision on seeded Gaussian log-luminance data (Eq. 7, Sec. 3.2).

def _scipy_t(x0, x1, C, equal_var):
    """Equal-size samples: Eq. 7 is the two-sample t statistic of
    H0: |mu1 - mu0| = C against the alternative "smaller"."""
    if x1.mean() >= x0.mean():
        r = stats.ttest_ind(x1 - C, x0, equal_var=equal_var, alternative="less")
    else:
        r = stats.ttest_ind(x0 - C, x1, equal_var=equal_var, alternative="less")
    return r.statistic, r.pvalue


@pytest.mark.parametrize("m", [4, 16, 64])
@pytest.mark.parametrize("gap_frac", [0.0, 0.5, 1.0, 2.0, -1.0])
@pytest.mark.parametrize("welch", [False, True])
def test_decision_matches_scipy_ttest(m, gap_frac, welch):
    C = 0.2
    rng = np.random.default_rng(1234 + m)
    for rep in range(20):
        x0 = rng.normal(0.0, 0.05, size=m)
        x1 = rng.normal(gap_frac * C, 0.05 * (1.0 + 0.5 * rep / 20), size=m)
        r = oracle.decide(x0, x1, np.float32(C), np.float32(0.01), df_mode=int(welch))
        Cd = float(np.float32(C))
        t_ref, p_ref = _scipy_t(x0, x1, Cd, equal_var=not welch)
        assert abs(r["t"] - t_ref) <= 1e-10 * max(1.0, abs(t_ref))
        assert abs(r["p"] - p_ref) <= 1e-10
        if not welch:
            assert r["df"] == 2 * m - 2
        assert r["stop"] == (p_ref < float(np.float32(0.01)))


def test_decision_zero_variance_cases():
    x = np.full(8, 0.75)  # exactly representable, so the two-pass variance is exactly 0
    r = oracle.decide(x, x, 0.2, 0.01)          # gap 0 < C: certain no-event
    assert r["t"] == -math.inf and r["p"] == 0.0 and r["stop"]
    r = oracle.decide(x, x + 0.5, 0.2, 0.01)    # gap > C: certain event, no stop
    assert r["t"] == math.inf and not r["stop"]
    r = oracle.decide(x, x, 0.0, 0.01)          # gap == C: t = 0, p = 1/2
    assert r["t"] == 0.0 and r["p"] == 0.5 and not r["stop"]


def test_decision_modes():
    rng = np.random.default_rng(5)
    x0 = rng.normal(0, 0.05, 16)
    far = oracle.decide(x0, x0 + 1.0, 0.2, 0.01, mode=oracle.MODE_ADAPTIVE_2T)
    assert far["stop"]                       # two-tailed also stops on a sure event
    assert not oracle.decide(x0, x0 + 1.0, 0.2, 0.01)["stop"]
    assert oracle.decide(x0, x0 + 0.1, 0.2, 0.01, mode=oracle.MODE_MEAN_ONLY)["stop"]
    assert not oracle.decide(x0, x0 + 0.3, 0.2, 0.01, mode=oracle.MODE_MEAN_ONLY)["stop"]
    assert not oracle.decide(x0, x0, 0.2, 0.01, mode=oracle.MODE_FIXED)["stop"]


def test_stop_rate_calibration_at_threshold():
    """With the true gap exactly C, the one-tailed test stops with
    probability alpha (binomial 99.9% interval over many pixels)."""
    rng = np.random.default_rng(99)
    C, alpha, m, n = 0.2, 0.05, 16, 20000
    x0 = rng.normal(0.0, 0.05, size=(n, m))
    x1 = rng.normal(float(np.float32(C)), 0.05, size=(n, m))
    stops = sum(oracle.decide(x0[i], x1[i], C, alpha)["stop"] for i in range(n))
    a = float(np.float32(alpha))
    sd = math.sqrt(n * a * (1 - a))
    assert abs(stops - n * a) < 3.3 * sd
