/*
 * evo_stats.c -- oracle: counter-based RNG, Student t distribution, and the
 * per-pixel statistics and decision of the adaptive sampler.
 * TEST INFRASTRUCTURE ONLY (see evo.h).
 */
#include "evo.h"

#include <math.h>
#include <stdlib.h>

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2,
 * 3", SC'11).  One round multiplies counter words 0 and 2 by the two round
 * multipliers, and the new counter is (hi(c2*M1) ^ c1 ^ k0, lo(c2*M1),
 * hi(c0*M0) ^ c3 ^ k1, lo(c0*M0)).  The key is bumped by the two Weyl
 * constants between rounds. */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void evo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in [0, 1 - 2^-24]: the top 24 bits scaled by 2^-24 (exact). */
float evo_u01(uint32_t x)
{
    return (float)(x >> 8) * 0x1p-24f;
}

/* ---------------------------------------------------------------------- */
/* Regularized incomplete beta I_x(a, b), evaluated with the continued
 * fraction for the incomplete beta function (DLMF 8.17.22) by the modified
 * Lentz method, using the symmetry I_x(a,b) = 1 - I_{1-x}(b,a) on the side
 * where the fraction converges fast. */
static double ibeta_cf(double a, double b, double x)
{
    const double tiny = 1e-300;
    double c = 1.0;
    double d = 1.0 - (a + b) * x / (a + 1.0);
    if (fabs(d) < tiny) d = tiny;
    d = 1.0 / d;
    double f = d;
    for (int m = 1; m < 100000; ++m) {
        double md = (double)m;
        /* even step: d_{2m} = m (b - m) x / ((a + 2m - 1)(a + 2m)) */
        double num = md * (b - md) * x / ((a + 2.0 * md - 1.0) * (a + 2.0 * md));
        d = 1.0 + num * d;
        if (fabs(d) < tiny) d = tiny;
        c = 1.0 + num / c;
        if (fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        f *= d * c;
        /* odd step: d_{2m+1} = -(a + m)(a + b + m) x / ((a + 2m)(a + 2m + 1)) */
        num = -(a + md) * (a + b + md) * x / ((a + 2.0 * md) * (a + 2.0 * md + 1.0));
        d = 1.0 + num * d;
        if (fabs(d) < tiny) d = tiny;
        c = 1.0 + num / c;
        if (fabs(c) < tiny) c = tiny;
        d = 1.0 / d;
        double delta = d * c;
        f *= delta;
        if (fabs(delta - 1.0) < 1e-16) break;
    }
    return f;
}

/* I_x(a, b) given both x and y = 1 - x, so that x close to 1 keeps full
 * relative precision in y. */
static double ibeta_xy(double a, double b, double x, double y)
{
    if (!(x > 0.0)) return 0.0;
    if (!(y > 0.0)) return 1.0;
    double log_front = lgamma(a + b) - lgamma(a) - lgamma(b) + a * log(x) + b * log(y);
    double front = exp(log_front);
    if (x < (a + 1.0) / (a + b + 2.0))
        return front * ibeta_cf(a, b, x) / a;
    return 1.0 - front * ibeta_cf(b, a, y) / b;
}

double evo_ibeta(double a, double b, double x)
{
    return ibeta_xy(a, b, x, 1.0 - x);
}

/* Lower-tail CDF of Student's t with df degrees of freedom:
 * F(t) = I_{df/(df+t^2)}(df/2, 1/2) / 2 for t < 0, 1 - that for t > 0. */
double evo_t_cdf(double t, double df)
{
    if (isnan(t) || !(df > 0.0)) return NAN;
    if (isinf(t)) return t < 0.0 ? 0.0 : 1.0;
    double t2 = t * t;
    double x = df / (df + t2);
    double y = t2 / (df + t2);
    double tail = 0.5 * ibeta_xy(0.5 * df, 0.5, x, y);
    return t < 0.0 ? tail : 1.0 - tail;
}

/* Quantile by bisection on the CDF (slow and plain). */
double evo_t_ppf(double p, double df)
{
    if (!(p > 0.0) || !(p < 1.0) || !(df > 0.0)) return NAN;
    if (p == 0.5) return 0.0;
    double lo, hi;
    if (p < 0.5) {
        hi = 0.0;
        lo = -1.0;
        while (evo_t_cdf(lo, df) > p) lo *= 2.0;
    } else {
        lo = 0.0;
        hi = 1.0;
        while (evo_t_cdf(hi, df) < p) hi *= 2.0;
    }
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        if (evo_t_cdf(mid, df) < p) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ---------------------------------------------------------------------- */
/* Sample mean and unbiased variance, two-pass, FP64 (calcMeanVar of
 * Algorithm 1; Eq. 3-4 read as the sample estimates with Bessel's
 * correction). */
static void mean_var(const double *x, uint32_t m, double *mean, double *var)
{
    double s = 0.0;
    for (uint32_t k = 0; k < m; ++k) s += x[k];
    double mu = s / (double)m;
    double q = 0.0;
    for (uint32_t k = 0; k < m; ++k) {
        double dx = x[k] - mu;
        q += dx * dx;
    }
    *mean = mu;
    *var = m > 1 ? q / (double)(m - 1) : 0.0;
}

/* Normality of a pixel's log-luminance samples (the pre-test suggested in
 * Sec. 5 for small sample counts).  The paper names Shapiro-Wilk and
 * Kolmogorov-Smirnov as examples; the Jarque-Bera test (Jarque and Bera
 * 1980) is used because it needs only central moments, which a one-pass
 * accumulator can carry: JB = m/6 (g1^2 + g2^2 / 4) with g1 = m3 / m2^(3/2),
 * g2 = m4 / m2^2 - 3 and m_k = (1/m) sum (x - mean)^k; under normality JB
 * is asymptotically chi^2 with 2 degrees of freedom, P(JB > x) = exp(-x/2).
 * Plain two-pass sums here. */
double evo_jarque_bera(const double *x, uint32_t m)
{
    double s = 0.0;
    for (uint32_t k = 0; k < m; ++k) s += x[k];
    const double mu = s / (double)m;
    double c2 = 0.0, c3 = 0.0, c4 = 0.0;
    for (uint32_t k = 0; k < m; ++k) {
        const double dx = x[k] - mu;
        const double d2 = dx * dx;
        c2 += d2;
        c3 += d2 * dx;
        c4 += d2 * d2;
    }
    const double m2 = c2 / (double)m, m3 = c3 / (double)m, m4 = c4 / (double)m;
    if (!(m2 > 0.0)) return 0.0;
    const double g1sq = (m3 * m3) / (m2 * m2 * m2);
    const double g2 = m4 / (m2 * m2) - 3.0;
    return (double)m / 6.0 * (g1sq + 0.25 * g2 * g2);
}

/* The pre-test at level a: normality rejected when P(JB > jb) = exp(-jb/2)
 * < a.  *margin (relative distance of jb from the critical value -2 ln a)
 * is lowered for the exemption band. */
static int normality_rejected(const double *x, uint32_t m, double a, double *margin)
{
    const double jb = evo_jarque_bera(x, m);
    const double crit = -2.0 * log(a);
    const double mg = fabs(jb - crit) / (crit > 1.0 ? crit : 1.0);
    if (mg < *margin) *margin = mg;
    return exp(-0.5 * jb) < a;
}

/* Eq. 7: t = (|mu_b - mu_a| - C) / sqrt((s_a^2 + s_b^2) / N) with N the
 * sample count at the second instant.  A zero variance sum gives -inf, +inf
 * or 0 according to the sign of |mu_b - mu_a| - C. */
static double t_value(double mean0, double var0, double mean1, double var1,
                      uint32_t m1, double C)
{
    double gap = fabs(mean1 - mean0) - C;
    double S = var0 + var1;
    if (S == 0.0) {
        if (gap < 0.0) return -INFINITY;
        if (gap > 0.0) return INFINITY;
        return 0.0;
    }
    return gap / sqrt(S / (double)m1);
}

static double t_df(double var0, uint32_t m0, double var1, uint32_t m1, int df_mode)
{
    double pooled = (double)m0 + (double)m1 - 2.0;
    if (df_mode != EVO_DF_WELCH) return pooled;
    double S = var0 + var1;
    double den = var0 * var0 / (double)(m0 - 1) + var1 * var1 / (double)(m1 - 1);
    if (!(den > 0.0)) return pooled;
    return S * S / den;
}

/* Stopping rule after a batch (Sec. 3.2).  One-tailed: stop when the lower
 * tail p-value of t is below alpha ("gap significantly smaller than C", no
 * event).  Two-tailed: alpha/2 in each tail.  Mean-only: stop once the gap
 * is at most C.  Fixed: never stop. */
static int stop_rule(int mode, double t, double p_lower, double gap_abs, double C,
                     double alpha)
{
    switch (mode) {
    case EVO_MODE_ADAPTIVE_1T: return p_lower < alpha;
    case EVO_MODE_ADAPTIVE_2T: return p_lower < 0.5 * alpha || (1.0 - p_lower) < 0.5 * alpha;
    case EVO_MODE_MEAN_ONLY: return gap_abs <= C;
    default: (void)t; return 0;
    }
}

/* Exemption margin of one executed decision: the distance of t from the
 * critical value(s) that decide it, so that a pixel whose t lies within
 * rounding noise of a boundary may legitimately go either way.  At the last
 * count only the event rule |gap| > C applies, i.e. the boundary t = 0.
 * One-tailed: t_alpha(df); two-tailed: t_{alpha/2}(df) and
 * t_{1-alpha/2}(df); mean-only: |gap| <= C, again t = 0; fixed mode tests
 * nothing before the last count. */
double evo_crit_margin(int mode, double t, double df, float alpha, int final_check)
{
    if (final_check) return fabs(t);
    switch (mode) {
    case EVO_MODE_ADAPTIVE_1T: return fabs(t - evo_t_ppf((double)alpha, df));
    case EVO_MODE_ADAPTIVE_2T: {
        double lo = fabs(t - evo_t_ppf(0.5 * (double)alpha, df));
        double hi = fabs(t - evo_t_ppf(1.0 - 0.5 * (double)alpha, df));
        return lo < hi ? lo : hi;
    }
    case EVO_MODE_MEAN_ONLY: return fabs(t);
    default: return INFINITY;
    }
}

int evo_decide(const double *x0, uint32_t m0, const double *x1, uint32_t m1,
               float C, float alpha, int df_mode, int mode,
               double *t_out, double *p_out, double *df_out, int *stop_out, double *margin_out)
{
    if (m0 < 2 || m1 < 2) return -1;
    double mean0, var0, mean1, var1;
    mean_var(x0, m0, &mean0, &var0);
    mean_var(x1, m1, &mean1, &var1);
    double t = t_value(mean0, var0, mean1, var1, m1, (double)C);
    double df = t_df(var0, m0, var1, m1, df_mode);
    double p = evo_t_cdf(t, df);
    *t_out = t;
    *p_out = p;
    *df_out = df;
    *stop_out = stop_rule(mode, t, p, fabs(mean1 - mean0), (double)C, (double)alpha);
    if (margin_out) *margin_out = evo_crit_margin(mode, t, df, alpha, 0);
    return 0;
}

/* Internal entry for the render loop (same arithmetic as evo_decide). */
void evo__stats_decide(const double *x0, uint32_t m0, const double *x1, uint32_t m1,
                       const evo_params *p, double *mean, double *var, double *t_out,
                       double *df_out, double *p_out, int *stop_out, double *norm_margin)
{
    mean_var(x0, m0, &mean[0], &var[0]);
    mean_var(x1, m1, &mean[1], &var[1]);
    double t = t_value(mean[0], var[0], mean[1], var[1], m1, (double)p->C);
    double df = t_df(var[0], m0, var[1], m1, p->df_mode);
    double pl = evo_t_cdf(t, df);
    *t_out = t;
    *df_out = df;
    *p_out = pl;
    *stop_out = stop_rule(p->mode, t, pl, fabs(mean[1] - mean[0]), (double)p->C,
                          (double)p->alpha);
    /* The pre-test gates an early stop only: a pixel the t-test would stop
     * goes on sampling while either instant's samples reject normality. */
    if (*stop_out && p->normality_alpha > 0.0f) {
        const double a = (double)p->normality_alpha;
        const int r0 = normality_rejected(x0, m0, a, norm_margin);
        const int r1 = normality_rejected(x1, m1, a, norm_margin);
        if (r0 || r1) *stop_out = 0;
    }
}
