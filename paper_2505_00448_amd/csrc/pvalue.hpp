// Two-sided p-value of a correlation coefficient, FP64.
//
// NApy (arXiv 2505.00448) takes Pearson's p from the Beta CDF (Section 3.5.2)
// and Spearman's from the t distribution (Section 3.5.3).  Under the null the
// coefficient r on [-1, 1] follows Beta(n/2 - 1, n/2 - 1), and the two-sided
// tail is the regularized incomplete beta function
//
//     p = I_{1 - r^2}(a, 1/2),   a = (n - 2) / 2,
//
// which is also the two-sided Student-t tail with n - 2 degrees of freedom.
//
// Method: the continued fraction of I_x(a, b) (Abramowitz & Stegun 26.5.8),
// evaluated by the forward recurrences of its convergents after an
// equivalence transformation that leaves no division in the loop.  It converges fast for x < (a + 1) / (a + b + 2); otherwise the
// symmetry I_x(a, b) = 1 - I_{1-x}(b, a) is used, so the tail that is computed
// directly is the small one (for p the complement is kept a little beyond
// that point, see corr_p_params).  The prefactor x^a (1-x)^b / (a B(a,b)) is
// formed in logs.  ln B(a, 1/2) = ln(sqrt(pi)) - [ln G(a + 1/2) - ln G(a)];
// for a >= 20 the bracket is evaluated as 0.5 ln a plus the asymptotic series
// obtained from Stirling's series of both log-gammas (so no two large
// log-gammas are subtracted), below that from lgamma directly; the factors
// |r| and a^(+-1/2) multiply the exponential instead of entering its
// argument as logarithms.
//
// Compiled for host and device: the host copy serves only to unit-test the
// arithmetic on a machine without a GPU.
#pragma once

#include <math.h>
#include <stdint.h>

#ifndef NAPY_HD
#define NAPY_HD __host__ __device__
#endif

namespace napy {

// 1/x: on the device the hardware reciprocal refined by two Newton steps
// (full double precision without the IEEE division sequence); on the host a
// plain division.
NAPY_HD inline double recip(double x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
    r = fma(fma(-x, r, 1.0), r, r);
    r = fma(fma(-x, r, 1.0), r, r);
    return r;
#else
    return 1.0 / x;
#endif
}

// ln G(a + 1/2) - ln G(a) - ln(a) / 2 for a >= 20: Stirling's series of the
// two log-gammas, -1/(8a) + 1/(192a^3) - 1/(640a^5) + 17/(14336a^7) -
// 31/(18432a^9) (the next term is below 1e-17 there)
NAPY_HD inline double lgamma_half_ratio_tail(double a)
{
    const double ia = recip(a);
    const double ia2 = ia * ia;
    double s = -31.0 / 18432.0;
    s = s * ia2 + 17.0 / 14336.0;
    s = s * ia2 - 1.0 / 640.0;
    s = s * ia2 + 1.0 / 192.0;
    s = s * ia2 - 1.0 / 8.0;
    return s * ia;
}

// Continued fraction of I_x(a, b) (A&S 26.5.8): I_x(a, b) = x^a (1-x)^b /
// (a B(a, b)) * h, h = 1 / (1 + e_1 / (1 + e_2 / (1 + ...))), with the
// partial numerators e_j = p_j / (d_{j-1} d_j), d_m = a + m, p_{2k} = k (b -
// k) x and p_{2k+1} = -(a + k)(a + b + k) x.
//
// Evaluation: the fundamental recurrences of the convergents A_n / B_n of a
// continued fraction (A_n = b_n A_{n-1} + a_n A_{n-2}, the same for B), after
// the equivalence transformation that multiplies the n-th partial
// denominator by d_{n-1} (n >= 2).  The transformed fraction has partial
// numerators p_j (and -(a + b) x for j = 1) and partial denominators d_j, so
// that each term is
//
//     A <- d_j A + p_j A_prev,   B <- d_j B + p_j B_prev
//
// (two products and two fused multiply-adds, no division), starting from
// A_0 = 0, A_1 = 1, B_0 = B_1 = 1.  The four values grow by about d_j per
// term; after each pair of terms all four are scaled by the power of two
// that brings B near one (exact, and the ratio A / B is unchanged).  Two
// successive convergents differ by W_n / (B_n B_{n-1}), where the
// determinant W_n = A_n B_{n-1} - A_{n-1} B_n obeys W_n = -p W_{n-1} for the
// term's partial numerator p: it is carried as a product (so the difference
// is known without the cancellation of forming it from A and B), and the
// fraction has converged when |W| < CF_EPS |A_{n-1} B_n|; h = A / B at the
// end.  CfState holds the two latest convergents, W and the index k of the
// next pair of terms, so a caller can interleave the steps of several
// evaluations.
struct CfState {
    double a, b, x;
    double A, Ap, B, Bp;  // latest and previous convergent
    double W;             // A Bp - Ap B
    int k;
};

constexpr double CF_EPS = 1e-16;
constexpr int CF_MAXK = 2000;

NAPY_HD inline void cf_start(CfState& s, double a, double b, double x)
{
    s.a = a;
    s.b = b;
    s.x = x;
    // the first term, e_1 = -(a + b) x / (a (a + 1)), transformed
    s.Ap = 1.0;
    s.Bp = 1.0;
    s.A = a + 1.0;
    s.B = fma(-(a + b), x, a + 1.0);
    s.W = (a + b) * x;
    s.k = 1;
}

// terms 2k and 2k + 1, then the scaling; true once the last two convergents
// agree to CF_EPS (or after CF_MAXK pairs)
NAPY_HD inline bool cf_advance(CfState& s)
{
    const double kk = (double)s.k, k2 = kk + kk;
    const double a = s.a, b = s.b, x = s.x;
    // term 2k: d = a + 2k, p = k (b - k) x
    const double de = a + k2, pe = kk * (b - kk) * x;
    double A = fma(pe, s.Ap, de * s.A), B = fma(pe, s.Bp, de * s.B);
    s.Ap = s.A;
    s.Bp = s.B;
    // term 2k + 1: d = a + 2k + 1, p = -(a + k)(a + b + k) x
    const double dq = de + 1.0, pq = -((a + kk) * (a + b + kk) * x);
    const double An = fma(pq, s.A, dq * A), Bn = fma(pq, s.B, dq * B);
    // An / Bn - A / B = W / (B Bn)
    const double W = s.W * (pe * pq);
    const bool done = fabs(W) < CF_EPS * fabs(A * Bn) || s.k >= CF_MAXK;
    // scale by 2^-e, e the exponent of Bn (Bn = 0 leaves the values as they
    // are); W is bilinear in them
    int e = 0;
    (void)frexp(Bn, &e);
    s.A = ldexp(An, -e);
    s.B = ldexp(Bn, -e);
    s.Ap = ldexp(A, -e);
    s.Bp = ldexp(B, -e);
    s.W = ldexp(W, -2 * e);
    ++s.k;
    return done;
}

// the continued-fraction factor h of I_x(a, b) = x^a (1-x)^b / (a B(a, b)) h
NAPY_HD inline double betacf(double a, double b, double x)
{
    CfState s;
    cf_start(s, a, b, x);
    while (!cf_advance(s)) {
    }
    return s.A / s.B;
}

// Setup of p = I_{1-r^2}((n-2)/2, 1/2) for n >= 3 and finite r: either a
// value that needs no continued fraction (done), or the fraction's
// parameters (a, b, x), the log of its prefactor and the tail (direct: p is
// the prefactor times the fraction; otherwise 1 minus it).  The parameters
// are chosen first so that one continued-fraction loop serves both tails
// (lanes of a wave taking different tails do not run two loops).
struct CorrPSetup {
    double a, b, x, lf, m, value;
    bool done, direct;
};

// The fraction's parameters and the tail alone (no logarithms): what a
// caller needs to start the continued fraction; lf is left zero.
NAPY_HD inline CorrPSetup corr_p_params(double r, int64_t n)
{
    CorrPSetup q;
    q.a = q.b = q.x = q.lf = 0.0;
    q.m = 1.0;
    q.direct = true;
    q.done = true;
    q.value = NAN;
    if (!(r == r) || n < 3) return q;
    const double ar = fabs(r);
    if (ar >= 1.0) {
        q.value = 0.0;
        return q;
    }
    if (ar == 0.0) {
        q.value = 1.0;
        return q;
    }
    const double a = 0.5 * (double)(n - 2);
    const double y = ar * ar;                 // r^2
    const double x = (1.0 - ar) * (1.0 + ar); // 1 - r^2 without cancellation
    // the direct tail I_x(a, 1/2), or 1 - I_{r^2}(1/2, a).  The usual switch,
    // direct for x < (a + 1) / (a + b + 2), i.e. r^2 (a + 2.5) > 1.5, leaves
    // the direct fraction's slowest region (up to about 48 steps at large a)
    // just above it.  For a >= 4 the complement is kept up to r^2 (a + 2.5)
    // = 3.75: its fraction takes at most about 15 steps there and the direct
    // one above at most about 25, while p stays above about 5e-3, so that
    // forming 1 - I loses at most two to three digits.
    const bool direct = (a >= 4.0) ? (y * (a + 2.5) >= 3.75) : (x < (a + 1.0) / (a + 2.5));
    q.a = direct ? a : 0.5;
    q.b = direct ? 0.5 : a;
    q.x = direct ? x : y;
    q.direct = direct;
    q.done = false;
    return q;
}

// The prefactor is m exp(lf).  With x = 1 - r^2, y = r^2 and ln B(a, 1/2) =
// ln(pi) / 2 - [ln G(a + 1/2) - ln G(a)], the direct tail's prefactor
// x^a y^(1/2) / (a B(a, 1/2)) is |r| exp(a ln x - ln a - ln B), and the
// complement's y^(1/2) x^a / ((1/2) B(1/2, a)) is 2 |r| exp(a ln x - ln B):
// |r| stays outside the exponential (no logarithm of it).  For a >= 20 the
// bracket is ln(a) / 2 plus Stirling's tail T(a), so that -ln a - ln B =
// T(a) - ln(pi a) / 2 and -ln B = T(a) + ln(a / pi) / 2: the square roots
// go into m as well, and the exponential's argument is a ln x + T(a) alone.
NAPY_HD inline CorrPSetup corr_p_setup(double r, int64_t n)
{
    CorrPSetup q = corr_p_params(r, n);
    if (q.done) return q;
    const double ar = fabs(r);
    const double a = 0.5 * (double)(n - 2);
    const double alnx = a * log1p(-(ar * ar));
    if (a >= 20.0) {
        constexpr double PI = 3.14159265358979323846;
        q.lf = alnx + lgamma_half_ratio_tail(a);
        q.m = q.direct ? ar * recip(sqrt(PI * a)) : 2.0 * ar * sqrt(a * (1.0 / PI));
    } else {
        const double lnB = 0.57236494292470008707 - (lgamma(a + 0.5) - lgamma(a));
        q.lf = q.direct ? alnx - log(a) - lnB : alnx + 0.69314718055994530942 - lnB;
        q.m = ar;
    }
    return q;
}

// p from the setup and the fraction's value h
NAPY_HD inline double corr_p_finish(const CorrPSetup& q, double h)
{
    const double t = q.m * exp(q.lf) * h;
    if (q.direct) return t;
    const double p = 1.0 - t;
    return p < 0.0 ? 0.0 : p;
}

// p = I_{1-r^2}((n-2)/2, 1/2) for n >= 3 and finite r; NaN otherwise.
NAPY_HD inline double corr_pvalue(double r, int64_t n)
{
    const CorrPSetup q = corr_p_setup(r, n);
    if (q.done) return q.value;
    return corr_p_finish(q, betacf(q.a, q.b, q.x));
}

// ln G(a + b) - ln G(a) for a, b > 0.  For a >= 20 from Stirling's series of
// both log-gammas, arranged so that nothing large cancels:
//   (a - 1/2) log1p(b/a) + b ln(a + b) - b + [s(a + b) - s(a)],
//   s(z) = 1/(12z) - 1/(360z^3) + 1/(1260z^5) - 1/(1680z^7)
// (the next term is below 1e-12 / z^9); below that from lgamma directly.
NAPY_HD inline double stirling_tail(double z)
{
    const double iz = 1.0 / z, iz2 = iz * iz;
    return iz * (1.0 / 12.0 - iz2 * (1.0 / 360.0 - iz2 * (1.0 / 1260.0 - iz2 * (1.0 / 1680.0))));
}

NAPY_HD inline double lgamma_ratio(double a, double b)
{
    if (a >= 20.0)
        return (a - 0.5) * log1p(b / a) + b * log(a + b) - b + (stirling_tail(a + b) - stirling_tail(a));
    return lgamma(a + b) - lgamma(a);
}

// Survival function of Fisher's F distribution with d1, d2 > 0 degrees of
// freedom: P(F' > f) = I_x(d2/2, d1/2) with x = d2 / (d2 + d1 f) (its
// complement y = d1 f / (d2 + d1 f) is formed directly, not as 1 - x).  The
// continued fraction runs on the smaller tail, as in corr_pvalue; ln B(a, b) =
// ln G(s) - [ln G(s + l) - ln G(l)] with s, l the smaller and larger of a, b.
// The two-sided p of a t statistic with df degrees of freedom is
// fdist_sf(t^2, 1, df).  f = +inf gives 0, f <= 0 gives 1, NaN gives NaN.
NAPY_HD inline double fdist_sf(double f, double d1, double d2)
{
    if (!(f == f) || !(d1 > 0.0) || !(d2 > 0.0)) return NAN;
    if (f <= 0.0) return 1.0;
    if (f == INFINITY) return 0.0;
    const double a = 0.5 * d2, b = 0.5 * d1;
    const double den = d2 + d1 * f;
    const double x = d2 / den, y = d1 * f / den;
    const double sm = a < b ? a : b, lg = a < b ? b : a;
    const double lnB = lgamma(sm) - lgamma_ratio(lg, sm);
    // ln x and ln y from the complement when it is the small one (x near 1
    // with a large a would otherwise lose digits)
    const double lnx = y < 0.5 ? log1p(-y) : log(x);
    const double lny = x < 0.5 ? log1p(-x) : log(y);
    // one continued-fraction loop for either tail, as in corr_pvalue
    const bool direct = x < (a + 1.0) / (a + b + 2.0);
    const double lf = direct ? a * lnx + b * lny - log(a) - lnB : b * lny + a * lnx - log(b) - lnB;
    const double t = exp(lf) * betacf(direct ? a : b, direct ? b : a, direct ? x : y);
    if (direct) return t;
    const double p = 1.0 - t;
    return p < 0.0 ? 0.0 : p;
}

// Regularized upper incomplete gamma Q(a, x) = Gamma(a, x) / Gamma(a), a > 0
// (A&S 6.5.3), with the prefactor e^-x x^a / Gamma(a) formed in logs.
//   x < a + 1: Q = 1 - P from the series of P (A&S 6.5.29), P = prefactor *
//     sum_{m >= 0} x^m / (a (a+1) ... (a+m)); its terms t_m = t_{m-1} x /
//     (a + m) are summed until one falls below 1e-17 of the sum.
//   otherwise: Q = prefactor * 1 / (x + 1 - a - 1 (1 - a) / (x + 3 - a -
//     2 (2 - a) / (x + 5 - a - ...))), the even contraction of A&S 6.5.31:
//     partial numerators -m (m - a), denominators x + 2m + 1 - a.  As for
//     the beta fraction above, by the forward recurrences of the convergents
//     (division-free: the coefficients are polynomials), rescaled by powers of
//     two and stopped from the running determinant W, which each term
//     multiplies by -(its partial numerator).
// The tail computed directly is the small one.
NAPY_HD inline double gamma_q(double a, double x)
{
    if (!(x == x) || !(a > 0.0)) return NAN;
    if (x <= 0.0) return 1.0;
    if (x == INFINITY) return 0.0;
    const double lpre = -x + a * log(x) - lgamma(a);
    if (x < a + 1.0) {
        double term = 1.0 / a, total = term, am = a;
        for (int m = 1; m <= 100000; ++m) {
            am += 1.0;
            term *= x / am;
            total += term;
            if (fabs(term) < fabs(total) * 1e-17) break;
        }
        const double q = 1.0 - total * exp(lpre);
        return q < 0.0 ? 0.0 : q;
    }
    // convergents: 0 / 1, then 1 / (x + 1 - a)
    const double d0 = x + 1.0 - a;
    double Ap = 0.0, Bp = 1.0, A = 1.0, B = d0, W = 1.0;
    for (int m = 1; m <= 100000; ++m) {
        const double num = -(double)m * ((double)m - a), den = fma(2.0, (double)m, d0);
        const double An = fma(num, Ap, den * A), Bn = fma(num, Bp, den * B);
        W *= -num;  // A_n B_{n-1} - A_{n-1} B_n
        const bool done = fabs(W) < CF_EPS * fabs(A * Bn);
        int e = 0;
        (void)frexp(Bn, &e);
        Ap = ldexp(A, -e);
        Bp = ldexp(B, -e);
        A = ldexp(An, -e);
        B = ldexp(Bn, -e);
        W = ldexp(W, -2 * e);
        if (done) break;
    }
    return exp(lpre) * (A / B);
}

// P(chi2_df > x) = Q(df / 2, x / 2)
NAPY_HD inline double chi2_sf(double x, double df) { return gamma_q(0.5 * df, 0.5 * x); }

}  // namespace napy
