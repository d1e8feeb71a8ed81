/*
 * CPU oracle for the modified Bessel function of the second kind and the
 * Matern covariance built from it.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg load this library. It shares no code, header, table or
 * constant generator with the GPU library; it is slow on purpose and written so
 * that each step can be checked against the paper by eye.
 *
 * What it computes (the plain definitions, not the paper's trapezoid):
 *   K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt,  x > 0       (Sec. IV-B, Eq. "integral")
 *   M(r)    = sigma2 / (2^(nu-1) Gamma(nu)) (r/beta)^nu K_nu(r/beta), M(0) = sigma2
 *                                                             (Sec. III-A, Matern formula; Alg. 3)
 * The integral is evaluated in x87 long double (64-bit significand) by globally
 * adaptive 7-point Gauss / 15-point Kronrod quadrature (Piessens et al., QUADPACK
 * 1983, routine QAG) applied to exp(g(t) - g_hat), where
 *   g(t) = log cosh(nu t) - x cosh t                        (Sec. IV-B, Eq. "logintegrand")
 * and g_hat = g(t_hat) is the log-integrand at a point found by golden-section
 * search. Factoring exp(g_hat) out is only a scale: any t_hat gives the same
 * integral, so the oracle does not depend on how precisely t_hat is located.
 *
 * A second, separate routine reproduces the integration window of Sec. IV-B
 * ({t : g(t) >= g(t_max) - L}) by bisection, for checking the GPU window export.
 *
 * Derivatives (the paper lists them as future work, Sec. VI) are the integrals
 * obtained by differentiating under the integral sign:
 *   dK/dx  = -int_0^inf cosh t exp(-x cosh t) cosh(nu t) dt
 *   dK/dnu =  int_0^inf t sinh(nu t) exp(-x cosh t) dt
 * evaluated by the same adaptive rule; and the gradient of the Matern covariance
 * in (beta, nu) written out with the chain rule.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include "gk15_table.h"

#define ORC_LN2 0.693147180559945309417232121458176568L

/* log cosh(y) for any real y without overflow. */
static long double orc_logcosh(long double y)
{
    y = fabsl(y);
    if (y < 16.0L) return logl(coshl(y));
    return y - ORC_LN2 + log1pl(expl(-2.0L * y));
}

/* g_{nu,x}(t) = log cosh(nu t) - x cosh(t)  (Sec. IV-B). */
static long double orc_g(long double nu, long double x, long double t)
{
    return orc_logcosh(nu * t) - x * coshl(t);
}

/* Maximiser of g over t >= 0. Sec. IV-B: g(0) = -x, g'(0) = 0; for nu^2 <= x the
 * log-integrand only decreases, so the maximum is at 0; otherwise it lies inside.
 * Inside, nu tanh(nu t) < nu bounds x sinh(t_max) from above, so
 * t_max < asinh(nu/x). g is unimodal there (tanh(nu t)/sinh t decreases), so a
 * golden-section search over [0, asinh(nu/x) + 1] finds it. */
static long double orc_tmax(long double nu, long double x)
{
    if (nu * nu <= x) return 0.0L;
    const long double ginv = 0.618033988749894848204586834365638118L;
    long double a = 0.0L, b = asinhl(nu / x) + 1.0L;
    long double c = b - ginv * (b - a), d = a + ginv * (b - a);
    long double gc = orc_g(nu, x, c), gd = orc_g(nu, x, d);
    for (int it = 0; it < 200 && (b - a) > 1e-15L * (1.0L + b); ++it) {
        if (gc > gd) { b = d; d = c; gd = gc; c = b - ginv * (b - a); gc = orc_g(nu, x, c); }
        else         { a = c; c = d; gc = gd; d = a + ginv * (b - a); gd = orc_g(nu, x, d); }
    }
    return 0.5L * (a + b);
}

/* Integrand kinds: 0 is the K integrand exp(g(t)); 1 multiplies it by cosh t
 * (-dK/dx); 2 by t tanh(nu t), so that the product is t sinh(nu t) exp(-x cosh t)
 * (dK/dnu). log of the extra factor: */
static long double orc_lfac(int kind, long double nu, long double t)
{
    if (kind == 1) return orc_logcosh(t);
    if (kind == 2) return logl(t) + logl(tanhl(nu * t));
    return 0.0L;
}

typedef struct { long double nu, x, that, lcref; int kind; long double lfref; } orc_integrand;

/* exp(g(t) - g(t_hat)). The difference is formed without cancellation:
 *   log cosh(nu t) - log cosh(nu t_hat) - 2 x sinh((t + t_hat)/2) sinh((t - t_hat)/2),
 * since cosh t - cosh t_hat = 2 sinh((t + t_hat)/2) sinh((t - t_hat)/2). Forming
 * g(t) - g(t_hat) from the two values instead leaves an absolute error of about
 * x * LDBL_EPSILON, which for x in the thousands is above the stopping tolerance. */
static long double orc_phi(const orc_integrand* f, long double t)
{
    long double d = orc_logcosh(f->nu * t) - f->lcref
                    - 2.0L * f->x * sinhl(0.5L * (t + f->that)) * sinhl(0.5L * (t - f->that));
    if (f->kind != 0) d += orc_lfac(f->kind, f->nu, t) - f->lfref;
    return expl(d);
}

/* One 15-point Kronrod evaluation on [a,b] with the embedded 7-point Gauss
 * value; returns the Kronrod value and |Kronrod - Gauss| as the error estimate. */
static long double orc_gk15(const orc_integrand* f, long double a, long double b, long double* err)
{
    const long double c = 0.5L * (a + b), hw = 0.5L * (b - a);
    long double fc = orc_phi(f, c);
    long double rk = GK15_WK[7] * fc, rg = GK15_WG[7] * fc;
    for (int j = 0; j < 7; ++j) {
        long double dx = hw * GK15_X[j];
        long double s = orc_phi(f, c - dx) + orc_phi(f, c + dx);
        rk += GK15_WK[j] * s;
        rg += GK15_WG[j] * s;
    }
    *err = fabsl((rk - rg) * hw);
    return rk * hw;
}

#define ORC_MAXSUB 4000

typedef struct { long double a, b, val, err; } orc_seg;

/* Globally adaptive quadrature over [a0,b0]: always bisect the segment with the
 * largest error estimate until the summed estimate is below reltol * |sum|.
 * Returns the integral; *ok is cleared if the subdivision limit was hit. */
static long double orc_adapt(const orc_integrand* f, long double a0, long double b0,
                             long double reltol, orc_seg* seg, int* ok)
{
    int ns = 1;
    seg[0].a = a0; seg[0].b = b0;
    seg[0].val = orc_gk15(f, a0, b0, &seg[0].err);
    for (;;) {
        long double tot = 0.0L, etot = 0.0L;
        int worst = 0;
        for (int i = 0; i < ns; ++i) {
            tot += seg[i].val;
            etot += seg[i].err;
            if (seg[i].err > seg[worst].err) worst = i;
        }
        if (etot <= reltol * fabsl(tot)) return tot;
        if (ns + 1 >= ORC_MAXSUB) { *ok = 0; return tot; }
        long double a = seg[worst].a, b = seg[worst].b, m = 0.5L * (a + b);
        seg[worst].b = m;
        seg[worst].val = orc_gk15(f, a, m, &seg[worst].err);
        seg[ns].a = m; seg[ns].b = b;
        seg[ns].val = orc_gk15(f, m, b, &seg[ns].err);
        ++ns;
    }
}

/* log K_nu(x) in long double for x > 0 (nu is used through |nu|: the integrand
 * is even in nu). Returns 0 in *ok when the adaptive rule did not converge. */
static long double orc_logk(long double nu, long double x, orc_seg* seg, int* ok)
{
    nu = fabsl(nu);
    orc_integrand f;
    f.nu = nu; f.x = x;
    f.kind = 0; f.lfref = 0.0L;
    long double th = orc_tmax(nu, x);
    f.that = th;
    f.lcref = orc_logcosh(nu * th);
    const long double gref = orc_g(nu, x, th);
    /* upper limit: step away from t_hat, doubling, until the integrand is
     * below e^-64 of its peak; past the peak g is decreasing. */
    long double step = 1.0L, T = th + step;
    while (logl(orc_phi(&f, T)) > -64.0L && step < 1e4L) { step *= 2.0L; T = th + step; }
    const long double tol = 1e-17L;
    long double I = 0.0L;
    if (th > 0.0L) I += orc_adapt(&f, 0.0L, th, tol, seg, ok);
    I += orc_adapt(&f, th, T, tol, seg, ok);
    return gref + logl(I);
}

/* Exported: K_nu(x) for n pairs, by OpenMP over entries.
 * logk[i]   = log K (NAN for x <= 0 or NaN input)
 * k[i]      = K    (+inf at x == 0, NaN for x < 0)
 * kscaled[i]= e^x K, the form that stays representable past x ~ 708
 * Any output pointer may be NULL. Returns the number of entries whose adaptive
 * rule hit its subdivision limit (0 when everything converged). */
int64_t oracle_besselk(const double* nu, const double* x, double* logk, double* k,
                       double* kscaled, int64_t n)
{
    int64_t bad = 0;
#pragma omp parallel reduction(+ : bad)
    {
        orc_seg* seg = (orc_seg*)malloc(sizeof(orc_seg) * ORC_MAXSUB);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            double xi = x[i], ni = nu[i];
            double lk, kk, ks;
            if (isnan(xi) || isnan(ni) || xi < 0.0) { lk = NAN; kk = NAN; ks = NAN; }
            else if (xi == 0.0) { lk = INFINITY; kk = INFINITY; ks = INFINITY; }
            else {
                int ok = 1;
                long double L = orc_logk((long double)ni, (long double)xi, seg, &ok);
                if (!ok) ++bad;
                lk = (double)L;
                kk = (double)expl(L);
                ks = (double)expl(L + (long double)xi);
            }
            if (logk) logk[i] = lk;
            if (k) k[i] = kk;
            if (kscaled) kscaled[i] = ks;
        }
        free(seg);
    }
    return bad;
}

/* Exported: selected Matern covariance entries (Sec. III-A; Alg. 3).
 * For entry e, the row location is (rx[ri[e]], ry[ri[e]]) and the column
 * location (cx[ci[e]], cy[ci[e]]). The distance is formed in long double from
 * the double inputs; an exact zero distance gives sigma2 (Alg. 3), otherwise
 * sigma2 * exp((1-nu) ln 2 - lgamma(nu) + nu ln(r/beta) + ln K_nu(r/beta)).
 * Returns the count of non-converged quadratures. */
int64_t oracle_matern(const double* rx, const double* ry, const double* cx, const double* cy,
                      const int64_t* ri, const int64_t* ci, int64_t n_entries,
                      double sigma2, double beta, double nu, double* out)
{
    int64_t bad = 0;
    const long double lnu = (long double)nu;
    const long double pre = (1.0L - lnu) * ORC_LN2 - lgammal(lnu);
#pragma omp parallel reduction(+ : bad)
    {
        orc_seg* seg = (orc_seg*)malloc(sizeof(orc_seg) * ORC_MAXSUB);
#pragma omp for schedule(dynamic, 16)
        for (int64_t e = 0; e < n_entries; ++e) {
            long double dx = (long double)cx[ci[e]] - (long double)rx[ri[e]];
            long double dy = (long double)cy[ci[e]] - (long double)ry[ri[e]];
            long double r = sqrtl(dx * dx + dy * dy);
            if (r == 0.0L) { out[e] = sigma2; continue; }
            long double z = r / (long double)beta;
            int ok = 1;
            long double lk = orc_logk(lnu, z, seg, &ok);
            if (!ok) ++bad;
            out[e] = (double)((long double)sigma2 * expl(pre + lnu * logl(z) + lk));
        }
        free(seg);
    }
    return bad;
}

/* Exported: the integration window of Sec. IV-B, [t0,t1] = {t >= 0 :
 * g(t) >= g(t_max) - L}, located by plain bisection in long double.
 *  t_max: sign of g'(t) = nu tanh(nu t) - x sinh t, bisected on [0, asinh(nu/x)+1]
 *  t0   : 0 if g(0) >= g(t_max) - L, else the crossing inside [0, t_max]
 *  t1   : the crossing beyond t_max, bracketed by doubling the step from t_max
 * Outputs t_max, g(t_max), t0, t1 as double. */
void oracle_window(const double* nu, const double* x, int64_t n, double L,
                   double* tmax, double* gmax, double* t0, double* t1)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        long double v = fabsl((long double)nu[i]), z = (long double)x[i];
        long double tm = 0.0L;
        if (v * v > z) {
            long double lo = 0.0L, hi = asinhl(v / z) + 1.0L;
            for (int it = 0; it < 200; ++it) {
                long double mid = 0.5L * (lo + hi);
                if (v * tanhl(v * mid) - z * sinhl(mid) > 0.0L) lo = mid; else hi = mid;
            }
            tm = 0.5L * (lo + hi);
        }
        long double gm = orc_g(v, z, tm), thr = gm - (long double)L;
        long double a = 0.0L;
        if (orc_g(v, z, 0.0L) < thr) {
            long double lo = 0.0L, hi = tm;
            for (int it = 0; it < 200; ++it) {
                long double mid = 0.5L * (lo + hi);
                if (orc_g(v, z, mid) >= thr) hi = mid; else lo = mid;
            }
            a = 0.5L * (lo + hi);
        }
        long double step = 1.0L;
        while (orc_g(v, z, tm + step) >= thr) step *= 2.0L;
        long double lo = tm + 0.5L * step, hi = tm + step;
        if (step == 1.0L) lo = tm;
        for (int it = 0; it < 200; ++it) {
            long double mid = 0.5L * (lo + hi);
            if (orc_g(v, z, mid) >= thr) lo = mid; else hi = mid;
        }
        tmax[i] = (double)tm;
        gmax[i] = (double)gm;
        t0[i] = (double)a;
        t1[i] = (double)(0.5L * (lo + hi));
    }
}

/* Exported: log of the truncated integral int_0^L exp(-x cosh t) cosh(nu t) dt,
 * the quantity RBK of the paper's empirical upper-bound finder (Alg. 1), by the
 * same adaptive rule as oracle_besselk. Returns the count of non-converged entries. */
int64_t oracle_log_truncated(const double* nu, const double* x, int64_t n, double L, double* out)
{
    int64_t bad = 0;
#pragma omp parallel reduction(+ : bad)
    {
        orc_seg* seg = (orc_seg*)malloc(sizeof(orc_seg) * ORC_MAXSUB);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            long double v = fabsl((long double)nu[i]), z = (long double)x[i], Lt = (long double)L;
            orc_integrand f;
            f.nu = v; f.x = z;
            f.kind = 0; f.lfref = 0.0L;
            long double th = orc_tmax(v, z);
            if (th > Lt) th = Lt;
            f.that = th;
            f.lcref = orc_logcosh(v * th);
            int ok = 1;
            long double I = 0.0L;
            if (th > 0.0L) I += orc_adapt(&f, 0.0L, th, 1e-17L, seg, &ok);
            if (Lt > th) I += orc_adapt(&f, th, Lt, 1e-17L, seg, &ok);
            if (!ok) ++bad;
            out[i] = (double)(orc_g(v, z, th) + logl(I));
        }
        free(seg);
    }
    return bad;
}

/* Exported: the fixed-window trapezoid sum of the paper's refined algorithm for
 * x >= 0.1 (Sec. IV-C, Alg. 2, integral branch; Eq. "refined" with the weights
 * c_m read as multiplicative trapezoid weights): with h = T / b and t_m = m h,
 *   S = sum_{m=0}^{b} h c_m exp(-x cosh t_m) cosh(nu t_m),  c_0 = c_b = 1/2, else 1.
 * The paper scales by the grid maximum before summing; that factor cancels, so
 * the oracle is the sum itself, in long double. Output: log S and S (double). */
void oracle_fixed_window(const double* nu, const double* x, int64_t n, int bins, double T,
                         double* logs, double* s)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const long double v = fabsl((long double)nu[i]), z = (long double)x[i];
        const long double h = (long double)T / (long double)bins;
        long double gmax = -1e4000L;
        for (int m = 0; m <= bins; ++m) {
            long double g = orc_g(v, z, (long double)m * h);
            if (g > gmax) gmax = g;
        }
        long double acc = 0.0L;
        for (int m = 0; m <= bins; ++m) {
            long double c = (m == 0 || m == bins) ? 0.5L : 1.0L;
            acc += c * expl(orc_g(v, z, (long double)m * h) - gmax);
        }
        long double ls = gmax + logl(h * acc);
        logs[i] = (double)ls;
        s[i] = (double)expl(ls);
    }
}

/* Exported: the log-integrand itself, for tests that pin the oracle's g. */
void oracle_logintegrand(const double* nu, const double* x, const double* t, double* out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = (double)orc_g(fabsl((long double)nu[i]), (long double)x[i], (long double)t[i]);
}

/* Maximiser over t >= 0 of the log of a derivative integrand (kinds 1 and 2),
 * g(t) + log F(t). Both are unimodal: for kind 1 the slope is
 * nu tanh(nu t) + tanh t - x sinh t, and (nu tanh(nu t) + tanh t) / sinh t
 * decreases; kind 2 is log-concave (log t, log sinh(nu t) and -x cosh t all
 * are). At the maximiser x sinh t equals nu tanh(nu t) + tanh t < nu + 1
 * (kind 1), or 1/t + nu coth(nu t) <= 2/t + nu (kind 2), so it lies below
 * asinh((nu + 2)/x) + 1; golden-section search on [0, that bound]. */
static long double orc_targmax(int kind, long double nu, long double x)
{
    const long double ginv = 0.618033988749894848204586834365638118L;
    long double a = 0.0L, b = asinhl((nu + 2.0L) / x) + 1.0L;
    long double c = b - ginv * (b - a), d = a + ginv * (b - a);
    long double gc = orc_g(nu, x, c) + orc_lfac(kind, nu, c);
    long double gd = orc_g(nu, x, d) + orc_lfac(kind, nu, d);
    for (int it = 0; it < 300 && (b - a) > 1e-16L * b; ++it) {
        if (gc > gd) { b = d; d = c; gd = gc; c = b - ginv * (b - a); gc = orc_g(nu, x, c) + orc_lfac(kind, nu, c); }
        else         { a = c; c = d; gc = gd; d = a + ginv * (b - a); gd = orc_g(nu, x, d) + orc_lfac(kind, nu, d); }
    }
    return 0.5L * (a + b);
}

/* log of int_0^inf exp(-x cosh t) cosh(nu t) F(t) dt for kind 1 or 2 (nu >= 0,
 * x > 0; kind 2 needs nu > 0), by the adaptive rule of orc_logk around the
 * integrand's own maximiser. */
static long double orc_logderiv(int kind, long double nu, long double x, orc_seg* seg, int* ok)
{
    orc_integrand f;
    f.nu = nu; f.x = x; f.kind = kind;
    const long double th = orc_targmax(kind, nu, x);
    f.that = th;
    f.lcref = orc_logcosh(nu * th);
    f.lfref = orc_lfac(kind, nu, th);
    const long double lref = orc_g(nu, x, th) + f.lfref;
    long double step = 1.0L, T = th + step;
    while (logl(orc_phi(&f, T)) > -64.0L && step < 1e4L) { step *= 2.0L; T = th + step; }
    const long double tol = 1e-17L;
    long double I = 0.0L;
    if (th > 0.0L) I += orc_adapt(&f, 0.0L, th, tol, seg, ok);
    I += orc_adapt(&f, th, T, tol, seg, ok);
    return lref + logl(I);
}

/* Exported: partial derivatives of K_nu(x) for n pairs (x > 0):
 *   lmdx[i] = log(-dK/dx),  ldnu[i] = log|dK/dnu|  (-inf at nu == 0)
 *   smdx[i] = -e^x dK/dx,   sdnu[i] = e^x |dK/dnu|  (formed in long double)
 * dK/dx < 0 always; dK/dnu has the sign of nu (K is even in nu). Entries with
 * x <= 0 or NaN inputs give NaN. Returns the count of non-converged entries. */
int64_t oracle_besselk_deriv(const double* nu, const double* x, int64_t n, double* lmdx, double* ldnu,
                             double* smdx, double* sdnu)
{
    int64_t bad = 0;
#pragma omp parallel reduction(+ : bad)
    {
        orc_seg* seg = (orc_seg*)malloc(sizeof(orc_seg) * ORC_MAXSUB);
#pragma omp for schedule(dynamic, 16)
        for (int64_t i = 0; i < n; ++i) {
            const long double v = fabsl((long double)nu[i]), z = (long double)x[i];
            if (isnan(nu[i]) || isnan(x[i]) || !(x[i] > 0.0)) {
                lmdx[i] = ldnu[i] = smdx[i] = sdnu[i] = NAN;
                continue;
            }
            int ok = 1;
            const long double a = orc_logderiv(1, v, z, seg, &ok);
            const long double b = v == 0.0L ? -INFINITY : orc_logderiv(2, v, z, seg, &ok);
            if (!ok) ++bad;
            lmdx[i] = (double)a;
            ldnu[i] = (double)b;
            smdx[i] = (double)expl(a + z);
            sdnu[i] = (double)expl(b + z);
        }
        free(seg);
    }
    return bad;
}

/* Digamma psi(v) for v > 0 in long double: psi(v) = psi(v + 1) - 1/v up to
 * v >= 20, then the asymptotic series
 *   psi(v) ~ ln v - 1/(2v) - sum_k B_2k / (2k v^2k)
 * through B_14 (Abramowitz & Stegun 6.3.18). */
static long double orc_digamma(long double v)
{
    long double acc = 0.0L;
    while (v < 20.0L) { acc -= 1.0L / v; v += 1.0L; }
    const long double r = 1.0L / (v * v);
    const long double ser =
        r * (1.0L / 12 - r * (1.0L / 120 - r * (1.0L / 252 - r * (1.0L / 240 - r * (1.0L / 132
        - r * (691.0L / 32760 - r * (1.0L / 12)))))));
    return acc + logl(v) - 0.5L / v - ser;
}

/* Exported: digamma for tests. */
void oracle_digamma(const double* v, double* out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) out[i] = (double)orc_digamma((long double)v[i]);
}

/* Exported: Matern covariance entries and their partial derivatives in beta and
 * nu (Sec. III-A formula, differentiated). With z = r / beta and
 * M = sigma2 2^(1-nu) / Gamma(nu) z^nu K_nu(z):
 *   dM/dbeta = (dM/dz)(-z / beta), and d/dz [z^nu K_nu(z)] = -z^nu K_{nu-1}(z)
 *              (DLMF 10.29.4), so dM/dbeta = sigma2 2^(1-nu)/Gamma(nu) z^(nu+1) K_{nu-1}(z) / beta;
 *   dM/dnu   = M (ln z - ln 2 - psi(nu)) + sigma2 2^(1-nu)/Gamma(nu) z^nu dK_nu/dnu(z).
 * K_{nu-1} = K_{|nu-1|} comes from the K integral, dK/dnu from the kind-2
 * integral. An exact zero distance gives M = sigma2 and zero derivatives.
 * Returns the count of non-converged quadratures. */
int64_t oracle_matern_grad(const double* rx, const double* ry, const double* cx, const double* cy,
                           const int64_t* ri, const int64_t* ci, int64_t n_entries,
                           double sigma2, double beta, double nu, double* m, double* dbeta, double* dnu)
{
    int64_t bad = 0;
    const long double lnu = (long double)nu, lb = (long double)beta, s2 = (long double)sigma2;
    const long double pre = (1.0L - lnu) * ORC_LN2 - lgammal(lnu);
    const long double psi = orc_digamma(lnu);
#pragma omp parallel reduction(+ : bad)
    {
        orc_seg* seg = (orc_seg*)malloc(sizeof(orc_seg) * ORC_MAXSUB);
#pragma omp for schedule(dynamic, 16)
        for (int64_t e = 0; e < n_entries; ++e) {
            long double dx = (long double)cx[ci[e]] - (long double)rx[ri[e]];
            long double dy = (long double)cy[ci[e]] - (long double)ry[ri[e]];
            long double r = sqrtl(dx * dx + dy * dy);
            if (r == 0.0L) { m[e] = sigma2; dbeta[e] = 0.0; dnu[e] = 0.0; continue; }
            const long double z = r / lb, lz = logl(z);
            int ok = 1;
            const long double lk = orc_logk(lnu, z, seg, &ok);
            const long double lk1 = orc_logk(fabsl(lnu - 1.0L), z, seg, &ok);
            const long double ld = orc_logderiv(2, lnu, z, seg, &ok);
            if (!ok) ++bad;
            const long double mv = s2 * expl(pre + lnu * lz + lk);
            m[e] = (double)mv;
            dbeta[e] = (double)(s2 / lb * expl(pre + (lnu + 1.0L) * lz + lk1));
            dnu[e] = (double)(mv * (lz - ORC_LN2 - psi) + s2 * expl(pre + lnu * lz + ld));
        }
        free(seg);
    }
    return bad;
}
