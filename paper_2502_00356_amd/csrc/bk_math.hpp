// bk_math.hpp - per-entry device routines for K_nu(x) by finite-window trapezoid
// quadrature of K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt (Sec. IV-B).
//
// Notation follows Sec. IV-B: g(t) = log cosh(nu t) - x cosh t is the
// log-integrand, t* its maximiser over t >= 0 ("t_max"), [t0, t1] the window on
// which g(t) >= g(t*) - L, and the trapezoid sum is taken relative to a reference
// point t_ref (Eq. "refined": log K = g(t_ref) + log sum h c_m exp(g(t_m) - g(t_ref))).
//
// The plain FP64 form builds its node terms without cancellation (below); the
// FP32-term forms form the exponent directly (WalkF, further down), which their
// precision allows. With u = t - t_ref, w = u/2:
//   g(t) - g(t_ref) = nu u + log(1+P(t)) - log(1+P(t_ref)) - xterm,
//   P(t) = exp(-2 nu t),   xterm = x (cosh t - cosh t_ref)
//                                = 2 sinh w (x cosh t_ref sinh w + x sinh t_ref cosh w),
// and along the node grid every exponential is an exact geometric progression,
// advanced by one multiply (or fused multiply-add) per node in FP64:
//   V = expm1(|w|), Bw = exp(w), Bb = exp(-w), P = exp(-2 nu t).
// t_ref is the node nearest t*, so w = 0 falls on a node. Left of it |w| shrinks
// and V follows V' = (V - qm1) / q; right of it |w| grows and V' = V q + qm1
// (q = e^(h/2), qm1 = expm1(h/2)). Both directions keep V's relative error at
// a few ulps; 2 sinh w = sign(w) V (1 + e^-|w|) then has no cancellation.
// The log(1+P(t_ref)) term cancels against the prefactor, so
//   K = exp(-x) exp(Delta) h sum_m c_m exp(nu u_m - xterm_m) (1 + P_m),
//   Delta = nu t_ref - ln 2 - 2 x sinh^2(t_ref / 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bk {

constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLog2e = 1.4426950408889634074;
constexpr int kNodeMin = 4;
constexpr int kNodeMax = 512;
constexpr int kRuleCand = 15;

// Tables of the table-driven exponential and log1p (kernels stage them in LDS):
// [0, 64): 2^(j/64); [64, 129): log(1 + j/64); [129, 194): 1 / (1 + j/64).
constexpr int kTabLog1p = 64, kTabInv1p = 129, kTabLen = 194;

// Node-count rule constants, filled on the host: for each strip half-width a_k,
// a_k, 1 - cos a_k and log sec a_k (see node_step); and the tables above.
struct RuleTable {
    double a[kRuleCand];
    double omc[kRuleCand];
    double lsec[kRuleCand];
    double tab[kTabLen];
};

// Chebyshev coefficients of Temme's Gamma1 and Gamma2 (see temme_k below).
constexpr int kTemmeCheb = 14;

struct TemmeCoef {
    double g1[kTemmeCheb];
    double g2[kTemmeCheb];
};

// kRuleTab and kTemmeTab: the two tables above as device constants (values made
// by gen_tables.py at 40 digits and rounded to double), so no call sets anything
// up on the GPU.
#include "bk_tables.inc"

// The tables as the kernels read them: through a pointer the optimiser cannot see
// through (an empty asm statement), so that their values are fetched by scalar
// loads from the constant segment instead of being folded into the code as
// 64-bit literals, which costs registers (measured: spills in the Matern kernels).
typedef __attribute__((address_space(4))) const RuleTable ConstSegRuleTable;
typedef __attribute__((address_space(4))) const TemmeCoef ConstSegTemmeCoef;

__device__ __forceinline__ const RuleTable& rule_tab()
{
    ConstSegRuleTable* p = (ConstSegRuleTable*)&kRuleTab;
    __asm__ volatile("" : "+s"(p));
    return *(const RuleTable*)p;
}

__device__ __forceinline__ const TemmeCoef& temme_tab()
{
    ConstSegTemmeCoef* p = (ConstSegTemmeCoef*)&kTemmeTab;
    __asm__ volatile("" : "+s"(p));
    return *(const TemmeCoef*)p;
}

// Per-entry quadrature plan.
struct Plan {
    double tref;   // reference point: node mc, the node nearest the peak
    double t0;     // first node
    double h;      // step
    int N;         // intervals; nodes m = 0..N
    int mc;        // index of the reference node (0 <= mc <= N)
};

// Inclusive prefix sum over the 64 lanes of a wave (all active) with DPP lane
// moves instead of LDS: a scan within each 16-lane row by shifts of 1, 2, 4 and 8
// (lanes shifted in from outside the row add 0), then the last lane of row 0 is
// added to row 1 and of row 2 to row 3 (row_bcast:15), and the last lane of row 1
// to rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ unsigned int wave_incl_scan(unsigned int v)
{
    v += __builtin_amdgcn_update_dpp(0u, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0u, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0u, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0u, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
    return v;
}

// 1/a for a normal nonzero double: hardware reciprocal refined by two Newton
// steps (within about an ulp; no IEEE division sequence).
__device__ __forceinline__ double recip(double a)
{
    double r = __builtin_amdgcn_rcp(a);
    r = fma(r, fma(-a, r, 1.0), r);
    return fma(r, fma(-a, r, 1.0), r);
}

// e^x from T[j] = 2^(j/64), j = 0..63 (Tang's table-driven method): with
// k = floor(64 x log2 e) and f = x - k ln2/64, in [0, ln2/64) up to rounding,
// e^x = 2^(k div 64) T[k mod 64] e^f, and e^f is its Taylor polynomial through f^6
// (truncation below 2e-18). ln2/64 rounded to FP64 is 3.6e-19 short, so the
// reduction adds |k| 3.6e-19 relative: below 1.5e-15 for |x| <= 40, which covers
// every use whose result matters (the walks' node exponents reach below -40 only
// for terms under e^-40 of their sum; the set-up arguments are smaller). Within a
// few ulps overall there. x is clamped at -746, where e^x is already below half the
// smallest subnormal and the final ldexp gives 0 (also for x = -inf); ldexp takes
// large x to infinity. The kernels stage T in LDS.
__device__ __forceinline__ double exp_tab(double x, const double* T)
{
    x = fmax(x, -746.0);
    const double k = floor(x * 92.332482616893656);          // 64 log2 e
    const double f = fma(-k, 0.010830424696249145, x);        // ln2 / 64
    double p = 1.0 / 720.0;
    p = fma(p, f, 1.0 / 120.0);
    p = fma(p, f, 1.0 / 24.0);
    p = fma(p, f, 1.0 / 6.0);
    p = fma(p, f, 0.5);
    p = fma(p, f, 1.0);
    p = fma(p, f, 1.0);
    const int ki = (int)k;
    return ldexp(T[ki & 63] * p, ki >> 6);
}

// log(1 + p) for 0 <= p <= 1 from the same tables: with j = floor(64 p) and
// c = 1 + j/64, log(1 + p) = log c + log(1 + r), r = (p - j/64) / c in [0, 1/64)
// (p - j/64 is exact), the second by its Taylor series through r^9 (truncation
// below 1e-18); a few ulps.
__device__ __forceinline__ double log1p_tab(double p, const double* T)
{
    const int j = min(max((int)(p * 64.0), 0), 64);
    const double r = (p - (double)j * 0.015625) * T[kTabInv1p + j];
    double q = 1.0 / 9.0;
    q = fma(q, -r, 1.0 / 8.0);
    q = fma(q, -r, 1.0 / 7.0);
    q = fma(q, -r, 1.0 / 6.0);
    q = fma(q, -r, 1.0 / 5.0);
    q = fma(q, -r, 1.0 / 4.0);
    q = fma(q, -r, 1.0 / 3.0);
    q = fma(q, -r, 0.5);
    q = fma(q, -r, 1.0);
    return fma(q, r, T[kTabLog1p + j]);
}

// The tables into LDS; every thread of the block must call it (it ends with a
// barrier).
__device__ __forceinline__ void stage_tab(double* s)
{
    for (int j = threadIdx.x; j < kTabLen; j += blockDim.x) s[j] = rule_tab().tab[j];
    __syncthreads();
}

// log y for a positive normal y: y = 2^e m with m in [1/2, 1), log y = (e - 1) ln 2
// + log1p(2m - 1), the second from the tables (a few ulps).
__device__ __forceinline__ double log_tab(double y, const double* T)
{
    int e;
    const double m = frexp(y, &e);
    return fma((double)(e - 1), kLn2, log1p_tab(2.0 * m - 1.0, T));
}

__device__ __forceinline__ void cosh_sinh_tab(double t, double& ch, double& sh, const double* T)
{
    const double e = exp_tab(t, T);
    const double ei = recip(e);
    ch = 0.5 * (e + ei);
    sh = 0.5 * (e - ei);
}

__device__ __forceinline__ void cosh_sinh(double t, double& ch, double& sh)
{
    double e = exp(t);
    double ei = recip(e);
    ch = 0.5 * (e + ei);
    sh = 0.5 * (e - ei);
}

// log cosh(y) for y >= 0 without overflow: y + log1p(exp(-2y)) - ln 2.
__device__ __forceinline__ double logcosh_pos(double y, const double* T)
{
    return y + log1p_tab(exp_tab(-2.0 * y, T), T) - kLn2;
}

// g and its first three derivatives at t >= 0 (g''' for Halley's method on g').
struct GDer {
    double g, g1, g2, g3;
};

__device__ __forceinline__ GDer g_derivs(double nu, double x, double t, const double* T)
{
    GDer d;
    const double p = exp_tab(-2.0 * nu * t, T);
    const double ip = recip(1.0 + p);
    const double th = (1.0 - p) * ip;                 // tanh(nu t)
    const double s2 = 4.0 * p * ip * ip;              // sech^2(nu t)
    double ch, sh;
    cosh_sinh_tab(t, ch, sh, T);
    d.g = nu * t + log1p_tab(p, T) - kLn2 - x * ch;
    d.g1 = nu * th - x * sh;
    d.g2 = nu * nu * s2 - x * ch;
    d.g3 = -2.0 * nu * nu * nu * th * s2 - x * sh;
    return d;
}

// Halley step for a root of f with derivatives f1, f2: 2 f f1 / (2 f1^2 - f f2),
// or the Newton step f / f1 where the Halley denominator is not a positive normal
// number.
__device__ __forceinline__ double halley_step(double f, double f1, double f2)
{
    const double den = 2.0 * f1 * f1 - f * f2;
    return den > 1e-300 ? 2.0 * f * f1 * recip(den) : f / f1;
}

// The three roots below are found by Halley's method (cubic convergence) and
// stop once a step is below 1e-7 (peak) or 1e-5 (window ends) of t: the error
// left after such a step is of order its cube, below 1e-15 relative.

// Starting points of the root searches below. They only seed Halley's method, so
// they come from FP32 hardware operations (a few instructions against the library
// asinh / acosh in FP64), moved outward by 1e-4 relative so that they keep the side
// of the root the searches start from; beyond the FP32 range, log(2y) by the
// table logarithm.
// Upper bound of asinh(y), y > 0.
__device__ __forceinline__ double asinh_start(double y, const double* T)
{
    if (y < 1e18) {
        const float yf = (float)y;
        return (double)(__logf(yf + __fsqrt_rn(fmaf(yf, yf, 1.0f))) * 1.0001f);
    }
    return log_tab(2.0 * y, T) * 1.0001;
}
// Lower bound of acosh(1 + eps), eps > 0: log1p(eps + sqrt(eps (2 + eps))).
__device__ __forceinline__ double acosh1p_start(double eps, const double* T)
{
    if (eps < 1e18) {
        const float e = (float)eps;
        return (double)(log1pf(e + __fsqrt_rn(e * (2.0f + e))) * 0.9999f);
    }
    return log_tab(2.0 * eps, T) * 0.9999;
}

// Maximiser t* of g over t >= 0 when nu^2 > x (Sec. IV-B: otherwise t* = 0), the
// zero of g' = nu tanh(nu t) - x sinh t. Since nu tanh < nu, it lies left of
// asinh(nu/x), where the iteration starts (the bracket search of FINDRANGE is
// replaced by this analytic upper bound); g' is decreasing right of t* and steps
// that would leave t > 0 are halved.
__device__ inline double peak_solve(double nu, double x, const double* T)
{
    double t = asinh_start(fmin(nu / x, 1e300), T);
    for (int it = 0; it < 64; ++it) {
        const GDer d = g_derivs(nu, x, t, T);
        const double dt = halley_step(d.g1, d.g2, d.g3);
        double tn = t - dt;
        if (!(tn > 0.0)) tn = 0.5 * t;
        t = tn;
        if (!(fabs(dt) > 1e-7 * t) || t < 1e-150) break;
    }
    return t;
}

// Root t1 > t* of G(t) = g(t) - gstar + L (g concave and decreasing beyond t*).
// Start at acosh(cosh t* + L/x): there the x-term alone has dropped by L and the
// log cosh term has grown, so G >= 0 (FINDRANGE's lower end). Iterates are kept
// in (t*, t* + 4 (start - t*) + 1].
__device__ inline double window_right(double nu, double x, double tstar, double chstar,
                                      double gstar, double L, const double* T)
{
    double t = acosh1p_start((chstar - 1.0) + L / x, T);
    const double tcap = tstar + 4.0 * (t - tstar) + 1.0;
    for (int it = 0; it < 64; ++it) {
        const GDer d = g_derivs(nu, x, t, T);
        const double dt = halley_step(d.g - gstar + L, d.g1, d.g2);
        double tn = fmin(t - dt, tcap);
        if (!(tn > tstar)) tn = 0.5 * (t + tstar);
        const bool done = !(fabs(tn - t) > 1e-5 * t);
        t = tn;
        if (done) break;
    }
    return t;
}

// Root t0 in (0, t*) of G when G(0) < 0 (only possible if nu t* > L, since g' <= nu).
// Bracket: G(0) < 0 and G(t* - L/nu) >= 0, shrunk at every iterate; a step that
// would leave it is replaced by bisection.
__device__ inline double window_left(double nu, double x, double tstar, double gstar, double L, const double* T)
{
    double lo = 0.0, hi = fmax(tstar - L / nu, 0.0);
    double t = hi;
    for (int it = 0; it < 100; ++it) {
        const GDer d = g_derivs(nu, x, t, T);
        const double G = d.g - gstar + L;
        if (G >= 0.0) hi = t; else lo = t;
        const double dt = halley_step(G, d.g1, d.g2);
        double tn = t - dt;
        if (!(fabs(dt) > 1e-5 * t)) { t = fmin(fmax(tn, lo), hi); break; }
        if (!(tn >= lo && tn <= hi)) tn = 0.5 * (lo + hi);
        t = tn;
        if (hi - lo <= 1e-15 * hi) break;
    }
    return t;
}

// Trapezoid step from the strip bound: the best over the candidate half-widths a
// of 2 pi a / (Lq + ln 2 + x (1 - cos a) + (nu + 1) log sec a).
__device__ inline double node_step(double nu, double x, double Lq, const RuleTable& R)
{
    double base = Lq + kLn2;
    double nu1 = nu + 1.0;
    double bn = R.a[0], bd = base + x * R.omc[0] + nu1 * R.lsec[0];
#pragma unroll
    for (int k = 1; k < kRuleCand; ++k) {
        double den = base + x * R.omc[k] + nu1 * R.lsec[k];
        bool better = R.a[k] * bd > bn * den;
        bn = better ? R.a[k] : bn;
        bd = better ? den : bd;
    }
    return 6.283185307179586477 * bn / bd;
}

__device__ __forceinline__ int node_count(double width, double h)
{
    double r = ceil(width / h);
    if (!(r >= (double)kNodeMin)) r = (double)kNodeMin;   // also maps NaN to the minimum
    if (r > (double)kNodeMax) r = (double)kNodeMax;
    return (int)r;
}

// Plain bracket solver (FP64): peak, window at threshold L, node count for Lq,
// reference node. Also returns, for the prefactor,
// Delta = nu t_ref - ln 2 - 2 x sinh^2(t_ref/2), and the constants
// A = x cosh(t_ref)/2, B = x sinh(t_ref)/2 of the cancellation-free xterm.
struct Solved {
    Plan p;
    double delta, dlo;   // Delta as an unevaluated sum delta + dlo (|dlo| below an ulp of delta)
    double A, B;         // x cosh(t_ref) / 2, x sinh(t_ref) / 2 (single walk, FP32-term walk)
    double E, Ei, Sr;    // e^t_ref, e^-t_ref, expm1(t_ref) (paired walk of the plain sum)
    double gstar;   // g(t*) (used by the window export)
    double t1;
};

// Rounding error of s = a + b (Knuth's two-sum): a + b = s + two_sum_err(a, b, s) exactly.
__device__ __forceinline__ double two_sum_err(double a, double b, double s)
{
    const double bb = s - a;
    return (a - (s - bb)) + (b - bb);
}

// ln 2 - kLn2 (the part of ln 2 below the double kLn2).
constexpr double kLn2Lo = 2.319046813846299558e-17;

// Delta = nu t_ref - ln 2 - q as hi + lo: the product split exactly by a fused
// multiply-add, the two sums' rounding errors carried by two_sum_err. Contraction
// is off here: fusing nu t_ref into the first sum (or q's product into it) would
// round something other than what the error terms describe.
__device__ __forceinline__ void delta_dd(double nu, double tref, double q, double& hi, double& lo)
{
#pragma clang fp contract(off)
    const double pr = nu * tref, pe = fma(nu, tref, -pr);
    const double s1 = pr - q, e1 = two_sum_err(pr, -q, s1);
    const double s2 = s1 - kLn2, e2 = two_sum_err(s1, -kLn2, s2);
    hi = s2;
    lo = ((pe + e1) + e2) - kLn2Lo;
}

// Node grid on [t0, t1] with step at most h0, reference node nearest tpk, and
// the prefactor constants for the node walk. Delta = nu t_ref - ln 2 -
// 2 x sinh^2(t_ref/2) reaches ~120 for large orders at small x, where rounding it
// to one double would cost ~1e-14 of K; it is kept as delta + dlo, with nu t_ref
// split exactly (fused multiply-add) and the sums' rounding errors carried, so
// that what is left is the ~3 ulps of the sinh^2 term.
__device__ inline Solved plan_window(double nu, double x, double t0, double t1, double tpk, double h0)
{
    Solved s;
    int N = node_count(t1 - t0, h0);
    double h = (t1 - t0) / (double)N;
    int mc = 0;
    if (tpk > t0) {
        double r = rint((tpk - t0) / h);
        mc = (int)fmin(fmax(r, 0.0), (double)N);
    }
    double tref = t0 + (double)mc * h;
    double ch, sh;
    cosh_sinh(tref, ch, sh);
    double em = expm1(0.5 * tref);                     // sinh(t/2) = em (em + 2) / (2 (em + 1))
    double sh2 = em * (em + 2.0) / (2.0 * (em + 1.0));
    s.p.tref = tref;
    s.p.t0 = t0;
    s.p.N = N;
    s.p.mc = mc;
    s.p.h = h;
    delta_dd(nu, tref, 2.0 * x * sh2 * sh2, s.delta, s.dlo);
    s.A = 0.5 * x * ch;
    s.B = 0.5 * x * sh;
    s.Sr = em * (em + 2.0);                            // expm1(t_ref), no cancellation
    s.E = s.Sr + 1.0;
    s.Ei = recip(s.E);
    s.gstar = 0.0;
    s.t1 = t1;
    return s;
}

__device__ inline Solved plain_solve(double nu, double x, double L, double Lq, const RuleTable& R,
                                     const double* T)
{
    double tstar = 0.0;
    if (nu * nu > x) tstar = peak_solve(nu, x, T);
    double chs, shs;
    cosh_sinh_tab(tstar, chs, shs, T);
    double gstar = logcosh_pos(nu * tstar, T) - x * chs;
    double t1 = window_right(nu, x, tstar, chs, gstar, L, T);
    double t0 = 0.0;
    if (-x < gstar - L) t0 = window_left(nu, x, tstar, gstar, L, T);
    Solved s = plan_window(nu, x, t0, t1, tstar, node_step(nu, x, Lq, R));
    s.gstar = gstar;
    return s;
}

// Geometric-progression state of one entry's node walk.
struct Walk {
    double k, V, Bw, Bb, P;        // at the current node; k = m - mc (exact), u = k h
    double h, q, qm1, qi, rho;     // per-step factors
    int mc;
};

__device__ __forceinline__ Walk walk_begin(double nu, const Plan& p)
{
    Walk w;
    w.mc = p.mc;
    w.k = -(double)p.mc;
    w.V = expm1(0.5 * (double)p.mc * p.h);        // expm1(|w_0|), w_0 = -mc h / 2
    w.Bb = w.V + 1.0;
    w.Bw = recip(w.Bb);
    w.P = exp(-2.0 * nu * p.t0);
    w.h = p.h;
    w.qm1 = expm1(0.5 * p.h);
    w.q = w.qm1 + 1.0;
    w.qi = recip(w.q);
    w.rho = exp(-2.0 * nu * p.h);
    return w;
}

// Exponent nu u - xterm at node m (FP64, cancellation-free).
__device__ __forceinline__ double walk_exponent(const Walk& w, int m, double nu, double A, double B)
{
    double sv = (m < w.mc) ? -w.V : w.V;
    double sg = sv * (1.0 + fmin(w.Bw, w.Bb));   // 2 sinh(u/2)
    double c2 = w.Bw + w.Bb;                      // 2 cosh(u/2)
    double xterm = sg * (A * sg + B * c2);        // x (cosh t - cosh t_ref)
    return nu * (w.k * w.h) - xterm;
}

// Advance from node m to node m + 1.
__device__ __forceinline__ void walk_step(Walk& w, int m)
{
    w.k += 1.0;                                   // u = k h is formed per node: no drift
    w.Bw *= w.q;
    w.Bb *= w.qi;
    w.P *= w.rho;
    double vin = fmax((w.V - w.qm1) * w.qi, 0.0);
    double vout = fma(w.V, w.q, w.qm1);
    w.V = (m + 1 <= w.mc) ? vin : vout;
}

// FP64 trapezoid sum of the plain form, S = sum_m c_m exp(d_m) (1 + P_m),
// c_0 = c_N = 1/2, as a paired walk outward from the reference node: iteration j
// takes node mc + j (right, j <= N - mc) and node mc - j (left, 1 <= j <= mc),
// both at |w| = j h / 2. With x (cosh t - cosh t_ref) = 2 x sinh(w) sinh(s),
// s = (t + t_ref) / 2 >= |w| (product-to-sum, no cancellation):
//   right: d = nu j h - (x/2) 2 sinh|w| 2 sinh(t_ref + |w|),
//   left:  d = -nu j h + (x/2) 2 sinh|w| 2 sinh(t_ref - |w|).
// 2 sinh|w| = V (1 + e^-|w|) with V = expm1(|w|) from V' = V q + expm1(h/2),
// which only ever runs outward from V = 0 (its relative error grows by about an
// ulp per step; an inward run loses relative accuracy as V shrinks, and that loss
// reached ~5e-14 of K left of interior peaks); 2 sinh(t_ref + |w|) the same way
// from expm1(t_ref); 2 sinh(t_ref - |w|) = e^t_ref e^-|w| - e^-t_ref e^|w|, whose
// terms differ by a factor e^(2 (t_ref - |w|)) >= e^t_ref. The two sides share V,
// e^-|w| and nu j h; a side no lane of the wave needs is skipped. T is exp_tab's
// table; E, Ei, Sr = e^t_ref, e^-t_ref, expm1(t_ref) from the solve.
__device__ inline double sum_f64(double nu, double x, const Plan& p, double E, double Ei, double Sr, const double* T)
{
    const int nr = p.N - p.mc, nl = p.mc, jmax = nr > nl ? nr : nl;
    const double h = p.h, xh = 0.5 * x;
    const double qm1 = expm1(0.5 * h), q = qm1 + 1.0, qi = recip(q);
    const double rho = exp_tab(-2.0 * nu * h, T), rhoi = recip(rho);
    double V = 0.0, Bq = 1.0;                 // expm1(|w|), e^-|w|
    double SR = Sr, ER = Ei;                  // expm1(t_ref + |w|), e^-(t_ref + |w|)
    double PR = exp_tab(-2.0 * nu * p.tref, T), PL = PR;   // e^(-2 nu t) at nodes mc + j, mc - j
    double S = 0.0, jd = 0.0;
    for (int j = 0; j <= jmax; ++j) {
        const double nuu = nu * (jd * h);     // j h formed per node: no drift
        const double xs = xh * fma(V, Bq, V);
        if (j <= nr) {
            const double ss = fma(SR, ER, SR);
            const double t = exp_tab(fma(-xs, ss, nuu), T) * (1.0 + PR);
            S = fma((j == nr || (j == 0 && nl == 0)) ? 0.5 : 1.0, t, S);   // ends: node N; node 0 if mc = 0
        }
        if (j >= 1 && j <= nl) {
            const double ss = fma(E, Bq, -Ei * (V + 1.0));
            const double t = exp_tab(fma(xs, ss, -nuu), T) * (1.0 + PL);
            S = fma(j == nl ? 0.5 : 1.0, t, S);                          // node 0
        }
        V = fma(V, q, qm1);
        Bq *= qi;
        SR = fma(SR, q, qm1);
        ER *= qi;
        PR *= rho;
        PL *= rhoi;
        jd += 1.0;
    }
    return S;
}

// Node walk of the FP32-term forms (mixed and learned). Their terms need the
// exponent only to ~1e-9 absolute, so it is formed directly in FP64, in base 2,
//   d_m = log2(e) (nu (t_m - t_ref) - x (cosh t_m - cosh t_ref)),
// with cosh t_m from the three-term recurrence c_{m+1} = 2 cosh(h) c_m - c_{m-1}
// run forward from t_0 (the growing solution: its relative error stays within a
// few m^2 ulps), so the absolute error of d_m is about x cosh(t_m) m^2 2^-53,
// below 1e-10 on the whole (nu, x) range. The factor Q = 1 + e^(-2 nu t) follows
// Q' = rho Q + (1 - rho), rho = e^(-2 nu h) (contracting, so no error growth).
struct WalkF {
    double c, cn, kappa;      // cosh t_m, cosh t_{m+1}, 2 cosh h
    double a2, e, b2;         // d_m = a2 c_m + e_m; e_m = x cosh(t_ref) log2 e + (m - m_ref) b2, advanced by b2
    double Q, rho, omr;       // Q = 1 + e^(-2 nu t_m)
};
// e_m accumulates one rounding per node: m ulps of |e| <= x cosh t_ref + 30, below
// 1e-11 absolute in d_m for the windows here (the FP32 terms need ~1e-8).

// Walk state from the exponentials e = e^{t_0}, ei = e^{-t_0}, q2 = e^h,
// qi2 = e^{-h}, rho = e^{-2 nu h} (given by the caller).
__device__ __forceinline__ WalkF walkf_begin_exp(double nu, double x, double t0, double h, int mref, double xch_ref,
                                                 double e, double ei, double q2, double qi2, double rho)
{
    WalkF w;
    w.kappa = q2 + qi2;
    w.c = 0.5 * (e + ei);
    w.cn = 0.5 * (e * q2 + ei * qi2);
    w.a2 = -x * kLog2e;
    w.b2 = nu * h * kLog2e;
    w.e = fma(-(double)mref, w.b2, xch_ref * kLog2e);
    w.rho = rho;
    w.omr = 1.0 - rho;                // absolute error 2^-53: Q's error stays ~m 2^-53
    // Q only needs FP32 accuracy: e^(-2 nu t_0) in FP32 moves Q by < 6e-8 relative
    w.Q = 1.0 + (double)__expf((float)(-2.0 * nu * t0));
    return w;
}

__device__ __forceinline__ double walkf_exponent2(const WalkF& w) { return fma(w.a2, w.c, w.e); }

// The same step without the FP64 factor Q (kept elsewhere).
__device__ __forceinline__ void walkf_step_noq(WalkF& w)
{
    const double c2n = fma(w.kappa, w.cn, -w.c);
    w.c = w.cn;
    w.cn = c2n;
    w.e += w.b2;
}

__device__ __forceinline__ void walkf_step(WalkF& w)
{
    const double c2n = fma(w.kappa, w.cn, -w.c);
    w.c = w.cn;
    w.cn = c2n;
    w.e += w.b2;
    w.Q = fma(w.Q, w.rho, w.omr);
}

// Mixed form: the walk above with the reference at the node nearest the peak
// (exponents <= about 0), exponential in FP32, Kahan-compensated FP32 sum.
// A = x cosh(t_ref) / 2 from the solve; T is exp_tab's table. Returns
// sum_m c_m e^{d_m} (1 + P_m).
__device__ inline double sum_mixed(double nu, double x, const Plan& p, double A, const double* T)
{
    const double e = exp_tab(p.t0, T), ei = recip(e);
    const double q2 = exp_tab(p.h, T), qi2 = recip(q2);
    WalkF w = walkf_begin_exp(nu, x, p.t0, p.h, p.mc, 2.0 * A, e, ei, q2, qi2, exp_tab(-2.0 * nu * p.h, T));
    float s = 0.0f, c = 0.0f, ends = 0.0f;
#pragma unroll 2
    for (int m = 0; m <= p.N; ++m) {
        const float term = __builtin_amdgcn_exp2f((float)walkf_exponent2(w)) * (float)w.Q;
        const float y = term - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
        ends += (m == 0 || m == p.N) ? term : 0.0f;
        walkf_step(w);
    }
    return (double)s - (double)c - 0.5 * (double)ends;
}

// ---------------------------------------------------------------------------
// Derivatives of K_nu(x), FP64 (the paper names them as future work, Sec. VI).
// Differentiating the integral of Sec. IV-B under the integral sign:
//   dK/dx  = -int_0^inf cosh t cosh(nu t) e^(-x cosh t) dt,
//   dK/dnu =  int_0^inf t sinh(nu t) e^(-x cosh t) dt =: D.
// Since cosh t cosh(nu t) = (cosh((nu+1)t) + cosh((nu-1)t)) / 2, the first is
// -(K_{nu+1} + K_{nu-1}) / 2 = -(K_{nu-1} + (nu/x) K_nu) (three-term recurrence);
// a sum of two positive integrals of the K kind, so it costs one more K solve at
// order |nu - 1| and no cancellation.
// D has its own window. Its log-integrand
//   d(t) = log t + log sinh(nu t) - x cosh t
// is strictly concave on t > 0 (each term is), tends to -inf at 0 and has one
// maximiser t_d, the zero of d'(t) = 1/t + nu coth(nu t) - x sinh t. At t_d,
// x sinh t_d = 1/t_d + nu coth(nu t_d), which lies in [max(nu, 2/t_d), 2/t_d + nu]
// (coth y >= 1/y, coth y <= 1 + 1/y), so with sinh t <= 1.1752 t on [0, 1]:
//   t_d >= lo = max(asinh(nu/x), min(1, sqrt(1.70/x))),  t_d <= asinh((2/lo + nu)/x).
// Its window is [t0, t1]: t0 is the left end of K's window (left of it the factor
// t tanh(nu t) is below its value at K's peak, so D's integrand is below e^-L of
// its maximum there; when K's window starts at 0 so does D's, and D's integrand
// is even in t, so the trapezoid keeps its accuracy from t = 0), and t1 > t_d the
// root of d(t) = d(t_d) - L. Node terms reuse the K walk: with P = e^(-2 nu t),
//   t sinh(nu t) e^(-x cosh t) = e^(-x) e^Delta e^(nu u - xterm) t (1 - P),
// and Q = 1 - P follows Q' = Q rho + (1 - rho) (rho = e^(-2 nu h)), a recurrence
// that never amplifies Q's relative error.
// ---------------------------------------------------------------------------
// d and its first three derivatives at t > 0:
//   d'   = 1/t + nu coth(nu t) - x sinh t
//   d''  = -1/t^2 - nu^2 csch^2(nu t) - x cosh t
//   d''' = 2/t^3 + 2 nu^3 coth(nu t) csch^2(nu t) - x sinh t
struct DDer {
    double d, d1, d2, d3;
};

__device__ __forceinline__ DDer dnu_derivs(double nu, double x, double t, const double* T)
{
    DDer r;
    const double omp = -expm1(-2.0 * nu * t);        // 1 - e^(-2 nu t)
    const double p = 1.0 - omp;
    const double it = recip(t), io = recip(omp);
    const double cth = (2.0 - omp) * io;               // coth(nu t)
    const double cs2 = 4.0 * p * io * io;              // csch^2(nu t)
    double ch, sh;
    cosh_sinh_tab(t, ch, sh, T);
    r.d = log_tab(t, T) + nu * t + log_tab(omp, T) - kLn2 - x * ch;
    r.d1 = it + nu * cth - x * sh;
    r.d2 = -it * it - nu * nu * cs2 - x * ch;
    r.d3 = 2.0 * it * it * it + 2.0 * nu * nu * nu * cth * cs2 - x * sh;
    return r;
}

// Maximiser t_d of d: Halley on d' inside the bracket above (bisection when a step
// leaves it), stopped once a step is below 1e-7 of t.
__device__ inline double dnu_peak(double nu, double x, const double* T)
{
    double lo = fmax(asinh(nu / x), fmin(1.0, sqrt(1.70 / x)));
    double hi = asinh((2.0 / lo + nu) / x);
    double t = 0.5 * (lo + hi);
    for (int it = 0; it < 100; ++it) {
        const DDer r = dnu_derivs(nu, x, t, T);
        if (r.d1 > 0.0) lo = t; else hi = t;
        const double dt = halley_step(r.d1, r.d2, r.d3);
        double tn = t - dt;
        if (!(fabs(dt) > 1e-7 * t)) { t = fmin(fmax(tn, lo), hi); break; }
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        t = tn;
        if (hi - lo <= 1e-15 * hi) break;
    }
    return t;
}

// Root t1 > t_d of d(t) = dstar - L by Halley, from acosh(cosh t_d + L/x): there
// the x term alone has dropped by L while log t + log sinh(nu t) grew, so the start
// is left of the root. Iterates are kept in (t_d, t_d + 4 (start - t_d) + 1].
__device__ inline double dnu_window_right(double nu, double x, double td, double chd, double dstar, double L,
                                          const double* T)
{
    double t = acosh(chd + L / x);
    const double tcap = td + 4.0 * (t - td) + 1.0;
    for (int it = 0; it < 64; ++it) {
        const DDer r = dnu_derivs(nu, x, t, T);
        const double dt = halley_step(r.d - dstar + L, r.d1, r.d2);
        double tn = fmin(t - dt, tcap);
        if (!(tn > td)) tn = 0.5 * (t + td);
        const bool done = !(fabs(tn - t) > 1e-5 * t);
        t = tn;
        if (done) break;
    }
    return t;
}

// Plan for D given K's window start t0 (nu > 0, 0 < x < inf). The node step uses
// the strip bound of K with the extra factor of D's integrand on the strip,
// |t + i a| |sinh(nu (t + i a))| / (t sinh(nu t)) <= (1 + a/t) coth(nu t),
// taken at the maximiser with a = pi/2.
__device__ inline Solved dnu_solve(double nu, double x, double t0, double L, double Lq, const RuleTable& R,
                                   const double* T)
{
    const double td = dnu_peak(nu, x, T);
    const DDer r = dnu_derivs(nu, x, td, T);
    double chd, shd;
    cosh_sinh(td, chd, shd);
    const double t1 = dnu_window_right(nu, x, td, chd, r.d, L, T);
    const double extra = log1p(1.5707963267948966 / td) - log(tanh(nu * td));
    return plan_window(nu, x, t0, t1, td, node_step(nu, x, Lq + extra, R));
}

// FP64 trapezoid sum of D's node terms e^(nu u - xterm) t (1 - P).
__device__ inline double sum_dnu_f64(double nu, const Plan& p, double A, double B, const double* T)
{
    Walk w = walk_begin(nu, p);
    double Q = -expm1(-2.0 * nu * p.t0);
    const double omr = -expm1(-2.0 * nu * p.h);
    double S = 0.0, ends = 0.0;
    for (int m = 0; m <= p.N; ++m) {
        const double t = fma((double)m, p.h, p.t0);
        const double term = exp_tab(walk_exponent(w, m, nu, A, B), T) * t * Q;
        S += term;
        if (m == 0 || m == p.N) ends += term;
        walk_step(w, m);
        Q = fma(Q, w.rho, omr);
    }
    return S - 0.5 * ends;
}

// ---------------------------------------------------------------------------
// The paper's refined algorithm, integral branch (Sec. IV-C, Alg. 2): fixed
// window [0, T], b bins, nodes t_m = m h (h = T / b), weights 1/2 at both ends,
// scaled by the largest node value. g is unimodal on t >= 0, so the sum is taken
// relative to the node nearest t* (within one node of the largest) with the
// cancellation-free walk of the plain form: one FP64 exponential and a few
// multiplies per node instead of evaluating g at every node. b may run to the
// thousands, so the walk's multiplicative state is re-seeded from closed forms
// every kReseed nodes (its rounding drift grows with the steps taken) and long
// sums are compensated. The scale factors out of the sum: K = exp(lscale) hs.
// ---------------------------------------------------------------------------
struct FixedOut {
    double lscale;   // log of the factor taken out of the sum
    double hs;       // h * sum_m c_m exp(nu u_m - xterm_m) (1 + P_m), the walk's terms
};

constexpr int kReseed = 32;

// Walk state at node m from closed forms (u = (m - mc) h, V = expm1(|u| / 2)).
__device__ inline void walk_reseed(Walk& w, const Plan& p, double nu, int m)
{
    const int k = m - p.mc;
    w.k = (double)k;
    w.V = expm1(0.5 * p.h * (double)(k < 0 ? -k : k));
    const double big = w.V + 1.0, small = recip(big);
    w.Bw = (k <= 0) ? small : big;                // e^(u/2)
    w.Bb = (k <= 0) ? big : small;                // e^(-u/2)
    w.P = exp(-2.0 * nu * (p.t0 + (double)m * p.h));
}

// Trapezoid sum of the fixed window on the re-seeded walk; Kahan-compensated when
// Comp (b beyond kFixedPlainMax nodes, where plain FP64 accumulation error grows
// past the walk's own).
constexpr int kFixedPlainMax = 256;

template <bool Comp>
__device__ inline double fixed_sum(double nu, const Plan& p, double A, double B, const double* T)
{
    Walk w = walk_begin(nu, p);
    double S = 0.0, c = 0.0, ends = 0.0;
    for (int m = 0; m <= p.N; ++m) {
        if (m > 0 && m % kReseed == 0) walk_reseed(w, p, nu, m);
        const double term = exp_tab(walk_exponent(w, m, nu, A, B), T) * (1.0 + w.P);
        if (Comp) {
            const double y = term - c, t = S + y;
            c = (t - S) - y;
            S = t;
        } else {
            S += term;
        }
        if (m == 0 || m == p.N) ends += term;
        walk_step(w, m);
    }
    return (S - c) - 0.5 * ends;
}

__device__ inline FixedOut paper_fixed(double nu, double x, int bins, double T, const double* E)
{
    const double tstar = (nu * nu > x) ? peak_solve(nu, x, E) : 0.0;
    Plan p;
    p.t0 = 0.0;
    p.h = T / (double)bins;
    p.N = bins;
    p.mc = (int)fmin(fmax(rint(tstar / p.h), 0.0), (double)bins);
    p.tref = (double)p.mc * p.h;
    double ch, sh;
    cosh_sinh(p.tref, ch, sh);
    const double em = expm1(0.5 * p.tref);               // sinh(t/2) = em (em + 2) / (2 (em + 1))
    const double sh2 = em * (em + 2.0) / (2.0 * (em + 1.0));
    const double A = 0.5 * x * ch, B = 0.5 * x * sh;
    FixedOut o;
    o.lscale = nu * p.tref - kLn2 - 2.0 * x * sh2 * sh2 - x;
    o.hs = p.h * (bins > kFixedPlainMax ? fixed_sum<true>(nu, p, A, B, E) : fixed_sum<false>(nu, p, A, B, E));
    return o;
}

// ---------------------------------------------------------------------------
// Temme's series for small x (Sec. IV-A, Eqs. "temme_main", "temme_initpq",
// "temme_initf") with Campbell's forward recurrence (Eq. "recurrence"), the
// paper's branch for x < 0.1 (Alg. 2). With nu = mu + M, M = floor(nu + 1/2),
// mu in [-1/2, 1/2):
//   K_mu = sum_k c_k f_k,  K_{mu+1} = (2/x) sum_k c_k h_k,  c_k = (x^2/4)^k / k!,
//   h_k = p_k - k f_k,  p_k = p_{k-1} / (k - mu),  q_k = q_{k-1} / (k + mu),
//   f_k = (k f_{k-1} + p_{k-1} + q_{k-1}) / (k^2 - mu^2),
//   p_0 = (x/2)^-mu Gamma(1+mu) / 2,  q_0 = (x/2)^mu Gamma(1-mu) / 2,
//   f_0 = (mu pi / sin(mu pi)) (cosh(s) Gamma1 + sinh(s)/s ln(2/x) Gamma2),
//   s = mu ln(2/x), Gamma1 = (1/Gamma(1-mu) - 1/Gamma(1+mu)) / (2 mu),
//   Gamma2 = (1/Gamma(1-mu) + 1/Gamma(1+mu)) / 2,
// then K_{eta+1} = (2 eta / x) K_eta + K_{eta-1} up to nu. Gamma1 and Gamma2 are
// even entire functions of mu; they are evaluated from Chebyshev coefficients in
// 8 mu^2 - 1 (kTemmeTab). The series stops when a
// term falls below 2^-53 of the sum (the paper caps it at 15000 terms).
// ---------------------------------------------------------------------------

__device__ __forceinline__ double cheb_eval(const double* c, double u)
{
    double b1 = 0.0, b2 = 0.0;
    for (int j = kTemmeCheb - 1; j >= 1; --j) {
        const double t = fma(2.0 * u, b1, c[j] - b2);
        b2 = b1;
        b1 = t;
    }
    return fma(u, b1, c[0] - b2);
}

// K_nu(x) for 0 < x (intended for x < 0.1, where the series converges in a few
// terms); returns K (not scaled).
__device__ inline double temme_k(double nu, double x, const TemmeCoef& C)
{
    const double M = floor(nu + 0.5);
    const double mu = nu - M;
    const double u = 8.0 * mu * mu - 1.0;
    const double G1 = cheb_eval(C.g1, u), G2 = cheb_eval(C.g2, u);
    const double rgp = G2 - mu * G1;                   // 1 / Gamma(1 + mu)
    const double rgm = G2 + mu * G1;                   // 1 / Gamma(1 - mu)
    const double lx = log(2.0 / x);
    const double sg = mu * lx;
    const double pimu = 3.14159265358979323846 * mu;
    const double fact = fabs(pimu) < 1e-8 ? 1.0 + pimu * pimu / 6.0 : pimu / sin(pimu);
    const double esg = exp(sg);
    const double chs = 0.5 * (esg + 1.0 / esg);
    const double shs_s = fabs(sg) < 1e-4 ? 1.0 + sg * sg / 6.0 : 0.5 * (esg - 1.0 / esg) / sg;
    double f = fact * (G1 * chs + G2 * shs_s * lx);
    double p = 0.5 * esg / rgp;                        // (x/2)^-mu Gamma(1+mu) / 2
    double q = 0.5 / (esg * rgm);                      // (x/2)^mu Gamma(1-mu) / 2
    const double d = 0.25 * x * x;
    double c = 1.0, sum = f, sum1 = p;
    for (int k = 1; k < 200; ++k) {
        const double kk = (double)k;
        f = (kk * f + p + q) / (kk * kk - mu * mu);
        c *= d / kk;
        p /= (kk - mu);
        q /= (kk + mu);
        const double del = c * f;
        sum += del;
        sum1 += c * (p - kk * f);
        if (fabs(del) < 1.1102230246251565e-16 * fabs(sum)) break;
    }
    double km = sum;                                   // K_mu
    double kp = sum1 * 2.0 / x;                        // K_{mu+1}
    // forward recurrence K_{eta+1} = (2 eta / x) K_eta + K_{eta-1}, eta = mu + 1, ..., nu - 1
    for (int j = 1; j < (int)M; ++j) {
        const double eta = mu + (double)j;
        const double kn = fma(2.0 * eta / x, kp, km);
        km = kp;
        kp = kn;
    }
    return M >= 1.0 ? kp : km;
}

}  // namespace bk
