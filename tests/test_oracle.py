"""Pins of the CPU oracle against facts fixed by mathematics, not by the oracle.

Each test names what it pins. The oracle's own formulas are never retyped here:
the references are closed forms (DLMF), identities, asymptotic expansions,
independent library implementations (mpmath, scipy) and exactness properties.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.special as sp

ULP = 2.0 ** -52


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.abs(a - b) / np.abs(b)


# ---------------------------------------------------------------- quadrature table
def test_gk15_table_exactness():
    """The 15-point Kronrod rule integrates x^j exactly for j <= 22 and the embedded
    7-point Gauss rule for j <= 13 (degrees 3n+1 and 2n-1 with n = 7)."""
    import re, os
    src = open(os.path.join(os.path.dirname(__file__), "..", "oracle", "gk15_table.h")).read()

    def arr(name):
        body = src.split(name + "[8] = {")[1].split("};")[0]
        return [mp.mpf(s.rstrip("L")) for s in re.findall(r"[-0-9.e]+L", body)]
    mp.mp.dps = 40
    X, WK, WG = arr("GK15_X"), arr("GK15_WK"), arr("GK15_WG")
    for j in range(0, 24):
        exact = mp.mpf(0) if j % 2 else mp.mpf(2) / (j + 1)
        k = sum(w * (x ** j + (-x) ** j) * (mp.mpf(0.5) if x == 0 else 1) for x, w in zip(X, WK))
        assert abs(k - exact) < mp.mpf("1e-33"), j
        if j <= 13:
            g = sum(w * (x ** j + (-x) ** j) * (mp.mpf(0.5) if x == 0 else 1) for x, w in zip(X, WG))
            assert abs(g - exact) < mp.mpf("1e-33"), j
    # K15 must NOT be exact at degree 24 (it is the 15-point Kronrod rule, not a Gauss rule)
    k24 = sum(w * 2 * x ** 24 * (mp.mpf(0.5) if x == 0 else 1) for x, w in zip(X, WK))
    assert abs(k24 - mp.mpf(2) / 25) > mp.mpf("1e-12")
    # Gauss nodes/weights are those of numpy's Gauss-Legendre n = 7
    xg, wg = np.polynomial.legendre.leggauss(7)
    gx = sorted([float(x) for x, w in zip(X, WG) if w != 0])
    assert np.allclose(gx, sorted(xg[xg >= -1e-15]), atol=1e-15)


# ---------------------------------------------------------------- closed forms
def half_integer_scaled(n, x):
    """e^x K_{n+1/2}(x) from DLMF 10.49.12 (finite sum; all terms positive)."""
    s = sum(math.factorial(n + k) / (math.factorial(k) * math.factorial(n - k)) / (2.0 * x) ** k
            for k in range(n + 1))
    return math.sqrt(math.pi / (2.0 * x)) * s


def test_half_integer_closed_forms(orc):
    xs = np.geomspace(1e-4, 1e3, 29)
    for n in range(0, 10):
        nu = np.full(xs.shape, n + 0.5)
        _, _, ks = orc.besselk(nu, xs)
        ref = np.array([half_integer_scaled(n, x) for x in xs])
        assert rel(ks, ref).max() < 8 * ULP, n


def test_matern_half_integer_closed_forms(orc):
    """Matern with nu = 1/2, 3/2, 5/2 reduces to exp, (1+z)exp, (1+z+z^2/3)exp."""
    rng = np.random.default_rng(11)
    xy = rng.random((40, 2))
    n = xy.shape[0]
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
    for nu, form in ((0.5, lambda z: np.exp(-z)),
                     (1.5, lambda z: (1 + z) * np.exp(-z)),
                     (2.5, lambda z: (1 + z + z * z / 3) * np.exp(-z))):
        beta, s2 = 0.07, 1.7
        c = orc.matern_entries(xy, xy, ii.ravel(), jj.ravel(), s2, beta, nu).reshape(n, n)
        ref = s2 * form(d / beta)
        assert np.allclose(np.diag(c), s2, rtol=0, atol=0)
        assert rel(c, ref).max() < 64 * ULP


# ---------------------------------------------------------------- identities
def test_recurrence(orc):
    """K_{nu+1}(x) = K_{nu-1}(x) + (2 nu / x) K_nu(x) (Sec. IV-A recurrence; DLMF 10.29.1)."""
    rng = np.random.default_rng(3)
    # dyadic orders so that nu - 1 and nu + 1 are exact in double (K_nu is
    # sensitive to the order: d ln K / d nu ~ ln(2 nu / x))
    nu = np.round(rng.uniform(1.0, 9.0, 400) * 1024) / 1024
    x = 10 ** rng.uniform(-3, 2.8, 400)
    _, _, kp = orc.besselk(nu + 1, x)
    _, _, km = orc.besselk(nu - 1, x)
    _, _, k0 = orc.besselk(nu, x)
    assert rel(km + 2 * nu / x * k0, kp).max() < 6 * ULP


def test_symmetry_and_domain(orc):
    nu = np.array([0.3, 2.2, 7.9]); x = np.array([0.01, 3.0, 300.0])
    a = orc.besselk(nu, x)[0]; b = orc.besselk(-nu, x)[0]
    assert np.array_equal(a, b)
    k, lk, ks = orc.besselk(np.array([1.0, 1.0, 1.0, np.nan]), np.array([0.0, -1.0, np.nan, 1.0]))
    assert k[0] == np.inf and np.isnan(k[1]) and np.isnan(k[2]) and np.isnan(k[3])


# ---------------------------------------------------------------- asymptotics
def test_small_x_asymptotics(orc):
    """K_nu(x) ~ Gamma(nu)/2 (2/x)^nu for nu > 0 and K_0(x) ~ -ln(x/2) - gamma (DLMF 10.30.2-3)."""
    for nu in (1.3, 2.7, 5.5, 9.9):
        x = np.array([1e-6, 1e-7])
        _, lk, _ = orc.besselk(np.full(2, nu), x)
        lead = math.lgamma(nu) - math.log(2.0) + nu * np.log(2.0 / x)
        # relative correction is O(x^2 / (nu - 1)) for nu > 1
        assert np.abs(lk - lead).max() < 1e-10
    x = np.array([1e-8, 1e-10])
    k, _, _ = orc.besselk(np.zeros(2), x)
    ref = -np.log(x / 2.0) - np.euler_gamma
    assert rel(k, ref).max() < 1e-14


def test_large_x_asymptotics(orc):
    """Hankel expansion e^x K_nu(x) ~ sqrt(pi/2x) sum_k a_k(nu) / x^k (DLMF 10.40.2);
    at x >= 600 with 12 terms the truncation is far below double rounding."""
    for nu in (0.01, 1.3, 4.4, 9.7):
        x = np.array([600.0, 800.0, 1000.0, 2500.0, 6000.0, 1e4])
        _, _, ks = orc.besselk(np.full(x.size, nu), x)
        mu = 4 * nu * nu
        ref = []
        for xv in x:
            s, a = 1.0, 1.0
            for k in range(1, 12):
                a *= (mu - (2 * k - 1) ** 2) / (k * 8.0)
                s += a / xv ** k
            ref.append(math.sqrt(math.pi / (2 * xv)) * s)
        assert rel(ks, ref).max() < 4 * ULP


# ---------------------------------------------------------------- independent libraries
def test_against_mpmath_grid(orc):
    """mpmath.besselk (30 digits) on a 24 x 24 grid over the paper's region and beyond."""
    mp.mp.dps = 30
    nus = np.linspace(0.01, 10.0, 24)
    xs = np.geomspace(1e-4, 1e3, 24)
    N, X = np.meshgrid(nus, xs, indexing="ij")
    _, _, ks = orc.besselk(N.ravel(), X.ravel())
    ref = np.array([float(mp.besselk(n, x) * mp.exp(x)) for n, x in zip(N.ravel(), X.ravel())])
    assert rel(ks, ref).max() < 2 * ULP


def test_against_scipy_random(orc):
    """scipy.special.kve (AMOS) on random pairs; AMOS itself carries ~1e-13 error."""
    rng = np.random.default_rng(5)
    nu = rng.uniform(0.01, 10, 20000)
    x = 10 ** rng.uniform(-4, 3, 20000)
    _, _, ks = orc.besselk(nu, x)
    assert rel(ks, sp.kve(nu, x)).max() < 1e-12


def test_brute_force_quadrature(orc):
    """Tanh-sinh quadrature of the defining integral at 40 digits (mpmath.quad) on a
    5 x 5 grid. The integrand is multiplied by e^x so that its scale is O(1): mpmath's
    stopping test is absolute, which would accept anything for K ~ e^-700."""
    mp.mp.dps = 40
    for nu in (0.05, 0.7, 2.3, 5.1, 9.6):
        for x in (2e-4, 0.03, 1.7, 40.0, 700.0):
            f = lambda t: mp.exp(-x * (mp.cosh(t) - 1)) * mp.cosh(nu * t)
            # beyond tmax the integrand is below e^-100 of its peak
            tmax = float(mp.asinh(nu / x) + mp.acosh(1 + 120 / x)) + 1
            ref = mp.quad(f, mp.linspace(0, tmax, 60))
            _, _, ks = orc.besselk(np.array([nu]), np.array([x]))
            assert abs(float((ks[0] - ref) / ref)) < 2 * ULP, (nu, x)


# ---------------------------------------------------------------- log-integrand and window
def test_logintegrand(orc):
    """g(0) = -x (Sec. IV-B) and g at other points against mpmath."""
    mp.mp.dps = 30
    rng = np.random.default_rng(8)
    nu = rng.uniform(0.01, 10, 50); x = 10 ** rng.uniform(-4, 3, 50); t = rng.uniform(0, 15, 50)
    assert np.array_equal(orc.logintegrand(nu, x, np.zeros(50)), -x)
    g = orc.logintegrand(nu, x, t)
    ref = np.array([float(mp.log(mp.cosh(a * c)) - b * mp.cosh(c)) for a, b, c in zip(nu, x, t)])
    assert np.all(np.abs(g - ref) <= 4 * ULP * np.maximum(1.0, np.abs(ref)))


def test_window_definition(orc):
    """t_max = 0 iff nu^2 <= x; g'(t_max) = 0 inside; g(t1) = g(t_max) - L and, when
    t0 > 0, g(t0) = g(t_max) - L, with the integrand above the threshold in between
    (Sec. IV-B window definition), all checked in mpmath."""
    mp.mp.dps = 40
    rng = np.random.default_rng(9)
    nu = rng.uniform(0.01, 10, 300); x = 10 ** rng.uniform(-4, 3, 300)
    L = 38.0
    tm, gm, t0, t1 = orc.window(nu, x, L)
    assert np.array_equal(tm == 0, nu * nu <= x)
    assert np.any(t0 > 0)
    for i in range(300):
        v, z = mp.mpf(nu[i]), mp.mpf(x[i])
        g = lambda t: mp.log(mp.cosh(v * t)) - z * mp.cosh(t)
        gp = lambda t: v * mp.tanh(v * t) - z * mp.sinh(t)
        if tm[i] > 0:
            assert abs(gp(mp.mpf(tm[i]))) < 1e-12 * (1 + float(v))
        assert abs(float(g(mp.mpf(t1[i])) - (mp.mpf(gm[i]) - L))) < 1e-9 * (1 + x[i])
        if t0[i] > 0:
            assert abs(float(g(mp.mpf(t0[i])) - (mp.mpf(gm[i]) - L))) < 1e-9
        else:
            assert float(g(0)) >= gm[i] - L - 1e-12
        mid = 0.5 * (t0[i] + t1[i])
        assert float(g(mp.mpf(mid))) > gm[i] - L


# ---------------------------------------------------------------- node-count rule
def test_node_rule_meets_its_bound(orc):
    """The strip-bound node rule with the oracle window gives a trapezoid sum within
    a small multiple of exp(-Lq) of mpmath's K_nu, at both tolerance levels used
    (the rule's claim, checked against an independent evaluation of K_nu)."""
    mp.mp.dps = 40
    rng = np.random.default_rng(10)
    nu = rng.uniform(0.01, 10, 60); x = 10 ** rng.uniform(-4, 3, 60)
    for L, Lq in ((38.0, 36.5), (16.0, 15.4)):
        tm, gm, t0, t1 = orc.window(nu, x, L)
        N = orc.node_count(nu, x, t0, t1, Lq)
        worst = 0.0
        for i in range(60):
            v, z = mp.mpf(nu[i]), mp.mpf(x[i])
            a, b, n = mp.mpf(t0[i]), mp.mpf(t1[i]), int(N[i])
            h = (b - a) / n
            s = mp.fsum(mp.exp(-z * mp.cosh(a + m * h)) * mp.cosh(v * (a + m * h)) * (mp.mpf(0.5) if m in (0, n) else 1)
                        for m in range(n + 1))
            ref = mp.besselk(v, z)
            worst = max(worst, abs(float(h * s / ref - 1)))
        assert worst < 20 * math.exp(-Lq), (L, worst)


def test_node_rule_tie_helper(orc):
    r = orc.node_count_ratio(np.array([1.0]), np.array([2.0]), np.array([0.0]), np.array([3.0]), 30.0)
    n = orc.node_count(np.array([1.0]), np.array([2.0]), np.array([0.0]), np.array([3.0]), 30.0)
    assert n[0] == max(4, math.ceil(r[0]))


# ---------------------------------------------------------------- MLP and Adam
def _params(seed=0):
    from oracle import MLP_SHAPES
    rng = np.random.default_rng(seed)
    return {k: rng.normal(0, 0.5, s) for k, s in MLP_SHAPES}


def test_mlp_forward_hand_case(orc):
    """Weights chosen so the network computes y = (relu(u0) + relu(u1), -relu(u0), 7)."""
    p = {k: np.zeros(s) for k, s in orc.MLP_SHAPES}
    p["W1"][0, 0] = 1.0; p["W1"][1, 1] = 1.0
    p["W2"][0, 0] = 1.0; p["W2"][1, 1] = 1.0
    p["W3"][0, 0] = 1.0; p["W3"][0, 1] = 1.0; p["W3"][1, 0] = -1.0; p["b3"][2] = 7.0
    u = np.array([[0.5, -2.0], [-1.0, 3.0], [2.0, 0.25]])
    y, _ = orc.mlp_forward(p, u)
    ref = np.array([[0.5, -0.5, 7.0], [3.0, 0.0, 7.0], [2.25, -2.0, 7.0]])
    assert np.array_equal(y, ref)


def test_mlp_loss_hand_values(orc):
    """Expectile loss on two hand-worked samples, one with every residual e = t - y
    positive (weights tau) and one with every residual negative (weights 1 - tau):
      sample 0: e = (1, 2, 3):    0.1*1 + 0.9*4 + 0.9*9 = 11.8
      sample 1: e = (-1, -1, -1): 0.9*1 + 0.1*1 + 0.1*1 = 1.1
    mean over the batch (summed over outputs): 6.45. Swapping tau and 1 - tau gives
    2.05, dropping the square 2.85, and dividing by outputs as well 2.15, so each of
    those slips fails."""
    y = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0]])
    t = np.array([[1.0, 2.0, 3.0], [0.0, 0.0, 0.0]])
    tau = np.array([0.1, 0.9, 0.9])
    assert orc.mlp_loss(y, t, tau) == pytest.approx(6.45, rel=1e-15)
    # a single output: tau = 0.9 weights an under-prediction (e > 0) nine times an
    # over-prediction of the same size
    one = np.array([0.9])
    assert orc.mlp_loss(np.array([[0.0]]), np.array([[2.0]]), one) == pytest.approx(3.6, rel=1e-15)
    assert orc.mlp_loss(np.array([[2.0]]), np.array([[0.0]]), one) == pytest.approx(0.4, rel=1e-15)


def test_mlp_backward_finite_differences(orc):
    """Analytic gradients against central differences of the loss."""
    p = _params(1)
    rng = np.random.default_rng(2)
    u = rng.uniform(-1, 1, (32, 2)); tgt = rng.normal(0, 1, (32, 3))
    tau = np.array([0.1, 0.9, 0.9])
    y, cache = orc.mlp_forward(p, u)
    g = orc.mlp_backward(p, cache, y, tgt, tau)
    for k in p:
        flat = p[k].ravel()
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]; eps = 1e-6
            flat[i] = old + eps; lp = orc.mlp_loss(orc.mlp_forward(p, u)[0], tgt, tau)
            flat[i] = old - eps; lm = orc.mlp_loss(orc.mlp_forward(p, u)[0], tgt, tau)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[k].ravel()[i]) <= 1e-6 * (1 + abs(fd)), (k, i)


def test_adam_first_step_is_signed_lr(orc):
    """With zero moments, the first bias-corrected Adam step moves each parameter by
    lr * g / (|g| + eps), i.e. -lr * sign(g) up to eps (Kingma & Ba 2015, Sec. 2)."""
    p = {"a": np.array([1.0, -2.0, 3.0])}
    g = {"a": np.array([0.3, -5.0, 1e-3])}
    m = {"a": np.zeros(3)}; v = {"a": np.zeros(3)}
    orc.adam_step(p, g, m, v, 1, lr=0.01, eps=0.0)
    assert np.allclose(p["a"], np.array([1.0, -2.0, 3.0]) - 0.01 * np.sign(g["a"]), rtol=0, atol=1e-15)


# ---------------------------------------------------------------- paper's fixed window and Alg. 1
def test_fixed_window_sum_converges_to_k(orc):
    """The fixed-window trapezoid sum tends to K_nu as the bins grow and the window
    covers the integrand (pinned to mpmath's K_nu through the main oracle)."""
    nu = np.array([0.3, 1.3, 4.7, 12.0]); x = np.array([0.2, 3.0, 40.0, 1.5])
    k, _, _ = orc.besselk(nu, x)
    s, _ = orc.fixed_window(nu, x, 8000, 16.0)
    assert rel(s, k).max() < 1e-13
    # with b = 1 the rule is h (f(0) + f(T)) / 2 exactly
    s1, _ = orc.fixed_window(np.array([1.0]), np.array([2.0]), 1, 3.0)
    f = lambda t: math.exp(-2.0 * math.cosh(t)) * math.cosh(t)
    assert abs(s1[0] - 1.5 * (f(0.0) + f(3.0))) <= 1e-16


def test_truncated_integral(orc):
    """int_0^L grows with L and reaches K_nu; at L = 0 it vanishes (log -> -inf is
    avoided by a tiny L) and small L matches the integrand times L."""
    nu = np.array([2.5]); x = np.array([0.7])
    vals = [orc.log_truncated(nu, x, L)[0] for L in (0.5, 1.0, 2.0, 4.0, 8.0, 16.0)]
    assert all(b > a for a, b in zip(vals[:4], vals[1:4]))
    assert all(b >= a for a, b in zip(vals, vals[1:]))
    _, lk, _ = orc.besselk(nu, x)
    assert abs(vals[-1] - lk[0]) < 1e-14
    L = 1e-6
    approx = math.log(L * math.exp(-0.7))          # f(0) = e^{-x}
    assert abs(orc.log_truncated(nu, x, L)[0] - approx) < 1e-9


def test_empirical_upper_bound_replay(orc):
    """Alg. 1 replayed with the oracle as the reference: over x in [0.1, 140] (the
    integral branch) and nu in (0, 20] the smallest bound reaching 1e-9 absolute in
    log K is at most the paper's t1 = 9 (Sec. IV-C)."""
    xs = np.geomspace(0.1, 140.0, 16)
    nus = np.linspace(0.05, 20.0, 16)
    L, err = orc.empirical_upper_bound(xs, nus, tol=1e-9)
    print("replayed upper bound: %s (max abs error %.3g)" % (L, err))
    assert L is not None and 5.0 <= L <= 9.0


# ---------------------------------------------------------------------------
# Derivatives (differentiation under the integral sign; the paper's future work,
# Sec. VI) and the Matern gradient.
# ---------------------------------------------------------------------------
def _log_close(a, b, rel=4e-16, abs_=2e-15):
    """|a - b| within rounding of log values of magnitude |b|."""
    return np.all(np.abs(a - b) <= abs_ + rel * np.abs(b))


def test_dx_integral_matches_recurrence(orc):
    """The direct integral of cosh t cosh(nu t) e^{-x cosh t} equals
    (K_{nu-1} + K_{nu+1}) / 2 (DLMF 10.29.2), with both K from the K integral."""
    rng = np.random.default_rng(31)
    nu = np.concatenate([rng.uniform(0.0, 12.0, 1500), [0.0, 0.5, 1.0, 2.0]])
    x = np.concatenate([10 ** rng.uniform(-4, 3, 1500), [1e-3, 0.7, 35.0, 900.0]])
    d = orc.besselk_deriv(nu, x)
    _, lkm, _ = orc.besselk(np.abs(nu - 1.0), x)
    _, lkp, _ = orc.besselk(nu + 1.0, x)
    ref = np.logaddexp(lkm, lkp) - math.log(2.0)
    assert _log_close(d["log_mdx"], ref)
    assert np.all(np.isfinite(d["log_mdx"])) and np.all(d["dx"][x < 700] < 0.0)


def test_dnu_half_order_closed_form(orc):
    """dK_nu/dnu at nu = 1/2 is sqrt(pi/(2x)) E1(2x) e^x (DLMF 10.38.7)."""
    x = 10 ** np.linspace(-3, 1.7, 60)
    d = orc.besselk_deriv(np.full(x.size, 0.5), x)
    ref = 0.5 * np.log(np.pi / (2 * x)) + np.log(sp.exp1(2 * x)) + x
    assert _log_close(d["log_dnu"], ref, rel=1e-15, abs_=3e-15)
    d = orc.besselk_deriv(np.full(x.size, -0.5), x)
    assert np.all(d["dnu"] < 0.0)


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_dnu_integer_order_closed_form(orc, n):
    """dK_nu/dnu at nu = n is (n!/2) (x/2)^-n sum_{k<n} (x/2)^k K_k(x) / ((n-k) k!)
    (DLMF 10.38.6), with K_k from the K integral."""
    x = np.array([0.01, 0.05, 0.3, 2.0, 7.5, 40.0, 300.0])
    d = orc.besselk_deriv(np.full(x.size, float(n)), x)
    lks = [orc.besselk(np.full(x.size, float(k)), x)[1] for k in range(n)]
    terms = np.stack([k * np.log(x / 2) + lks[k] - math.log((n - k) * math.factorial(k)) for k in range(n)])
    ref = math.log(math.factorial(n) / 2.0) - n * np.log(x / 2) + np.logaddexp.reduce(terms, axis=0)
    assert _log_close(d["log_dnu"], ref, rel=1e-15, abs_=4e-15)


def test_dnu_order_zero_and_sign(orc):
    x = np.array([1e-3, 0.5, 20.0])
    d = orc.besselk_deriv(np.zeros(3), x)
    assert np.all(d["dnu"] == 0.0)
    a = orc.besselk_deriv(np.full(3, 2.7), x)["dnu"]
    b = orc.besselk_deriv(np.full(3, -2.7), x)["dnu"]
    assert np.all(a > 0) and np.array_equal(a, -b)


def test_derivatives_against_mpmath(orc):
    """Both derivatives against mpmath's own Bessel K, differentiated numerically at
    30 digits (an independent implementation)."""
    mp.mp.dps = 30
    pts = [(0.3, 0.01), (1.7, 0.9), (4.2, 3.3), (9.5, 0.05), (0.05, 12.0), (6.0, 150.0), (13.0, 2.0)]
    nu = np.array([p[0] for p in pts]); x = np.array([p[1] for p in pts])
    d = orc.besselk_deriv(nu, x)
    for i, (v, z) in enumerate(pts):
        rx = float(mp.diff(lambda s: mp.besselk(v, s), z))
        rn = float(mp.diff(lambda s: mp.besselk(s, z), v))
        assert abs(d["dx"][i] / rx - 1) < 1e-14, (v, z)
        assert abs(d["dnu"][i] / rn - 1) < 1e-14, (v, z)


def test_digamma(orc):
    v = np.array([1e-3, 0.1, 0.5, 1.0, 2.3, 7.7, 19.5, 20.5, 140.0])
    got = orc.digamma(v)
    assert np.allclose(got, sp.digamma(v), rtol=2e-15, atol=0)
    assert abs(orc.digamma(np.array([1.0]))[0] + 0.57721566490153286061) < 1e-16


def test_matern_grad_closed_forms(orc):
    """nu = 1/2: M = s2 e^{-z}, dM/dbeta = s2 z e^{-z} / beta,
    dM/dnu = s2 (e^{-z} (ln 2z + gamma) + e^{z} E1(2z)) (from DLMF 10.38.7 and
    psi(1/2) = -gamma - 2 ln 2); nu = 3/2: dM/dbeta = s2 z^2 e^{-z} / beta."""
    rng = np.random.default_rng(37)
    xy = rng.uniform(0, 1, (40, 2))
    ii, jj = np.meshgrid(np.arange(40), np.arange(40), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    s2, beta = 1.7, 0.13
    r = np.sqrt(((xy[ii] - xy[jj]) ** 2).sum(1))
    z = r / beta
    m, db, dn = orc.matern_grad_entries(xy, xy, ii, jj, s2, beta, 0.5)
    off = r > 0
    assert np.allclose(m[off], s2 * np.exp(-z[off]), rtol=1e-14, atol=0)
    assert np.allclose(db[off], s2 * z[off] * np.exp(-z[off]) / beta, rtol=1e-14, atol=0)
    zo = z[off]
    ref = s2 * (np.exp(-zo) * (np.log(2 * zo) + np.euler_gamma) + np.exp(zo) * sp.exp1(2 * zo))
    scale = s2 * (np.exp(-zo) * (np.abs(np.log(2 * zo)) + 1) + np.exp(zo) * sp.exp1(2 * zo))
    assert np.all(np.abs(dn[off] - ref) <= 1e-14 * scale)
    assert np.all(m[~off] == s2) and np.all(db[~off] == 0) and np.all(dn[~off] == 0)
    _, db, _ = orc.matern_grad_entries(xy, xy, ii, jj, s2, beta, 1.5)
    assert np.allclose(db[off], s2 * z[off] ** 2 * np.exp(-z[off]) / beta, rtol=1e-14, atol=0)


def test_matern_grad_finite_differences(orc):
    """dM/dbeta and dM/dnu against fourth-order central differences of the oracle's
    own Matern entries (a different code path: no derivative integral)."""
    rng = np.random.default_rng(41)
    xy = rng.uniform(0, 1, (12, 2))
    ii, jj = np.triu_indices(12, 1)
    s2, beta, nu = 1.3, 0.2, 2.3
    _, db, dn = orc.matern_grad_entries(xy, xy, ii, jj, s2, beta, nu)
    f = lambda b, v: orc.matern_entries(xy, xy, ii, jj, s2, b, v)
    hb, hv = 1e-3 * beta, 1e-3
    fdb = (8 * (f(beta + hb, nu) - f(beta - hb, nu)) - (f(beta + 2 * hb, nu) - f(beta - 2 * hb, nu))) / (12 * hb)
    fdn = (8 * (f(beta, nu + hv) - f(beta, nu - hv)) - (f(beta, nu + 2 * hv) - f(beta, nu - 2 * hv))) / (12 * hv)
    assert np.allclose(db, fdb, rtol=1e-9, atol=1e-12)
    assert np.allclose(dn, fdn, rtol=1e-8, atol=1e-11)


# ---------------------------------------------------------------------------
# Gaussian log-likelihood (the downstream use of the Matern matrix, Sec. III-A)
# ---------------------------------------------------------------------------
def test_loglik_exponential_kernel_against_scipy(orc):
    """nu = 1/2 (exponential kernel, closed form sigma2 e^{-r/beta}): the oracle's
    likelihood equals scipy's multivariate normal log-density of that matrix."""
    from scipy.stats import multivariate_normal
    rng = np.random.default_rng(43)
    n = 60
    xy = rng.uniform(0, 1, (n, 2))
    z = rng.standard_normal(n)
    s2, beta = 1.3, 0.2
    r = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
    ref = multivariate_normal(mean=np.zeros(n), cov=s2 * np.exp(-r / beta)).logpdf(z)
    assert abs(orc.matern_loglik(xy, z, s2, beta, 0.5) - ref) <= 1e-10 * abs(ref)


def test_loglik_gradient_finite_differences(orc):
    rng = np.random.default_rng(47)
    n = 40
    xy = rng.uniform(0, 1, (n, 2))
    z = rng.standard_normal(n)
    th = np.array([1.1, 0.15, 1.7])
    ll, g = orc.matern_loglik(xy, z, *th, grad=True)
    f = lambda t: orc.matern_loglik(xy, z, *t)
    for k in range(3):
        h = 1e-4 * th[k]
        e = np.zeros(3); e[k] = h
        fd = (8 * (f(th + e) - f(th - e)) - (f(th + 2 * e) - f(th - 2 * e))) / (12 * h)
        assert abs(g[k] - fd) <= 1e-6 * (abs(fd) + 1.0), (k, g[k], fd)
