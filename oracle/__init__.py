"""CPU oracle for K_nu(x), the Matern covariance, the integration window, the
node-count rule and the window-predicting MLP.

TEST INFRASTRUCTURE. Only tests/, the smoke check and the benchmark's CPU
baseline import this package. It shares no code with the GPU library
(paper_2502_00356_amd) and neither imports the other.

Contents
  besselk(nu, x)            K_nu(x), log K_nu(x), e^x K_nu(x) by adaptive
                            Gauss-Kronrod in long double (besselk_oracle.c)
  matern_entries(...)       selected Matern entries, same quadrature
  matern_full(...)          a whole small matrix
  besselk_deriv(nu, x)      dK/dx and dK/dnu, the integrals differentiated under
                            the integral sign, same quadrature
  matern_grad_entries(...)  Matern entries with their beta and nu derivatives
  digamma(v)                psi(v) in long double
  matern_loglik(...)        Gaussian log-likelihood of observations under the
                            Matern covariance, and its gradient (numpy / scipy)
  window(nu, x, L)          t_max, g(t_max), [t0, t1] by bisection
  node_count(...)           node-count rule for a per-entry window
  mlp_*                     numpy float64 forward / loss / backward / Adam
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_P = ctypes.POINTER(ctypes.c_double)
_PI64 = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_besselk.restype = ctypes.c_int64
        lib.oracle_besselk.argtypes = [_P, _P, _P, _P, _P, ctypes.c_int64]
        lib.oracle_matern.restype = ctypes.c_int64
        lib.oracle_matern.argtypes = [_P, _P, _P, _P, _PI64, _PI64, ctypes.c_int64,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double, _P]
        lib.oracle_window.restype = None
        lib.oracle_window.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_double, _P, _P, _P, _P]
        lib.oracle_fixed_window.restype = None
        lib.oracle_fixed_window.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_int, ctypes.c_double, _P, _P]
        lib.oracle_log_truncated.restype = ctypes.c_int64
        lib.oracle_log_truncated.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_double, _P]
        lib.oracle_logintegrand.restype = None
        lib.oracle_logintegrand.argtypes = [_P, _P, _P, _P, ctypes.c_int64]
        lib.oracle_besselk_deriv.restype = ctypes.c_int64
        lib.oracle_besselk_deriv.argtypes = [_P, _P, ctypes.c_int64, _P, _P, _P, _P]
        lib.oracle_digamma.restype = None
        lib.oracle_digamma.argtypes = [_P, _P, ctypes.c_int64]
        lib.oracle_matern_grad.restype = ctypes.c_int64
        lib.oracle_matern_grad.argtypes = [_P, _P, _P, _P, _PI64, _PI64, ctypes.c_int64,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double, _P, _P, _P]
        _lib = lib
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_P)


def besselk(nu, x):
    """K_nu(x) by the integral of Sec. IV-B (Eq. "integral").

    Returns (k, logk, kscaled) as float64 arrays, kscaled = e^x K_nu(x).
    Domain: x < 0 or NaN -> NaN; x == 0 -> +inf; nu enters through |nu|.
    Raises if the adaptive quadrature failed to converge on any entry."""
    nu, x = np.broadcast_arrays(_d(nu), _d(x))
    nu, x = _d(nu).ravel(), _d(x).ravel()
    n = x.size
    k, lk, ks = np.empty(n), np.empty(n), np.empty(n)
    bad = _load().oracle_besselk(_ptr(nu), _ptr(x), _ptr(lk), _ptr(k), _ptr(ks), n)
    if bad:
        raise RuntimeError("oracle quadrature did not converge on %d entries" % bad)
    return k, lk, ks


def besselk_deriv(nu, x):
    """Partial derivatives of K_nu(x), by differentiating the integral of Sec. IV-B
    under the integral sign (derivatives are the paper's future work, Sec. VI):
        dK/dx  = -int_0^inf cosh t exp(-x cosh t) cosh(nu t) dt
        dK/dnu =  int_0^inf t sinh(nu t) exp(-x cosh t) dt      (sign of nu for nu < 0)
    Returns a dict of float64 arrays, for x > 0:
      dx, dnu        the derivatives
      log_mdx        log(-dK/dx);       log_dnu   log|dK/dnu|
      scaled_dx      e^x dK/dx;         scaled_dnu e^x dK/dnu  (exponentiated in long double)"""
    nu, x = (a.ravel() for a in np.broadcast_arrays(_d(nu), _d(x)))
    nu, x = _d(nu), _d(x)
    lmdx, ldnu, smdx, sdnu = (np.empty(x.size) for _ in range(4))
    bad = _load().oracle_besselk_deriv(_ptr(nu), _ptr(x), x.size, _ptr(lmdx), _ptr(ldnu), _ptr(smdx), _ptr(sdnu))
    if bad:
        raise RuntimeError("oracle quadrature did not converge on %d entries" % bad)
    sg = np.sign(nu)
    return {"dx": -np.exp(lmdx), "dnu": sg * np.exp(ldnu), "log_mdx": lmdx, "log_dnu": ldnu,
            "scaled_dx": -smdx, "scaled_dnu": sg * sdnu}


def digamma(v):
    """psi(v) = Gamma'(v) / Gamma(v) for v > 0, long double."""
    v = _d(v).ravel()
    out = np.empty(v.size)
    _load().oracle_digamma(_ptr(v), _ptr(out), v.size)
    return out


def matern_grad_entries(row_xy, col_xy, ri, ci, sigma2, beta, nu):
    """Matern entries M (Sec. III-A) and dM/dbeta, dM/dnu at entries (ri[e], ci[e]).
    Returns (M, dM/dbeta, dM/dnu)."""
    rx, ry = _d(row_xy[:, 0]), _d(row_xy[:, 1])
    cx, cy = _d(col_xy[:, 0]), _d(col_xy[:, 1])
    ri = np.ascontiguousarray(ri, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int64)
    m, db, dn = np.empty(ri.size), np.empty(ri.size), np.empty(ri.size)
    bad = _load().oracle_matern_grad(_ptr(rx), _ptr(ry), _ptr(cx), _ptr(cy),
                                     ri.ctypes.data_as(_PI64), ci.ctypes.data_as(_PI64), ri.size,
                                     float(sigma2), float(beta), float(nu), _ptr(m), _ptr(db), _ptr(dn))
    if bad:
        raise RuntimeError("oracle quadrature did not converge on %d entries" % bad)
    return m, db, dn


def matern_full_grad(xy, sigma2, beta, nu):
    """Whole n x n Matern matrix and its beta and nu derivative matrices."""
    n = xy.shape[0]
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    m, db, dn = matern_grad_entries(xy, xy, ii.ravel(), jj.ravel(), sigma2, beta, nu)
    return m.reshape(n, n), db.reshape(n, n), dn.reshape(n, n)


def matern_loglik(xy, z, sigma2, beta, nu, grad=False, details=False):
    """Gaussian log-likelihood of observations z (n) at locations xy (n x 2) under
    the Matern covariance Sigma (Sec. III-A; the likelihood the paper maximises):
        l = -1/2 z^T Sigma^-1 z - 1/2 log det Sigma - n/2 log(2 pi),
    by a Cholesky factorisation Sigma = L L^T (log det Sigma = 2 sum log L_ii).
    With grad=True also returns (dl/dsigma2, dl/dbeta, dl/dnu) from
        dl/dtheta = 1/2 a^T (dSigma/dtheta) a - 1/2 tr(Sigma^-1 dSigma/dtheta),
    a = Sigma^-1 z, and dSigma/dsigma2 = Sigma / sigma2. details=True returns a dict
    with the parts (quad, logdet, cond, and per parameter the two gradient terms)."""
    import scipy.linalg as sl
    z = np.asarray(z, np.float64)
    n = z.size
    if grad:
        S, dB, dN = matern_full_grad(xy, sigma2, beta, nu)
    else:
        S = matern_full(xy, sigma2, beta, nu)
    L = np.linalg.cholesky(S)
    w = sl.solve_triangular(L, z, lower=True)
    quad = float(w @ w)
    logdet = 2.0 * float(np.sum(np.log(np.diag(L))))
    ll = -0.5 * quad - 0.5 * logdet - 0.5 * n * math.log(2.0 * math.pi)
    info = {"ll": ll, "quad": quad, "logdet": logdet}
    if details:
        info["cond"] = float(np.linalg.cond(S))
    if not grad:
        return info if details else ll
    a = sl.cho_solve((L, True), z)
    Sinv = sl.cho_solve((L, True), np.eye(n))
    g, t1, t2 = [], [], []
    for dS in (S / sigma2, dB, dN):
        t1.append(0.5 * float(a @ dS @ a))
        t2.append(0.5 * float(np.sum(Sinv * dS)))
        g.append(t1[-1] - t2[-1])
    if details:
        info.update(grad=np.array(g), t_quad=np.array(t1), t_trace=np.array(t2))
        return info
    return ll, np.array(g)


def fixed_window(nu, x, bins=40, T=9.0):
    """Trapezoid sum of the paper's refined algorithm (Sec. IV-C, Alg. 2, x >= 0.1):
    b bins on the fixed window [0, T]. Returns (S, log S)."""
    nu, x = (a.ravel() for a in np.broadcast_arrays(_d(nu), _d(x)))
    nu, x = _d(nu), _d(x)
    ls, s = np.empty(x.size), np.empty(x.size)
    _load().oracle_fixed_window(_ptr(nu), _ptr(x), x.size, int(bins), float(T), _ptr(ls), _ptr(s))
    return s, ls


def log_truncated(nu, x, L):
    """log of int_0^L exp(-x cosh t) cosh(nu t) dt (RBK of the paper's Alg. 1)."""
    nu, x = (a.ravel() for a in np.broadcast_arrays(_d(nu), _d(x)))
    nu, x = _d(nu), _d(x)
    out = np.empty(x.size)
    bad = _load().oracle_log_truncated(_ptr(nu), _ptr(x), x.size, float(L), _ptr(out))
    if bad:
        raise RuntimeError("oracle quadrature did not converge on %d entries" % bad)
    return out


def empirical_upper_bound(x_grid, nu_grid, tol=1e-9, candidates=None):
    """The paper's empirical upper-bound finder (Alg. 1) with this oracle in place of
    the reference library: the smallest candidate L such that
    max over the (x, nu) grid of |log K - log int_0^L| <= tol.
    Returns (L, max abs error at L), or (None, error at the largest candidate)."""
    X, V = np.meshgrid(np.asarray(x_grid, float), np.asarray(nu_grid, float), indexing="ij")
    X, V = X.ravel(), V.ravel()
    _, lk, _ = besselk(V, X)
    if candidates is None:
        candidates = np.arange(1.0, 20.01, 0.25)
    err = None
    for L in candidates:
        err = float(np.max(np.abs(lk - log_truncated(V, X, L))))
        if err <= tol:
            return float(L), err
    return None, err


def logintegrand(nu, x, t):
    """g_{nu,x}(t) = log cosh(nu t) - x cosh t (Sec. IV-B, Eq. "logintegrand")."""
    nu, x, t = (a.ravel() for a in np.broadcast_arrays(_d(nu), _d(x), _d(t)))
    nu, x, t = _d(nu), _d(x), _d(t)
    out = np.empty(x.size)
    _load().oracle_logintegrand(_ptr(nu), _ptr(x), _ptr(t), _ptr(out), x.size)
    return out


def matern_entries(row_xy, col_xy, ri, ci, sigma2, beta, nu):
    """Matern covariance (Sec. III-A) at entries (ri[e], ci[e]) of the matrix whose
    rows are the locations row_xy (n1 x 2) and columns col_xy (n2 x 2)."""
    rx, ry = _d(row_xy[:, 0]), _d(row_xy[:, 1])
    cx, cy = _d(col_xy[:, 0]), _d(col_xy[:, 1])
    ri = np.ascontiguousarray(ri, dtype=np.int64)
    ci = np.ascontiguousarray(ci, dtype=np.int64)
    out = np.empty(ri.size)
    bad = _load().oracle_matern(_ptr(rx), _ptr(ry), _ptr(cx), _ptr(cy),
                                ri.ctypes.data_as(_PI64), ci.ctypes.data_as(_PI64), ri.size,
                                float(sigma2), float(beta), float(nu), _ptr(out))
    if bad:
        raise RuntimeError("oracle quadrature did not converge on %d entries" % bad)
    return out


def matern_full(xy, sigma2, beta, nu):
    """Whole n x n Matern matrix (row-major numpy array; A[i, j] = C(|l_i - l_j|))."""
    n = xy.shape[0]
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return matern_entries(xy, xy, ii.ravel(), jj.ravel(), sigma2, beta, nu).reshape(n, n)


def window(nu, x, L):
    """Window of Sec. IV-B at threshold g(t_max) - L, by bisection in long double.
    Returns (t_max, g_max, t0, t1)."""
    nu, x = (a.ravel() for a in np.broadcast_arrays(_d(nu), _d(x)))
    nu, x = _d(nu), _d(x)
    n = x.size
    tm, gm, t0, t1 = np.empty(n), np.empty(n), np.empty(n), np.empty(n)
    _load().oracle_window(_ptr(nu), _ptr(x), n, float(L), _ptr(tm), _ptr(gm), _ptr(t0), _ptr(t1))
    return tm, gm, t0, t1


# ---------------------------------------------------------------------------
# Node-count rule for a per-entry window.
#
# The paper fixes b = 40 bins on the fixed window [0, 9] (Sec. IV-C) and gives
# no rule for a window that varies per entry. The reading used here takes the
# classical error bound of the trapezoid rule for a function analytic in the
# strip |Im t| < a (Trefethen & Weideman, SIAM Review 56, 2014, Thm 5.1):
#     error <= 2 M_a / (exp(2 pi a / h) - 1),  M_a = int |f(t + i a)| dt.
# For f = exp(-x cosh t) cosh(nu t): |f(t + i a)| <= exp(-x cos(a) cosh t) cosh(nu t),
# so M_a / int f <= K_nu(x cos a) / K_nu(x) = exp(int_{x cos a}^{x} <cosh t>_z dz),
# with <cosh t>_z = K_{nu+1}(z)/K_nu(z) - nu/z <= 1 + (|nu| + 1)/z. Hence
#     log(M_a / int f) <= x (1 - cos a) + (|nu| + 1) log sec a,
# and any a in (0, pi/2) gives an admissible step
#     h(a) = 2 pi a / (Lq + log 2 + x (1 - cos a) + (|nu| + 1) log sec a),
# for relative error about exp(-Lq). The rule takes the best of a fixed set of
# a values and N = max(N_MIN, ceil((t1 - t0) / h)).
# ---------------------------------------------------------------------------

NODE_N_MIN = 4


def node_candidates():
    """The fixed set of strip half-widths a: (pi/2) 2^(-k/2) and (pi/2)(1 - 2^(-k/2)),
    k = 1..8, 15 distinct values in (0, pi/2)."""
    vals = set()
    for k in range(1, 9):
        f = 2.0 ** (-k / 2.0)
        vals.add((math.pi / 2) * f)
        vals.add((math.pi / 2) * (1.0 - f))
    return sorted(vals)


def node_step(nu, x, Lq):
    """Largest admissible trapezoid step h from the strip bound above."""
    nu, x = np.broadcast_arrays(_d(nu), _d(x))
    best = np.zeros(x.shape)
    for a in node_candidates():
        den = Lq + math.log(2.0) + x * (1.0 - math.cos(a)) + (np.abs(nu) + 1.0) * math.log(1.0 / math.cos(a))
        best = np.maximum(best, 2.0 * math.pi * a / den)
    return best


def node_count(nu, x, t0, t1, Lq, n_min=NODE_N_MIN):
    """Number of trapezoid intervals N for the window [t0, t1] (integer array)."""
    h = node_step(nu, x, Lq)
    return np.maximum(n_min, np.ceil((np.asarray(t1) - np.asarray(t0)) / h)).astype(np.int64)


def node_count_ratio(nu, x, t0, t1, Lq):
    """(t1 - t0) / h before rounding up, for tie handling in comparisons."""
    return (np.asarray(t1) - np.asarray(t0)) / node_step(nu, x, Lq)


# ---------------------------------------------------------------------------
# Window-predicting MLP, 2 -> 64 -> 64 -> 3, ReLU hidden activations, float64.
# Parameters are a dict with W1 (64x2), b1 (64), W2 (64x64), b2 (64), W3 (3x64), b3 (3);
# y = W3 relu(W2 relu(W1 u + b1) + b2) + b3 for an input row u.
# ---------------------------------------------------------------------------

MLP_SHAPES = (("W1", (64, 2)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)),
              ("W3", (3, 64)), ("b3", (3,)))


def mlp_forward(p, u):
    """Forward pass for a batch u (B x 2). Returns (y, cache)."""
    z1 = u @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (u, z1, h1, z2, h2)


def mlp_loss(y, target, tau):
    """Expectile (asymmetric squared) loss averaged over the batch:
    sum_k mean_b |tau_k - 1[e_bk < 0]| e_bk^2, e = target - y.
    tau_k near 1 penalises under-prediction of output k more than over-prediction."""
    e = target - y
    w = np.where(e < 0.0, 1.0 - tau[None, :], tau[None, :])
    return float(np.sum(w * e * e) / y.shape[0])


def mlp_backward(p, cache, y, target, tau):
    """Gradients of mlp_loss with respect to every parameter (dict)."""
    u, z1, h1, z2, h2 = cache
    B = y.shape[0]
    e = target - y
    w = np.where(e < 0.0, 1.0 - tau[None, :], tau[None, :])
    gy = -2.0 * w * e / B
    g = {"W3": gy.T @ h2, "b3": gy.sum(0)}
    gh2 = (gy @ p["W3"]) * (z2 > 0.0)
    g["W2"] = gh2.T @ h1
    g["b2"] = gh2.sum(0)
    gh1 = (gh2 @ p["W2"]) * (z1 > 0.0)
    g["W1"] = gh1.T @ u
    g["b1"] = gh1.sum(0)
    return g


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, ICLR 2015, Algorithm 1), in place.
    step is the 1-based step count used for bias correction."""
    for k in p:
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mh = m[k] / (1.0 - beta1 ** step)
        vh = v[k] / (1.0 - beta2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
