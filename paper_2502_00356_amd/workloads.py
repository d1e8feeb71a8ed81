"""Seeded synthetic inputs for the K_nu and Matern workloads.

This module only draws random numbers and orders points; it holds none of the
method's arithmetic, so both the GPU path and the CPU oracle can be fed from it.
All draws use numpy's PCG64 generator (np.random.default_rng(seed)) in float64.

The paper evaluates K_nu over (nu, x) grids and builds Matern covariance
matrices over 2-D locations in the unit square (Sec. IV-C, Sec. V); the
workloads below have those shapes and value distributions.
"""
import numpy as np


def pairs_loguniform(n, seed, nu_lo, nu_hi, log10x_lo, log10x_hi):
    """n pairs with nu ~ U[nu_lo, nu_hi] and x log-uniform on [10^lo, 10^hi]."""
    rng = np.random.default_rng(seed)
    nu = rng.uniform(nu_lo, nu_hi, n)
    x = 10.0 ** rng.uniform(log10x_lo, log10x_hi, n)
    return nu, x


def small_pairs(n=4096, seed=1):
    """Small standalone set: nu ~ U[0.1, 4], x log-uniform on [1e-3, 1e2]."""
    return pairs_loguniform(n, seed, 0.1, 4.0, -3.0, 2.0)


def grid_pairs(n=1 << 24, seed=2, half_integer_fraction=0.01):
    """Standalone K_nu grid: nu ~ U[0.01, 10], x log-uniform on [1e-4, 1e3].
    A fraction of the entries (chosen without replacement) get nu = k + 1/2,
    k uniform in 0..9, so closed forms can be checked on them.
    Returns (nu, x, half_integer_index)."""
    rng = np.random.default_rng(seed)
    nu = rng.uniform(0.01, 10.0, n)
    x = 10.0 ** rng.uniform(-4.0, 3.0, n)
    m = int(round(half_integer_fraction * n))
    idx = np.sort(rng.choice(n, size=m, replace=False)) if m > 0 else np.zeros(0, np.int64)
    nu[idx] = rng.integers(0, 10, size=m) + 0.5
    return nu, x, idx


def training_pairs(n=1 << 20, seed=4):
    """Training set for the window predictor, same law as grid_pairs (no half-integers)."""
    return pairs_loguniform(n, seed, 0.01, 10.0, -4.0, 3.0)


def eval_pairs(n=1 << 24, seed=5):
    """Fresh evaluation set for the window predictor, same law."""
    return pairs_loguniform(n, seed, 0.01, 10.0, -4.0, 3.0)


def out_of_range_pairs(n=1 << 16, seed=6):
    """Pairs outside the predictor's training box: nu in (10, 20] or [0.001, 0.01),
    x in [1e-6, 1e-4) or (1e3, 1e4]; each coordinate picks its side at random."""
    rng = np.random.default_rng(seed)
    side_nu = rng.integers(0, 2, n).astype(bool)
    nu = np.where(side_nu, rng.uniform(10.0, 20.0, n) + 1e-9, rng.uniform(0.001, 0.01, n))
    side_x = rng.integers(0, 2, n).astype(bool)
    x = np.where(side_x, 10.0 ** rng.uniform(3.0, 4.0, n) * (1 + 1e-12), 10.0 ** rng.uniform(-6.0, -4.0, n) * (1 - 1e-12))
    return nu, x


def morton_order(xy, bits=16):
    """Permutation sorting 2-D points in [0,1]^2 along the Z-order (Morton) curve:
    coordinates are quantised to `bits` bits and their bits interleaved.
    Ties keep their input order (stable sort)."""
    q = np.clip((np.asarray(xy) * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(q.shape[0], dtype=np.int64)
    for b in range(bits):
        code |= ((q[:, 0] >> b) & 1) << (2 * b)
        code |= ((q[:, 1] >> b) & 1) << (2 * b + 1)
    return np.argsort(code, kind="stable")


def uniform_locations(n, seed, morton=True):
    """n locations uniform in [0,1]^2, as an (n, 2) float64 array, optionally
    Morton-sorted (Sec. IV-D orders locations this way)."""
    xy = np.random.default_rng(seed).random((n, 2))
    if morton:
        xy = xy[morton_order(xy)]
    return np.ascontiguousarray(xy)


def jittered_grid_locations(side=316, seed=7, jitter=0.4, morton=True):
    """side x side jittered grid in [0,1]^2: point (i, j) is
    ((i + 0.5 + u) / side, (j + 0.5 + v) / side), u, v ~ U[-jitter, jitter]."""
    rng = np.random.default_rng(seed)
    i, j = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    u = rng.uniform(-jitter, jitter, (side, side))
    v = rng.uniform(-jitter, jitter, (side, side))
    xy = np.stack([((i + 0.5 + u) / side).ravel(), ((j + 0.5 + v) / side).ravel()], axis=1)
    if morton:
        xy = xy[morton_order(xy)]
    return np.ascontiguousarray(xy)


# Workload parameter sets (sigma2, beta, nu) of the Matern configurations.
def gp_observations(xy, seed, length=0.05):
    """Observations for the likelihood workloads: one draw z ~ N(0, R) with the
    exponential correlation R_ij = exp(-|l_i - l_j| / length) (a closed form, not
    the K_nu path), standard normal noise through numpy's Cholesky factor. It gives
    z the spatial structure of the paper's synthetic fields; the likelihood itself
    is defined for any z."""
    r = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
    L = np.linalg.cholesky(np.exp(-r / length) + 1e-12 * np.eye(xy.shape[0]))
    return L @ np.random.default_rng(seed).standard_normal(xy.shape[0])


MATERN_SMALL = dict(n=1024, seed=0, sigma2=1.0, beta=0.1, nu=1.3, tile=1024, lower_only=0, morton=False)
MATERN_MEDIUM = dict(n=40000, seed=3, sigma2=1.0, beta=0.05, nus=(0.8, 2.3), tile=960, lower_only=1)
MATERN_LARGE = dict(side=316, seed=7, sigma2=1.0, beta=0.02, nu=3.7, tile=1024, lower_only=1)
# likelihood and gradient on a dense n x n covariance (Cholesky on the GPU)
LOGLIK = dict(n=8192, seed=11, obs_seed=12, sigma2=1.0, beta=0.05, nu=0.8)
