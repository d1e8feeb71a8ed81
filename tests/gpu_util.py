"""Shared helpers of the GPU tests (no method arithmetic)."""
import numpy as np

DBL_MIN = np.finfo(np.float64).tiny

# Parity bars. Plain FP64: relative 1e-13. Mixed and learned: relative 2e-6.
TOL_PLAIN = 1e-13
TOL_MIXED = 2e-6


def rel_err(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.abs(got - ref) / np.abs(ref)
    e[(got == ref)] = 0.0
    return e


def k_result_err_ok(got, kref, tol):
    """Element-wise check of a K output (BK_RESULT_K) against the oracle's K: relative
    error <= tol where K is a normal double; where it underflows (x beyond ~708) both
    sides round once into the subnormal range, so |got - ref| <= tol ref + 2^-1074
    (one subnormal unit), which also holds for K = 0 past x ~ 745."""
    got = np.asarray(got, np.float64)
    kref = np.asarray(kref, np.float64)
    ok = np.empty(kref.shape, bool)
    nrm = kref >= DBL_MIN
    ok[nrm] = rel_err(got[nrm], kref[nrm]) <= tol
    ok[~nrm] = np.abs(got[~nrm] - kref[~nrm]) <= tol * kref[~nrm] + 2.0 ** -1074
    return ok


def re_metric(logk_got, logk_ref):
    """RE = log10(1 + |log K_ref - log K| / 2^-52), the accuracy metric of Sec. IV-C."""
    return np.log10(1.0 + np.abs(np.asarray(logk_got) - np.asarray(logk_ref)) / 2.0 ** -52)


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def packed_index(api, n, ts, lower, i, j):
    """Offsets in the packed tile output of global entries (i, j) (with lower_only,
    tile row i // ts must be at least tile column j // ts)."""
    i = np.asarray(i, np.int64)
    j = np.asarray(j, np.int64)
    I, J = i // ts, j // ts
    off = np.array([api.matern_tile_offset(n, ts, lower, int(a), int(b)) for a, b in zip(I, J)], dtype=np.int64)
    mI = np.minimum(ts, n - I * ts)
    return off + (i - I * ts) + (j - J * ts) * mI
