"""GPU parity of the paper's refined algorithm (Sec. IV-C, Alg. 2; Alg. 3 for
tiles): the fixed-window branch (x >= 0.1) against the oracle of the same finite
sum, the Temme branch (x < 0.1, Sec. IV-A) against K_nu itself, and the fixed
window's accuracy against K_nu as a function of the number of bins b."""
import math

import numpy as np
import pytest

from gpu_util import DBL_MIN, TOL_PLAIN, re_metric, rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_00356_amd import api
    return api


def _paper_region(n, seed):
    """(nu, x) over the paper's study region for this branch: nu in (0, 20],
    x in [0.1, 140] (Sec. IV-C)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(1e-3, 20.0, n), 10 ** rng.uniform(-1.0, math.log10(140.0), n)


@pytest.mark.parametrize("bins,T", [(40, 9.0), (16, 9.0), (128, 9.0), (200, 14.0), (5000, 14.0)])
def test_fixed_window_sum_matches_oracle(api, orc, bins, T):
    """x >= 0.1: the b-bin trapezoid on [0, T] against the oracle's long-double sum."""
    import torch
    nu, x = _paper_region(20000, seed=bins)
    s_ref, ls_ref = orc.fixed_window(nu, x, bins, T)
    got = api.besselk(to_dev(nu), to_dev(x), mode="paper", bins=bins, t_upper=T)
    lg = api.besselk(to_dev(nu), to_dev(x), mode="paper", bins=bins, t_upper=T, result=api.RESULT_LOG)
    torch.cuda.synchronize()
    m = s_ref >= DBL_MIN
    assert rel_err(got.cpu().numpy()[m], s_ref[m]).max() <= TOL_PLAIN
    assert np.all(np.abs(lg.cpu().numpy() - ls_ref) <= TOL_PLAIN + 4e-16 * np.abs(ls_ref))


def test_bins_accuracy_tradeoff(api, orc):
    """Accuracy of the fixed window against K_nu (the oracle's integral) grows with b
    (the paper's observation, Sec. V-C); printed as the RE metric of Sec. IV-C."""
    import torch
    nu, x = _paper_region(4000, seed=7)
    _, lk, _ = orc.besselk(nu, x)
    prev = None
    for bins in (16, 40, 128, 400):
        lg = api.besselk(to_dev(nu), to_dev(x), mode="paper", bins=bins, result=api.RESULT_LOG)
        torch.cuda.synchronize()
        re = re_metric(lg.cpu().numpy(), lk)
        small = x < 10
        print("b=%d: max RE %.3f (x < 10: %.3f, x >= 10: %.3f)" % (bins, re.max(), re[small].max(), re[~small].max()))
        if prev is not None:
            assert re.max() <= prev + 1e-9
        prev = re.max()


def test_fixed_window_matern(api, orc):
    """Alg. 3 with the refined BesselK: tiles against sigma2 2^(1-nu)/Gamma(nu) z^nu
    times the oracle's fixed-window sum (z >= 0.1) or K_nu (z < 0.1)."""
    import torch
    from paper_2502_00356_amd import workloads as w
    xy = w.uniform_locations(200, seed=61)
    nu, beta, s2 = 1.3, 0.1, 1.5
    lx, ly = to_dev(xy[:, 0]), to_dev(xy[:, 1])
    out = api.matern_tiles(lx, ly, s2, beta, nu, 64, 1, mode="paper")
    torch.cuda.synchronize()
    A = api.unpack_tiles(out, 200, 64, 1).numpy()
    d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
    z = d / beta
    off = z > 0
    s, _ = orc.fixed_window(np.full(off.sum(), nu), z[off], 40, 9.0)
    kk, _, _ = orc.besselk(np.full(off.sum(), nu), z[off])
    s = np.where(z[off] < 0.1, kk, s)
    ref = np.full(z.shape, s2)
    ref[off] = s2 * 2.0 ** (1 - nu) / math.gamma(nu) * z[off] ** nu * s
    assert rel_err(A, ref).max() <= 1e-13


def test_invalid_bins(api):
    import torch
    a = torch.ones(4, dtype=torch.float64, device="cuda")
    with pytest.raises(api.BkError):
        api.besselk(a, a, mode="paper", bins=-3)


def test_temme_branch_matches_k(api, orc):
    """x < 0.1: Temme's series with Campbell's forward recurrence computes K_nu itself;
    within 1e-13 of the oracle, including integer and half-integer orders."""
    import torch
    rng = np.random.default_rng(71)
    nu = np.concatenate([rng.uniform(0.0, 10.0, 20000), np.arange(0, 10.5, 0.5), np.arange(0, 10.5, 0.5)])
    x = np.concatenate([10 ** rng.uniform(-4.0, -1.0, 20000), np.full(21, 0.0999), np.full(21, 1e-4)])
    k, _, _ = orc.besselk(nu, x)
    got = api.besselk(to_dev(nu), to_dev(x), mode="paper")
    torch.cuda.synchronize()
    e = rel_err(got.cpu().numpy(), k)
    print("Temme branch: max rel %.3g" % e.max())
    assert e.max() <= TOL_PLAIN


def test_refined_algorithm_over_paper_region(api, orc):
    """Alg. 2 over (nu, x) in (0, 20] x [0.001, 140]: Temme below x = 0.1, the b = 40
    fixed window above; each branch against its own oracle."""
    import torch
    rng = np.random.default_rng(73)
    nu = rng.uniform(1e-3, 20.0, 20000)
    x = 10 ** rng.uniform(-3.0, math.log10(140.0), 20000)
    got = api.besselk(to_dev(nu), to_dev(x), mode="paper")
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    small = x < 0.1
    k, _, _ = orc.besselk(nu[small], x[small])
    s, _ = orc.fixed_window(nu[~small], x[~small], 40, 9.0)
    assert rel_err(got[small], k).max() <= TOL_PLAIN
    m = s >= DBL_MIN
    assert rel_err(got[~small][m], s[m]).max() <= TOL_PLAIN
