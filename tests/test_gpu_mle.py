"""GPU parity of the Gaussian log-likelihood and its gradient (bk_matern_loglik)
against the oracle (long-double Matern entries, numpy / scipy Cholesky).

Both sides factorise a covariance whose entries agree to ~1e-14, so the bar is the
first-order perturbation bound of the likelihood: an entry-wise relative error d
moves z^T Sigma^-1 z by at most about cond(Sigma) d |quad| and log det by
n cond(Sigma) d; with d = 1e-13 and a factor 10 of slack,
  |dl| <= 1e-12 cond(Sigma) (|quad| + n),
and each gradient component by 1e-12 cond(Sigma)^2 times the sum of its two terms'
magnitudes (Sigma^-1 enters twice)."""
import numpy as np
import pytest

from gpu_util import to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_00356_amd import api
    return api


@pytest.mark.parametrize("n,beta,nu", [(300, 0.03, 0.8), (400, 0.05, 1.5), (257, 0.04, 3.7)])
def test_loglik_and_gradient(api, orc, n, beta, nu):
    from paper_2502_00356_amd import workloads as w
    xy = w.uniform_locations(n, seed=95)
    z = w.gp_observations(xy, seed=97, length=beta)
    s2 = 1.2
    ref = orc.matern_loglik(xy, z, s2, beta, nu, grad=True, details=True)
    lx, ly, zd = to_dev(xy[:, 0]), to_dev(xy[:, 1]), to_dev(z)
    ll = api.matern_loglik(lx, ly, zd, s2, beta, nu)
    ll_g, g = api.matern_loglik(lx, ly, zd, s2, beta, nu, grad=True)
    k = ref["cond"]
    tol = 1e-12 * k * (abs(ref["quad"]) + n)
    print("n=%d beta=%g nu=%g: cond %.3g, |dl| %.3g (bar %.3g), grad %s vs %s"
          % (n, beta, nu, k, abs(ll - ref["ll"]), tol, np.array(g), ref["grad"]))
    assert abs(ll - ref["ll"]) <= tol
    assert ll_g == ll
    gt = 1e-12 * k * k * (np.abs(ref["t_quad"]) + np.abs(ref["t_trace"]))
    assert np.all(np.abs(np.array(g) - ref["grad"]) <= gt)


def test_loglik_forms(api, orc):
    """The mixed and learned forms build Sigma to ~1e-7; their likelihood stays
    within the same perturbation bar at d = 2e-6."""
    import os
    from paper_2502_00356_amd import workloads as w
    n, beta, nu, s2 = 200, 0.03, 1.3, 0.9
    xy = w.uniform_locations(n, seed=99)
    z = w.gp_observations(xy, seed=101, length=beta)
    ref = orc.matern_loglik(xy, z, s2, beta, nu, details=True)
    lx, ly, zd = to_dev(xy[:, 0]), to_dev(xy[:, 1]), to_dev(z)
    tol = 2e-5 * ref["cond"] * (abs(ref["quad"]) + n)
    assert abs(api.matern_loglik(lx, ly, zd, s2, beta, nu, mode="mixed") - ref["ll"]) <= tol
    path = os.path.join(os.path.dirname(api.__file__), "models", "window_mlp.bin")
    if os.path.exists(path):
        m = api.Model(path)
        assert abs(api.matern_loglik(lx, ly, zd, s2, beta, nu, mode="learned", model=m) - ref["ll"]) <= tol


def test_loglik_rejects_bad_arguments(api):
    import torch
    a = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(api.BkError):
        api.matern_loglik(a, a, a, 1.0, 0.1, 1.0, grad=True, mode="mixed")
    with pytest.raises(api.BkError):
        api.matern_loglik(a, a, a, 0.0, 0.1, 1.0)
