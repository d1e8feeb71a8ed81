"""GPU parity of tiled Matern covariance generation (Sec. III-A formula, Alg. 3)
against the CPU oracle, plus the matrix invariants."""
import numpy as np
import pytest

from gpu_util import TOL_MIXED, TOL_PLAIN, rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_00356_amd import api
    return api


def _dense(api, xy, sigma2, beta, nu, ts, lower, mode, out_dtype=0):
    import torch
    lx, ly = to_dev(xy[:, 0]), to_dev(xy[:, 1])
    out = api.matern_tiles(lx, ly, sigma2, beta, nu, ts, lower, mode=mode, out_dtype=out_dtype)
    torch.cuda.synchronize()
    return api.unpack_tiles(out, xy.shape[0], ts, lower).double().numpy(), out


@pytest.mark.parametrize("mode,tol", [("plain", TOL_PLAIN), ("mixed", TOL_MIXED)])
@pytest.mark.parametrize("n,ts,lower", [(300, 300, 0), (350, 100, 1), (350, 64, 0), (130, 1000, 1), (1, 7, 1)])
def test_tiles_match_oracle(api, orc, mode, tol, n, ts, lower):
    """Small matrices, several tilings (ragged last tile, single tile, tile larger
    than n, one location), every entry against the oracle."""
    from paper_2502_00356_amd import workloads as w
    xy = w.uniform_locations(n, seed=20 + n)
    A, _ = _dense(api, xy, 1.3, 0.1, 1.3, ts, lower, mode)
    R = orc.matern_full(xy, 1.3, 0.1, 1.3)
    assert rel_err(A, R).max() <= tol


def test_small_matrix_config(api, orc):
    """n = 1,024 uniform locations (seed 0), sigma2 = 1, beta = 0.1, nu = 1.3, the whole
    n x n column-major matrix (one 1024 tile): every 7th entry against the oracle,
    plus symmetry, unit diagonal, 0 < C <= sigma2 and positive definiteness."""
    from paper_2502_00356_amd import workloads as w
    cfg = w.MATERN_SMALL
    xy = w.uniform_locations(cfg["n"], cfg["seed"], morton=False)
    A, packed = _dense(api, xy, cfg["sigma2"], cfg["beta"], cfg["nu"], cfg["tile"], cfg["lower_only"], "plain")
    # column-major layout of the single tile: packed[i + j n] = A[i, j]
    n = cfg["n"]
    P = packed.cpu().numpy()
    assert P[5 + 17 * n] == A[5, 17]
    idx = np.arange(0, n * n, 7)
    ii, jj = idx % n, idx // n
    ref = orc.matern_entries(xy, xy, ii, jj, cfg["sigma2"], cfg["beta"], cfg["nu"])
    assert rel_err(A[ii, jj], ref).max() <= TOL_PLAIN
    assert np.array_equal(A, A.T)
    assert np.all(np.diag(A) == 1.0)
    off = A[~np.eye(n, dtype=bool)]
    assert np.all(off > 0) and np.all(off < 1.0)
    np.linalg.cholesky(A)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_half_integer_matern(api, nu):
    """nu = 1/2, 3/2, 5/2: C = sigma2 e^-z, sigma2 (1+z) e^-z, sigma2 (1+z+z^2/3) e^-z."""
    from paper_2502_00356_amd import workloads as w
    xy = w.uniform_locations(200, seed=31)
    d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
    z = d / 0.05
    form = {0.5: lambda z: np.exp(-z), 1.5: lambda z: (1 + z) * np.exp(-z),
            2.5: lambda z: (1 + z + z * z / 3) * np.exp(-z)}[nu]
    for mode, tol in (("plain", TOL_PLAIN), ("mixed", TOL_MIXED)):
        A, _ = _dense(api, xy, 2.0, 0.05, nu, 64, 1, mode)
        ref = 2.0 * form(z)
        m = ref > 1e-300
        assert rel_err(A[m], ref[m]).max() <= tol


def test_fp32_output(api, orc):
    from paper_2502_00356_amd import workloads as w
    xy = w.uniform_locations(257, seed=41)
    A, packed = _dense(api, xy, 1.0, 0.02, 3.7, 128, 1, "mixed", out_dtype=1)
    assert str(packed.dtype) == "torch.float32"
    R = orc.matern_full(xy, 1.0, 0.02, 3.7)
    # FP32 storage adds at most half an FP32 ulp (2^-24) to the mixed-form error
    m = R > 1e-30
    assert rel_err(A[m], R[m]).max() <= TOL_MIXED + 2 ** -24


def test_coincident_points(api):
    """Exactly equal locations give sigma2 (Alg. 3, r == 0), off the diagonal too."""
    xy = np.array([[0.3, 0.4], [0.3, 0.4], [0.7, 0.1], [0.3, 0.4 + 1e-5]])
    A, _ = _dense(api, xy, 1.7, 0.1, 2.3, 3, 1, "plain")
    assert A[0, 1] == 1.7 and A[1, 0] == 1.7 and A[0, 0] == 1.7
    # r = 1e-5, z = 1e-4: C = sigma2 (1 - z^2 / (4 (nu - 1)) + ...) lies just below sigma2
    assert A[0, 3] < 1.7 and A[0, 3] > 1.7 * (1 - 1e-7)


def test_invalid_parameters(api):
    import torch
    a = torch.zeros(4, dtype=torch.float64, device="cuda")
    for bad in (dict(beta=0.0), dict(beta=-1.0), dict(nu=0.0), dict(sigma2=-1.0)):
        kw = dict(sigma2=1.0, beta=0.1, nu=1.0); kw.update(bad)
        with pytest.raises(api.BkError):
            api.matern_tiles(a, a, kw["sigma2"], kw["beta"], kw["nu"], 2, 1)
    with pytest.raises(api.BkError):
        api.matern_tiles(a, a, 1.0, 0.1, 1.0, 0, 1)


@pytest.mark.parametrize("mode", ["plain", "mixed"])
def test_counting_variant(api, orc, mode):
    """A call with statistics runs the counting variant of the Matern kernel: the
    same bits, one quadrature per stored entry at nonzero distance, N + 1 >= 5 nodes
    each (ragged last tile row and a duplicated point)."""
    import torch
    from paper_2502_00356_amd import workloads as w
    n, ts = 301, 128
    xy = w.uniform_locations(n, seed=71)
    xy[7] = xy[150]                        # an exact duplicate: r == 0 off the diagonal
    lx, ly = to_dev(xy[:, 0]), to_dev(xy[:, 1])
    ref = api.matern_tiles(lx, ly, 1.0, 0.07, 1.9, ts, 1, mode=mode)
    stats = torch.zeros(api.STATS_LEN, dtype=torch.int64, device="cuda")
    got = api.matern_tiles(lx, ly, 1.0, 0.07, 1.9, ts, 1, mode=mode, stats=stats)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    st = stats.cpu().numpy()
    # the duplicate pair (7, 150) is stored in tile (1, 0) only; (150, 7) and (7, 150)
    # both sit in stored tiles when they share a diagonal tile, which they do not here
    assert int(st[api.STAT_ENTRIES]) == api.matern_out_elems(n, ts, 1) - n - 1
    assert int(st[api.STAT_NODES]) >= 5 * int(st[api.STAT_ENTRIES])


def test_kernel_events_bracket_matern(api):
    import torch
    from paper_2502_00356_amd import workloads as w
    xy = w.uniform_locations(1500, seed=72)
    lx, ly = to_dev(xy[:, 0]), to_dev(xy[:, 1])
    ref = api.matern_tiles(lx, ly, 1.0, 0.05, 1.2, 500, 1, mode="mixed")
    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    for e in ev:
        e.record()
    torch.cuda.synchronize()
    got = api.matern_tiles(lx, ly, 1.0, 0.05, 1.2, 500, 1, mode="mixed", kernel_events=ev)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
    assert ev[0].elapsed_time(ev[1]) > 0.0
