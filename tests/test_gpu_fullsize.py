"""Parity at the full workload sizes, in the launch configuration bench.py times,
on outputs the oracle computes one by one (sampled entries and whole-tile
subsets), plus properties that hold at any size."""
import numpy as np
import pytest

from gpu_util import DBL_MIN, TOL_MIXED, TOL_PLAIN, k_result_err_ok, rel_err, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_00356_amd import api
    return api


@pytest.fixture(scope="module")
def model(api):
    """A model trained on the GPU on the training law (2^20 pairs, seed 4)."""
    from paper_2502_00356_amd import train_window_mlp
    m, _ = train_window_mlp.train(out=None, verbose=False)
    return m


def _packed_index(api, n, ts, lower, i, j):
    """Packed offsets of global entries (i, j) (lower_only requires i >= j by tiles)."""
    I, J = i // ts, j // ts
    off = np.array([api.matern_tile_offset(n, ts, lower, a, b) for a, b in zip(I, J)], dtype=np.int64)
    mI = np.minimum(ts, n - I * ts)
    return off + (i - I * ts) + (j - J * ts) * mI


def _sample_entries(n, ts, rng, count):
    """Random stored entries of the lower tile set, plus four whole-tile subsets: a
    diagonal tile, the tile below it, a middle tile and the farthest tile."""
    T = (n + ts - 1) // ts
    i = rng.integers(0, n, count)
    j = rng.integers(0, n, count)
    swap = (i // ts) < (j // ts)
    i[swap], j[swap] = j[swap], i[swap]
    parts_i, parts_j = [i], [j]
    for (I, J) in ((0, 0), (1, 0), (T // 2, T // 4), (T - 1, 0)):
        m = min(ts, n - I * ts)
        w = min(ts, n - J * ts)
        ii = rng.integers(0, m, 3000) + I * ts
        jj = rng.integers(0, w, 3000) + J * ts
        parts_i.append(ii)
        parts_j.append(jj)
    return np.concatenate(parts_i), np.concatenate(parts_j)


@pytest.mark.parametrize("nu", [0.8, 2.3])
def test_matern_medium_full_size(api, orc, model, nu):
    """n = 40,000 uniform locations (seed 3, Morton order), beta = 0.05, lower 960-tiles
    in FP64 (6.55 GB per form): plain within 1e-13, mixed and learned within 2e-6."""
    import torch
    from paper_2502_00356_amd import workloads as w
    cfg = w.MATERN_MEDIUM
    xy = w.uniform_locations(cfg["n"], cfg["seed"])
    n, ts = cfg["n"], cfg["tile"]
    lx, ly = to_dev(xy[:, 0]), to_dev(xy[:, 1])
    rng = np.random.default_rng(int(nu * 10))
    i, j = _sample_entries(n, ts, rng, 20000)
    ref = orc.matern_entries(xy, xy, i, j, cfg["sigma2"], cfg["beta"], nu)
    pidx = torch.from_numpy(_packed_index(api, n, ts, 1, i, j)).cuda()
    out = torch.empty(api.matern_out_elems(n, ts, 1), dtype=torch.float64, device="cuda")
    for mode, tol in (("plain", TOL_PLAIN), ("mixed", TOL_MIXED), ("learned", TOL_MIXED)):
        out.fill_(-1.0)
        api.matern_tiles(lx, ly, cfg["sigma2"], cfg["beta"], nu, ts, 1, mode=mode, out=out, model=model)
        torch.cuda.synchronize()
        got = out[pidx].cpu().numpy()
        m = ref > DBL_MIN
        assert rel_err(got[m], ref[m]).max() <= tol, mode
        # every stored entry was written and lies in [0, sigma2]
        assert float(out.min()) >= 0.0 and float(out.max()) <= cfg["sigma2"]


def test_matern_large_full_size(api, orc, model):
    """316 x 316 jittered grid (n = 99,856, seed 7), beta = 0.02, nu = 3.7, lower
    1,024-tiles: FP32 output (20.1 GB) for mixed and learned, FP64 (40.3 GB) for
    plain; sampled entries against the oracle."""
    import torch
    from paper_2502_00356_amd import workloads as w
    cfg = w.MATERN_LARGE
    xy = w.jittered_grid_locations(cfg["side"], cfg["seed"])
    n, ts, nu = xy.shape[0], cfg["tile"], cfg["nu"]
    assert n == 99856
    lx, ly = to_dev(xy[:, 0]), to_dev(xy[:, 1])
    rng = np.random.default_rng(17)
    i, j = _sample_entries(n, ts, rng, 20000)
    ref = orc.matern_entries(xy, xy, i, j, cfg["sigma2"], cfg["beta"], nu)
    pidx = torch.from_numpy(_packed_index(api, n, ts, 1, i, j)).cuda()
    elems = api.matern_out_elems(n, ts, 1)
    assert elems == 5036605696
    m = ref > 1e-30
    out32 = torch.empty(elems, dtype=torch.float32, device="cuda")
    for mode in ("mixed", "learned"):
        api.matern_tiles(lx, ly, cfg["sigma2"], cfg["beta"], nu, ts, 1, mode=mode, out_dtype=1, out=out32,
                         model=model)
        torch.cuda.synchronize()
        got = out32[pidx].double().cpu().numpy()
        assert rel_err(got[m], ref[m]).max() <= TOL_MIXED + 2 ** -24, mode
    del out32
    torch.cuda.empty_cache()
    out64 = torch.empty(elems, dtype=torch.float64, device="cuda")
    api.matern_tiles(lx, ly, cfg["sigma2"], cfg["beta"], nu, ts, 1, mode="plain", out=out64)
    torch.cuda.synchronize()
    got = out64[pidx].cpu().numpy()
    mm = ref > DBL_MIN
    assert rel_err(got[mm], ref[mm]).max() <= TOL_PLAIN
    del out64
    torch.cuda.empty_cache()


def test_grid_full_size_per_region(api, orc, model):
    """The 2^24-pair standalone grid (seed 2) in all three forms, launched whole;
    a 2^16 sample plus every half-integer entry of the sample against the oracle,
    per region of x (decades) and of the peak regime (nu^2 <= x or not)."""
    import torch
    from paper_2502_00356_amd import workloads as w
    nu, x, hidx = w.grid_pairs(1 << 24, seed=2)
    dnu, dx = to_dev(nu), to_dev(x)
    rng = np.random.default_rng(23)
    s = np.unique(np.concatenate([rng.choice(nu.size, 1 << 16, replace=False), hidx[:4096]]))
    kref, _, ks = orc.besselk(nu[s], x[s])
    sel = torch.from_numpy(s).cuda()
    assert (x[s] > 708).sum() > 500 and (kref == 0).sum() > 100     # the sample reaches the underflow zone
    for mode, tol in (("plain", TOL_PLAIN), ("mixed", TOL_MIXED), ("learned", TOL_MIXED)):
        # K itself (the output the benchmark times), element by element, including
        # the subnormal zone
        outk = api.besselk(dnu, dx, mode=mode, model=model, result=api.RESULT_K)
        torch.cuda.synchronize()
        okk = k_result_err_ok(outk[sel].cpu().numpy(), kref, tol)
        assert okk.all(), (mode, int((~okk).sum()))
        del outk
        out = api.besselk(dnu, dx, mode=mode, model=model, result=api.RESULT_SCALED)
        torch.cuda.synchronize()
        got = out[sel].cpu().numpy()
        e = rel_err(got, ks)
        lxs = np.log10(x[s])
        inner = nu[s] ** 2 > x[s]
        rep = []
        for lo in range(-4, 3):
            for reg, msk in (("t*>0", inner), ("t*=0", ~inner)):
                sel_r = (lxs >= lo) & (lxs < lo + 1) & msk
                if sel_r.any():
                    rep.append("1e%d %s %.2g" % (lo, reg, e[sel_r].max()))
        print(mode, "max %.3g |" % e.max(), " | ".join(rep))
        assert e.max() <= tol, mode


def test_learned_eval_set_and_probe(api, orc, model):
    """Fresh 2^24-pair evaluation set (seed 5): sampled parity and the fallback count;
    the 2^16-pair out-of-range probe (seed 6): every entry falls back to the solver."""
    import torch
    from paper_2502_00356_amd import workloads as w
    nu, x = w.eval_pairs(1 << 24, seed=5)
    stats = torch.zeros(api.STATS_LEN, dtype=torch.int64, device="cuda")
    out = api.besselk(to_dev(nu), to_dev(x), mode="learned", model=model, result=api.RESULT_SCALED, stats=stats)
    torch.cuda.synchronize()
    st = stats.cpu().numpy()
    fb = int(st[api.STAT_FB_RANGE] + st[api.STAT_FB_TAIL] + st[api.STAT_FB_NONFINITE])
    print("eval set: fallbacks %d of %d (range %d, tail %d, nonfinite %d), N raised %d" % (
        fb, nu.size, st[api.STAT_FB_RANGE], st[api.STAT_FB_TAIL], st[api.STAT_FB_NONFINITE],
        st[api.STAT_NODE_RAISED]))
    s = np.random.default_rng(29).choice(nu.size, 1 << 16, replace=False)
    kref, _, ks = orc.besselk(nu[s], x[s])
    assert rel_err(out.cpu().numpy()[s], ks).max() <= TOL_MIXED
    assert fb < 1e-3 * nu.size
    outk = api.besselk(to_dev(nu), to_dev(x), mode="learned", model=model, result=api.RESULT_K)
    torch.cuda.synchronize()
    assert k_result_err_ok(outk.cpu().numpy()[s], kref, TOL_MIXED).all()
    del outk
    pn, px = w.out_of_range_pairs(1 << 16, seed=6)
    stats.zero_()
    out = api.besselk(to_dev(pn), to_dev(px), mode="learned", model=model, result=api.RESULT_SCALED, stats=stats)
    torch.cuda.synchronize()
    assert int(stats.cpu().numpy()[api.STAT_FB_RANGE]) == pn.size
    s = np.random.default_rng(31).choice(pn.size, 4096, replace=False)
    _, _, ks = orc.besselk(pn[s], px[s])
    assert rel_err(out.cpu().numpy()[s], ks).max() <= TOL_MIXED
