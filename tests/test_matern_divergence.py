"""How far apart the node counts of one wave's entries lie in the tiled Matern
kernels (a wave covers 64 consecutive rows of one tile column), from the oracle's
window and node-count rule on sampled waves of the medium (n = 40,000 uniform,
Morton order) and large (316 x 316 jittered grid) workloads. A wave runs as long
as its largest node count; the ratio mean N / max N over a wave bounds what sorting
a block's entries by N (as the standalone kernel does) could recover. It stays
above 0.95 for every workload and form, which is why the Matern kernels keep the
tile order. CPU only."""
import numpy as np
import pytest


def _wave_efficiency(orc, xy, beta, nu, ts, L, Lq, nwaves=1500, seed=0):
    n = xy.shape[0]
    rng = np.random.default_rng(seed)
    T = (n + ts - 1) // ts
    rows_all, cols_all = [], []
    for _ in range(nwaves):
        I = rng.integers(0, T)
        J = rng.integers(0, I + 1)
        mI = min(ts, n - I * ts)
        rb = rng.integers(0, (mI + 63) // 64)
        rows = I * ts + rb * 64 + np.arange(64)
        rows = rows[rows < min(n, (I + 1) * ts)]
        col = J * ts + rng.integers(0, min(ts, n - J * ts))
        rows_all.append(rows)
        cols_all.append(np.full(rows.size, col))
    r, c = np.concatenate(rows_all), np.concatenate(cols_all)
    z = np.hypot(xy[r, 0] - xy[c, 0], xy[r, 1] - xy[c, 1]) / beta
    z = np.where(z == 0.0, 1e-300, z)
    _, _, t0, t1 = orc.window(np.full(z.size, nu), z, L)
    N = orc.node_count(np.full(z.size, nu), z, t0, t1, Lq)
    effs, o = [], 0
    for rows in rows_all:
        Nw = N[o:o + rows.size]
        o += rows.size
        effs.append(Nw.mean() / Nw.max())
    return float(np.mean(effs)), float(N.mean())


@pytest.mark.parametrize("workload,nu", [("medium", 0.8), ("medium", 2.3), ("large", 3.7)])
@pytest.mark.parametrize("form,L,Lq", [("plain", 36.0, 35.0), ("mixed", 15.0, 14.5)])
def test_wave_node_counts_are_uniform(orc, workload, nu, form, L, Lq):
    from paper_2502_00356_amd import workloads as w
    if workload == "medium":
        c = w.MATERN_MEDIUM
        xy, beta, ts = w.uniform_locations(c["n"], c["seed"]), c["beta"], c["tile"]
    else:
        c = w.MATERN_LARGE
        xy, beta, ts = w.jittered_grid_locations(c["side"], c["seed"]), c["beta"], c["tile"]
    eff, mean_n = _wave_efficiency(orc, xy, beta, nu, ts, L, Lq)
    print("%s nu=%g %s: mean N %.2f, wave efficiency mean N / max N %.4f" % (workload, nu, form, mean_n, eff))
    assert eff > 0.95
