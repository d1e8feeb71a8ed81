"""Benchmark: Matern covariance entries per second (K_nu evaluations fused into
tiled Matern generation), learned window with FP32 terms against plain FP64.

Default workload (one step): the 316 x 316 jittered grid in [0, 1]^2 (jitter
U[-0.4, 0.4] cell, seed 7, Morton order; n = 99,856), sigma^2 = 1, beta = 0.02,
nu = 3.7, lower-triangle 1,024-tiles, 5,036,605,696 entries, locations resident
in HBM. A step is one bk_matern_tiles call in the learned form with FP32 output
(window table, interval plans, main kernel, fallback). The mixed form (FP32
output) and the plain FP64 form (FP64 output) are timed on the same inputs and
reported beside it.

Other workloads (--workload): grid (2^24 standalone (nu, x) pairs), matern-medium,
deriv-grid, matern-grad-medium, loglik, paper-grid.

Prints one JSON line. Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs at 2.4 GHz; a CU issues one full-rate wave64 VALU instruction
# per clock (64 lane-ops) across its four SIMDs. Measured on gfx950: FP64 add, mul
# and fma, conversions and FP32 max/ldexp run at that rate; FP32 add, mul and fma,
# integer adds and moves at twice it (half an issue clock each); FP32
# transcendentals at half of it (two clocks); FP64 reciprocal at a quarter (four).
# The peak is the full-rate lane-op rate.
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# VALU issue clocks of one trapezoid node: the loop body of each form's node walk
# in the gfx950 code of libbesselk.so, weighted by those rates, counted by the
# build (paper_2502_00356_amd/build.py writes node_slots.json).
def load_node_slots():
    path = os.path.join(ROOT, "paper_2502_00356_amd", "node_slots.json")
    if not os.path.exists(path):
        sys.exit("bench.py: %s is missing; build the library first (python -c 'import __graft_entry__ as g; "
                 "g.build()'), which writes it from the gfx950 assembly" % path)
    with open(path) as f:
        return {k: float(v) for k, v in json.load(f).items()}


NODE_SLOTS = load_node_slots()

# Counter figures per launch of a dominant kernel (profiles/), valid only for the
# kernel code they were taken on (hash of the sources with comments removed), else
# null: HBM bytes from the FETCH_SIZE and WRITE_SIZE runs scaled by a plain 1 GiB
# copy, and SQ_INSTS_VALU of one launch without statistics.
TRAFFIC = {
    "grid": {"src_sha": "53987bbd1f5b7a90", "n": 1 << 24, "bytes": 4.22539e8, "valu_insts": 1.17947e8},
    "matern_large": {"src_sha": "53987bbd1f5b7a90", "bytes": 2.02873e10, "valu_insts": 9.58373e9},
}
KERNEL_SOURCES = ("bk_mlp.hip", "bk_math.hpp", "bk_internal.hpp")


def kernel_src_sha():
    """Hash of the learned kernel's sources with comments and blank space removed,
    so that edits to comments alone do not invalidate the traffic figure."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2502_00356_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--form", default="auto", choices=["auto", "plain", "mixed", "learned"])
    ap.add_argument("--model", default=os.path.join(ROOT, "paper_2502_00356_amd", "models", "window_mlp.bin"))
    ap.add_argument("--cpu-sample", type=int, default=1 << 20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="matern-large",
                    choices=["matern-large", "grid", "matern-medium", "deriv-grid", "matern-grad-medium", "loglik",
                             "paper-grid", "small-x", "matern-order", "valu-rates", "table-source"],
                    help="matern-large: the headline (316 x 316 grid, nu = 3.7, FP32 learned vs FP64 plain)")
    ap.add_argument("--forms", default="learned,mixed,plain",
                    help="matern-large: forms to time (comma-separated; the headline needs learned)")
    ap.add_argument("--cpu-tiles", type=int, default=4,
                    help="matern-large: whole tiles of the last tile row in the CPU baseline sample (0-4)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="time a plain 1 GiB device-to-device copy instead (HBM reference for counters)")
    return ap.parse_args()


def copy_probe(torch):
    """A plain copy kernel of known size: 2^27 doubles (1 GiB) read and 1 GiB written."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / 5
    print(json.dumps({"copy_bytes_read": 1 << 30, "copy_bytes_written": 1 << 30, "ms": ms,
                      "gbps_read_plus_write": 2 * (1 << 30) / (ms * 1e-3) / 1e9}), flush=True)


def time_form(api, torch, nu, x, out, form, steps, warmup, model, ws):
    """Per step: HIP-event time of the whole call, host wall time, and the time of
    the form's main kernel alone (a pair of events the library records around it on
    the same stream)."""
    kw = dict(mode=form, model=model, workspace=ws)
    for _ in range(warmup):
        api.besselk(nu, x, out=out, **kw)
    stream = torch.cuda.current_stream()
    kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in kev:            # create the events; the library records them again
        a.record(stream)
        b.record(stream)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for k in range(steps):
        api.besselk(nu, x, out=out, kernel_events=kev[k], **kw)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = sum(a.elapsed_time(b) for a, b in kev) / steps
    return ev0.elapsed_time(ev1) / steps, wall / steps * 1e3, kernel_ms


def per_region(nu, x, e, half_idx, idx):
    """Max relative error (of e^x K) on the sample by region: decades of x, the
    peak regime (nu^2 <= x: peak at t = 0), order bands, the half-integer subset,
    the paper's region x in [0.1, 140], x < 0.1 and the underflow zone x > 708."""
    out = {}
    dec = np.floor(np.log10(x)).astype(int)
    for d in range(-4, 3):
        m = dec == d
        if m.any():
            out["x 1e%d..1e%d" % (d, d + 1)] = float(e[m].max())
    flat = nu * nu <= x
    out["peak at 0 (nu^2<=x)"] = float(e[flat].max()) if flat.any() else None
    out["interior peak"] = float(e[~flat].max()) if (~flat).any() else None
    for lo, hi in ((0.01, 1.0), (1.0, 4.0), (4.0, 10.0 + 1e-9)):
        m = (nu >= lo) & (nu < hi)
        if m.any():
            out["nu %g..%g" % (lo, round(hi))] = float(e[m].max())
    h = np.isin(idx, half_idx)
    if h.any():
        out["half-integer nu"] = float(e[h].max())
    for name, m in (("paper region x 0.1..140", (x >= 0.1) & (x <= 140)), ("x < 0.1", x < 0.1), ("x > 708", x > 708)):
        if m.any():
            out[name] = float(e[m].max())
    return out


def node_total(api, torch, nu, x, out, form, model, ws):
    stats = torch.zeros(api.STATS_LEN, dtype=torch.int64, device=x.device)
    api.besselk(nu, x, out=out, mode=form, model=model, workspace=ws, stats=stats)
    torch.cuda.synchronize()
    return stats.cpu().numpy()


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the K_nu and Matern paths need no "
              "cross-GPU exchange, and no multi-GPU run is provided "
              "(requested --gpus %d)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if a.copy_probe:
        copy_probe(torch)
        return
    from paper_2502_00356_amd import api, workloads
    if a.workload in ("deriv-grid", "matern-grad-medium"):
        deriv_bench(a, torch, api, workloads)
        return
    if a.workload == "loglik":
        loglik_bench(a, torch, api, workloads)
        return
    if a.workload == "paper-grid":
        paper_bench(a, torch, api, workloads)
        return
    if a.workload == "matern-large":
        matern_headline(a, torch, api, workloads)
        return
    if a.workload == "small-x":
        small_x_bench(a, torch, api, workloads)
        return
    if a.workload == "matern-order":
        matern_order_bench(a, torch, api, workloads)
        return
    if a.workload == "valu-rates":
        valu_rates_bench(torch)
        return
    if a.workload == "table-source":
        table_source_bench(a, torch, api, workloads)
        return
    if a.workload != "grid":
        matern_bench(a, torch, api, workloads)
        return
    grid_bench(a, torch, api, workloads)


def traffic_entry(key, n=None):
    """The counter figures of TRAFFIC[key] if they were taken on the current kernel
    sources (and size), else None."""
    t = TRAFFIC.get(key)
    if t is None or kernel_src_sha() != t["src_sha"] or (n is not None and t.get("n") != n):
        return None
    return t


def load_model(a, api):
    if os.path.exists(a.model):
        return api.Model(a.model)
    # no stored model: train one on the GPU (2^20 pairs, about a second), outside the timed region
    from paper_2502_00356_amd import train_window_mlp
    model, _ = train_window_mlp.train(out=None, verbose=False)
    return model


def cpu_sample_entries(n, ts, count, tiles, seed):
    """The CPU baseline sample of the tiled Matern workload: count stored entries
    drawn uniformly, then whole tiles of the last tile row (the diagonal tile, the one
    left of it, a middle one and the farthest one), as (row, column) index arrays."""
    rng = np.random.default_rng(seed)
    T = (n + ts - 1) // ts
    i = rng.integers(0, n, count)
    j = rng.integers(0, n, count)
    swap = (i // ts) < (j // ts)
    i[swap], j[swap] = j[swap], i[swap]
    parts_i, parts_j = [i], [j]
    I = T - 1
    for J in (T - 1, T - 2, T // 2, 0)[:tiles]:
        m, w = n - I * ts, min(ts, n - J * ts)
        ii, jj = np.meshgrid(np.arange(m) + I * ts, np.arange(w) + J * ts, indexing="ij")
        parts_i.append(ii.ravel())
        parts_j.append(jj.ravel())
    return np.concatenate(parts_i), np.concatenate(parts_j)


def packed_index(api, n, ts, i, j):
    """Offsets in the packed lower-tile output of entries (i, j), i's tile >= j's."""
    I, J = i // ts, j // ts
    T = (n + ts - 1) // ts
    offs = np.array([[api.matern_tile_offset(n, ts, 1, r, c) if c <= r else -1 for c in range(T)] for r in range(T)],
                    dtype=np.int64)
    mI = np.minimum(ts, n - I * ts)
    return offs[I, J] + (i - I * ts) + (j - J * ts) * mI


def matern_headline(a, torch, api, workloads):
    """The headline line: the 316 x 316 grid Matern build (see the module docstring)."""
    dev = torch.device("cuda:0")
    c = workloads.MATERN_LARGE
    xy = workloads.jittered_grid_locations(c["side"], c["seed"])
    n, ts, nu, beta, s2 = xy.shape[0], c["tile"], c["nu"], c["beta"], c["sigma2"]
    lx = torch.from_numpy(np.ascontiguousarray(xy[:, 0])).to(dev)
    ly = torch.from_numpy(np.ascontiguousarray(xy[:, 1])).to(dev)
    elems = api.matern_out_elems(n, ts, 1)
    model = load_model(a, api)
    ws = torch.empty(api.matern_workspace_bytes(n, ts, 1), dtype=torch.uint8, device=dev)
    want = set(a.forms.split(","))
    outs = {torch.float32: torch.empty(elems, dtype=torch.float32, device=dev)}
    if "plain" in want:
        outs[torch.float64] = torch.empty(elems, dtype=torch.float64, device=dev)
    forms = tuple(f for f in (("learned", api.OUT_F32, "matern_learned"), ("mixed", api.OUT_F32, "matern_mixed"),
                              ("plain", api.OUT_F64, "matern_plain")) if f[0] in want or f[0] == "learned")
    stream = torch.cuda.current_stream()
    res = {}
    for f, odt, slot_key in forms:
        out = outs[torch.float32 if odt == api.OUT_F32 else torch.float64]
        kw = dict(mode=f, out_dtype=odt, out=out, model=model, workspace=ws)
        steps = a.steps if f == "learned" else max(1, min(a.steps, 5))
        for _ in range(a.warmup):
            api.matern_tiles(lx, ly, s2, beta, nu, ts, 1, **kw)
        kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for e0, e1 in kev:                  # create the events; the library records them again
            e0.record(stream)
            e1.record(stream)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for k in range(steps):
            api.matern_tiles(lx, ly, s2, beta, nu, ts, 1, kernel_events=kev[k], **kw)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps * 1e3
        ms = ev0.elapsed_time(ev1) / steps
        kms = sum(e0.elapsed_time(e1) for e0, e1 in kev) / steps
        # the counting variant, once, outside the timed region
        st = torch.zeros(api.STATS_LEN, dtype=torch.int64, device=dev)
        api.matern_tiles(lx, ly, s2, beta, nu, ts, 1, stats=st, **kw)
        torch.cuda.synchronize()
        st = st.cpu().numpy()
        nodes_main = int(st[api.STAT_NODES] - st[api.STAT_FB_NODES])
        quad_main = int(st[api.STAT_ENTRIES])
        fb = int(st[api.STAT_FB_RANGE] + st[api.STAT_FB_TAIL] + st[api.STAT_FB_NONFINITE]) if f == "learned" else 0
        if f == "learned":
            quad_main -= fb - int(st[api.STAT_FB_RANGE])     # fallback recomputations are counted in ENTRIES too
        res[f] = dict(ms_per_step=ms, wall_ms_per_step=wall, kernel_ms=kms, steps=steps,
                      entries_per_s=elems / (ms * 1e-3),
                      write_gbps=elems * out.element_size() / (ms * 1e-3) / 1e9,
                      out_dtype="f32" if odt == api.OUT_F32 else "f64",
                      mean_nodes=nodes_main / max(1, quad_main), node_total_main=nodes_main,
                      lane_efficiency=nodes_main / max(1, int(st[api.STAT_LANE_SLOTS])),
                      fallbacks=fb, fallback_nodes=int(st[api.STAT_FB_NODES]),
                      node_slots=NODE_SLOTS.get(slot_key),
                      node_work_frac=(NODE_SLOTS[slot_key] * nodes_main / (kms * 1e-3) / 1e12 / VALU_PEAK_TOPS
                                      if slot_key in NODE_SLOTS else None))
    head = res["learned"]

    # accuracy of each form's timed output on the CPU sample, and the oracle's own
    # throughput on it (the CPU baseline)
    cpu, acc = None, {}
    if not a.no_cpu:
        import oracle
        i, j = cpu_sample_entries(n, ts, a.cpu_sample, max(0, min(4, a.cpu_tiles)), seed=99)
        t0 = time.perf_counter()
        ref = oracle.matern_entries(xy, xy, i, j, s2, beta, nu)
        dt = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = dict(value=i.size / dt, unit="entries/s", cores=cores, kind="oracle",
                   sample="%d stored entries drawn uniformly plus the %d whole tiles of the last tile row (diagonal, "
                          "its left neighbour, middle, farthest): %d entries; long-double adaptive Gauss-Kronrod, "
                          "OpenMP over entries, %.1f s" % (a.cpu_sample, max(0, min(4, a.cpu_tiles)), i.size, dt))
        pidx = torch.from_numpy(packed_index(api, n, ts, i, j)).to(dev)
        m = ref > 1e-30
        for f, odt, _ in forms:
            out = outs[torch.float32 if odt == api.OUT_F32 else torch.float64]
            api.matern_tiles(lx, ly, s2, beta, nu, ts, 1, mode=f, out_dtype=odt, out=out, model=model, workspace=ws)
            got = out[pidx].double().cpu().numpy()
            acc[f] = float((np.abs(got[m] - ref[m]) / ref[m]).max())
    kms = head["kernel_ms"]
    achieved = NODE_SLOTS["matern_learned"] * head["node_total_main"] / (kms * 1e-3) / 1e12
    tr = traffic_entry("matern_large")
    line = {
        "metric": "K_nu evals/s (Matern entries/s) mixed+learned vs FP64 at <=2e-6 rel err",
        "value": head["entries_per_s"],
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 solve and distance + f32 node terms, f32 out",
        "data": "synthetic",
        "config": {"workload": "Matern build on a 316x316 jittered grid in [0,1]^2 (jitter U[-0.4,0.4] cell, seed 7, "
                               "Morton order), n=99856, sigma2=1, beta=0.02, nu=3.7, lower-triangle 1024-tiles, "
                               "5036605696 entries, FP32 output; plain FP64 (FP64 output) on the same inputs",
                   "n": n, "tile": ts, "entries": elems, "form": "learned",
                   "also": "bench.py --workload grid: the 2^24-pair standalone K_nu grid"},
        "forms": {f: {k: (round(v, 6) if isinstance(v, float) else v) for k, v in d.items()} for f, d in res.items()},
        "speedup_vs_plain_f64": res["plain"]["ms_per_step"] / head["ms_per_step"] if "plain" in res else None,
        "speedup_vs_mixed": res["mixed"]["ms_per_step"] / head["ms_per_step"] if "mixed" in res else None,
        "max_rel_err_sample": acc,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                     "unit": "TOP/s (full-rate VALU lane-op slots)", "frac": achieved / VALU_PEAK_TOPS,
                     "traffic": tr["bytes"] if tr else None,
                     "kernel": "k_matern_learned<float>", "kernel_ms": kms,
                     "work": "%.2f VALU issue clocks (full-rate lane-op slots) per trapezoid node x %d nodes per step"
                             % (NODE_SLOTS["matern_learned"], head["node_total_main"]),
                     "hbm_gbps": 4.0 * elems / (kms * 1e-3) / 1e9,
                     "hbm_frac": 4.0 * elems / (kms * 1e-3) / 8e12,
                     "valu_issue_per_cu_clock": (tr["valu_insts"] / (kms * 1e-3 * 256 * 2.4e9) if tr else None)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def grid_bench(a, torch, api, workloads):
    """The 2^24-pair standalone K_nu grid: learned (or mixed) beside plain FP64."""
    dev = torch.device("cuda:0")
    nu_h, x_h, half_idx = workloads.grid_pairs(a.n, seed=2)
    nu = torch.from_numpy(nu_h).to(dev)
    x = torch.from_numpy(x_h).to(dev)
    out = torch.empty_like(x)

    model = load_model(a, api) if (os.path.exists(a.model) or a.form in ("auto", "learned")) else None
    form = a.form
    if form == "auto":
        form = "learned" if model is not None else "mixed"
    ws = torch.empty(api.workspace_bytes(a.n), dtype=torch.uint8, device=dev) if form == "learned" else None

    forms = {}
    for f in ([form] + (["plain"] if form != "plain" else [])):
        ms_ev, ms_wall, ms_kernel = time_form(api, torch, nu, x, out, f, a.steps, a.warmup, model, ws)
        st = node_total(api, torch, nu, x, out, f, model, ws)
        forms[f] = dict(ms_per_step=ms_ev, wall_ms_per_step=ms_wall, kernel_ms=ms_kernel,
                        evals_per_s=a.n / (ms_ev * 1e-3),
                        mean_nodes=float(st[api.STAT_NODES]) / max(1, int(st[api.STAT_ENTRIES])),
                        node_total=int(st[api.STAT_NODES]),
                        fallbacks=int(st[api.STAT_FB_RANGE] + st[api.STAT_FB_TAIL] + st[api.STAT_FB_NONFINITE]),
                        nodes_raised=int(st[api.STAT_NODE_RAISED]),
                        # share of the node walk's lane slots (64 x a wave's largest N + 1) doing work
                        lane_efficiency=float(st[api.STAT_NODES] - st[api.STAT_FB_NODES])
                        / max(1, int(st[api.STAT_LANE_SLOTS])))
    head = forms[form]

    # accuracy of the timed forms on a bounded sample against the oracle, and the
    # oracle's own throughput on that sample (CPU baseline)
    cpu = None
    acc = {}
    region = {}
    if not a.no_cpu:
        import oracle
        m = min(a.cpu_sample, a.n)
        idx = np.random.default_rng(99).permutation(a.n)[:m]
        t0 = time.perf_counter()
        k_ref, _, ks_ref = oracle.besselk(nu_h[idx], x_h[idx])
        dt = time.perf_counter() - t0
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = dict(value=m / dt, unit="evals/s", cores=cores, kind="oracle",
                   sample="%d pairs drawn uniformly from the 2^24 grid (seed 99); long-double "
                          "adaptive Gauss-Kronrod, OpenMP over entries, %.1f s" % (m, dt))
        sel = torch.from_numpy(idx).to(dev)
        for f in forms:
            o = api.besselk(nu[sel].contiguous(), x[sel].contiguous(), mode=f, model=model,
                            result=api.RESULT_SCALED,
                            workspace=(torch.empty(api.workspace_bytes(m), dtype=torch.uint8, device=dev)
                                       if f == "learned" else None))
            torch.cuda.synchronize()
            e = np.abs(o.cpu().numpy() - ks_ref) / ks_ref
            acc[f] = float(e.max())
            region[f] = per_region(nu_h[idx], x_h[idx], e, half_idx, idx)
            # the timed output itself (K) at the sampled entries: relative error where K
            # is normal; where it underflows, the worst excess over one subnormal unit
            if f == form:
                api.besselk(nu, x, out=out, mode=f, model=model, workspace=ws)     # the timed call
                torch.cuda.synchronize()
                full = out[sel].cpu().numpy()
                nrm = k_ref >= np.finfo(np.float64).tiny
                acc[f + " K (timed output), normal range"] = float((np.abs(full[nrm] - k_ref[nrm]) / k_ref[nrm]).max())
                sub = ~nrm
                acc[f + " K, underflow zone: max |dK| / (2e-6 K + 2^-1074)"] = float(
                    (np.abs(full[sub] - k_ref[sub]) / (2e-6 * k_ref[sub] + 2.0 ** -1074)).max()) if sub.any() else None

    achieved = NODE_SLOTS[form] * head["node_total"] / (head["kernel_ms"] * 1e-3) / 1e12
    tr = traffic_entry("grid", a.n) if form == "learned" else None
    line = {
        "metric": "K_nu evals/s (Matern entries/s) mixed+learned vs FP64 at <=2e-6 rel err",
        "value": head["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 solve + f32 node terms" if form != "plain" else "f64",
        "data": "synthetic",
        "config": {"workload": "standalone K_nu grid: 2^24 pairs, nu~U[0.01,10], x log-uniform "
                               "[1e-4,1e3], 1% half-integer nu (seed 2), FP64 in/out",
                   "n": a.n, "form": form},
        "forms": {f: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()} for f, d in forms.items()},
        "speedup_vs_plain_f64": forms["plain"]["ms_per_step"] / head["ms_per_step"] if "plain" in forms else 1.0,
        "max_rel_err_sample": acc,
        "max_rel_err_by_region": region,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s (full-rate VALU lane-op slots)",
                     "frac": achieved / VALU_PEAK_TOPS,
                     "traffic": (tr["bytes"] if tr else None),
                     "kernel": "k_besselk_learned" if form == "learned" else "k_besselk<%s>" % form,
                     "kernel_ms": head["kernel_ms"],
                     "work": "%.2f VALU issue clocks (full-rate lane-op slots) per trapezoid node x %d nodes per step"
                             % (NODE_SLOTS[form], head["node_total"]),
                     "hbm_gbps": 24.0 * a.n / (head["kernel_ms"] * 1e-3) / 1e9,
                     # all VALU instructions of the launch (counter run) per CU-clock of
                     # the kernel's time; one wave64 instruction per CU-clock is the
                     # full-rate issue limit
                     "valu_issue_per_cu_clock": (tr["valu_insts"] / (head["kernel_ms"] * 1e-3 * 256 * 2.4e9)
                                                 if tr else None)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def matern_bench(a, torch, api, workloads):
    """Tiled Matern generation: entries/s and HBM write GB/s per form (one JSON line).
    matern-medium: n = 40,000 uniform (seed 3, Morton), beta = 0.05, nu in {0.8, 2.3},
    lower 960-tiles, FP64 output. matern-large: 316 x 316 jittered grid (seed 7),
    beta = 0.02, nu = 3.7, lower 1,024-tiles, FP32 output for mixed/learned and FP64
    for plain."""
    dev = torch.device("cuda:0")
    model = api.Model(a.model) if os.path.exists(a.model) else None
    if a.workload == "matern-medium":
        c = workloads.MATERN_MEDIUM
        xy = workloads.uniform_locations(c["n"], c["seed"])
        cases = [(nu, f, api.OUT_F64) for nu in c["nus"] for f in ("plain", "mixed", "learned")]
        beta, ts = c["beta"], c["tile"]
    else:
        c = workloads.MATERN_LARGE
        xy = workloads.jittered_grid_locations(c["side"], c["seed"])
        cases = [(c["nu"], "plain", api.OUT_F64), (c["nu"], "mixed", api.OUT_F32), (c["nu"], "learned", api.OUT_F32)]
        beta, ts = c["beta"], c["tile"]
    n = xy.shape[0]
    lx = torch.from_numpy(np.ascontiguousarray(xy[:, 0])).to(dev)
    ly = torch.from_numpy(np.ascontiguousarray(xy[:, 1])).to(dev)
    elems = api.matern_out_elems(n, ts, 1)
    res = {}
    bufs = {}
    for nu, f, dt in cases:
        if f == "learned" and model is None:
            continue
        tdt = torch.float32 if dt == api.OUT_F32 else torch.float64
        if tdt not in bufs:
            bufs[tdt] = torch.empty(elems, dtype=tdt, device=dev)
        out = bufs[tdt]
        ws = (torch.empty(api.matern_workspace_bytes(n, ts, 1), dtype=torch.uint8, device=dev)
              if f == "learned" else None)
        kw = dict(mode=f, out_dtype=dt, out=out, model=model, workspace=ws)
        for _ in range(max(1, a.warmup)):
            api.matern_tiles(lx, ly, 1.0, beta, nu, ts, 1, **kw)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        steps = max(1, min(a.steps, 5))
        ev0.record()
        for _ in range(steps):
            api.matern_tiles(lx, ly, 1.0, beta, nu, ts, 1, **kw)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        st = torch.zeros(api.STATS_LEN, dtype=torch.int64, device=dev)      # counting pass, untimed
        api.matern_tiles(lx, ly, 1.0, beta, nu, ts, 1, stats=st, **kw)
        torch.cuda.synchronize()
        st = st.cpu().numpy()
        fb = int(st[api.STAT_FB_RANGE] + st[api.STAT_FB_TAIL] + st[api.STAT_FB_NONFINITE])
        main_nodes = int(st[api.STAT_NODES] - st[api.STAT_FB_NODES])
        main_ents = int(st[api.STAT_ENTRIES]) - (fb - int(st[api.STAT_FB_RANGE]))
        res["nu=%g/%s" % (nu, f)] = {"ms": round(ms, 3), "entries_per_s": elems / (ms * 1e-3),
                                     "write_gbps": elems * out.element_size() / (ms * 1e-3) / 1e9,
                                     "out_dtype": str(tdt).replace("torch.", ""),
                                     "mean_nodes": main_nodes / max(1, main_ents), "fallbacks": fb,
                                     "lane_efficiency": main_nodes / max(1, int(st[api.STAT_LANE_SLOTS]))}
    line = {"metric": "Matern entries/s", "workload": a.workload, "n": n, "tile": ts, "entries": elems,
            "beta": beta, "results": res}
    print(json.dumps(line), flush=True)


def table_source_bench(a, torch, api, workloads):
    """What the network adds over the same tables filled by the plain window solver
    (bk_model_set_table_source): the learned kernels on the 2^24-pair evaluation set
    (seed 5) and on the 316 x 316 Matern build (nu = 3.7, beta = 0.02, lower
    1,024-tiles, FP32), with the cells / window table from the network (its
    calibrated margins), from the solver with the same margins, and from the solver
    with none. Per source: main-kernel time (HIP events around it), mean nodes per
    entry walked, fallbacks."""
    dev = torch.device("cuda:0")
    nu_h, x_h = workloads.eval_pairs(a.n, seed=5)
    nu = torch.from_numpy(nu_h).to(dev)
    x = torch.from_numpy(x_h).to(dev)
    out = torch.empty_like(x)
    ws = torch.empty(api.workspace_bytes(a.n), dtype=torch.uint8, device=dev)
    c = workloads.MATERN_LARGE
    xy = workloads.jittered_grid_locations(c["side"], c["seed"])
    n, ts = xy.shape[0], c["tile"]
    lx = torch.from_numpy(np.ascontiguousarray(xy[:, 0])).to(dev)
    ly = torch.from_numpy(np.ascontiguousarray(xy[:, 1])).to(dev)
    elems = api.matern_out_elems(n, ts, 1)
    mout = torch.empty(elems, dtype=torch.float32, device=dev)
    mws = torch.empty(api.matern_workspace_bytes(n, ts, 1), dtype=torch.uint8, device=dev)
    res = {}
    for name, src, zero in (("network", api.TABLE_NETWORK, False), ("solver+margins", api.TABLE_SOLVER, False),
                            ("solver", api.TABLE_SOLVER, True)):
        m = api.Model(a.model)
        if zero:
            m.set_margins(0.0, 0.0, 0.0, 0.0)
        m.set_table_source(src)
        row = {}
        for wl, call in (("grid_2^24", lambda ev=None, st=None: api.besselk(nu, x, out=out, mode="learned", model=m,
                                                                           workspace=ws, kernel_events=ev, stats=st)),
                         ("matern_316^2", lambda ev=None, st=None: api.matern_tiles(
                             lx, ly, c["sigma2"], c["beta"], c["nu"], ts, 1, mode="learned", out_dtype=api.OUT_F32,
                             out=mout, model=m, workspace=mws, kernel_events=ev, stats=st))):
            for _ in range(max(1, a.warmup)):
                call()
            reps = max(3, min(a.steps, 10))
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
            for e0, e1 in ev:
                e0.record()
                e1.record()
            torch.cuda.synchronize()
            for k in range(reps):
                call(ev=ev[k])
            torch.cuda.synchronize()
            kms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
            st = torch.zeros(api.STATS_LEN, dtype=torch.int64, device=dev)
            call(st=st)
            torch.cuda.synchronize()
            st = st.cpu().numpy()
            fb = int(st[api.STAT_FB_RANGE] + st[api.STAT_FB_TAIL] + st[api.STAT_FB_NONFINITE])
            walked = int(st[api.STAT_ENTRIES]) - (fb - int(st[api.STAT_FB_RANGE]))
            row[wl] = {"kernel_ms": round(kms, 4), "mean_nodes": int(st[api.STAT_NODES] - st[api.STAT_FB_NODES])
                       / max(1, walked), "fallbacks": fb}
        res[name] = row
    print(json.dumps({"metric": "learned kernels with network-filled vs solver-filled tables", "n_grid": a.n,
                      "matern_entries": elems, "results": res}), flush=True)


RATE_OPS = ("v_fma_f64", "v_add_f64", "v_mul_f64", "v_fma_f32", "v_add_f32", "v_mul_f32", "v_exp_f32", "v_log_f32",
            "v_rcp_f32", "v_rcp_f64", "v_sqrt_f32", "v_cvt_f32_f64+v_cvt_f64_f32", "v_max_f32", "v_ldexp_f64",
            "v_rsq_f64", "v_add_u32")


def valu_rates_bench(torch):
    """Issue rate of single VALU instructions (paper_2502_00356_amd/csrc/valu_rates.hip):
    eight independent chains per lane, 2^15 workgroups of 256 lanes (2^17 waves), one
    timed launch per instruction. Reports wave64 instructions per CU-clock (256 CUs at
    2.4 GHz): 1.0 is one instruction per clock per CU across its four SIMDs."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2502_00356_amd", "libvalurates.so"))
    f = lib.valu_rate_ms
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)]
    blocks, iters = 1 << 15, 256
    sink = torch.empty(blocks * 256, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    rates = {}
    for op, name in enumerate(RATE_OPS):
        ms = ctypes.c_float(0.0)
        st = f(op, iters, blocks, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(ms))
        if st != 0:
            sys.exit("valu_rate_ms(%d) failed with %d" % (op, st))
        insts = blocks * 4 * iters * 8 * (2 if op == 11 else 1)      # wave64 instructions
        rates[name] = round(insts / (ms.value * 1e-3) / (256 * 2.4e9), 3)
    print(json.dumps({"metric": "VALU wave64 instructions per CU-clock (256 CUs, 2.4 GHz)", "waves": blocks * 4,
                      "chains_per_lane": 8, "iters": iters, "rates": rates}), flush=True)


def _event_ms(torch, fn, steps, warmup):
    for _ in range(max(1, warmup)):
        fn()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def deriv_bench(a, torch, api, workloads):
    """Derivatives (one JSON line). deriv-grid: K, dK/dx, dK/dnu (e^x-scaled, FP64)
    on the 2^24-pair grid, beside plain K alone. matern-grad-medium: Matern tiles
    with dC/dbeta and dC/dnu for n = 40,000 uniform points (seed 3), beta = 0.05,
    nu in {0.8, 2.3}, lower 960-tiles, FP64, beside the plain tiles alone."""
    dev = torch.device("cuda:0")
    res = {}
    if a.workload == "deriv-grid":
        nu_h, x_h, _ = workloads.grid_pairs(a.n, seed=2)
        nu = torch.from_numpy(nu_h).to(dev)
        x = torch.from_numpy(x_h).to(dev)
        outs = {k: torch.empty_like(x) for k in ("k", "dx", "dnu")}
        steps = max(1, a.steps)
        ms = _event_ms(torch, lambda: api.besselk_deriv(nu, x, result=api.RESULT_SCALED, out=outs), steps, a.warmup)
        ms_k = _event_ms(torch, lambda: api.besselk(nu, x, out=outs["k"], mode="plain", result=api.RESULT_SCALED),
                         steps, a.warmup)
        st = torch.zeros(api.STATS_LEN, dtype=torch.int64, device=dev)
        api.besselk_deriv(nu, x, result=api.RESULT_SCALED, out=outs, stats=st)
        torch.cuda.synchronize()
        st = st.cpu().numpy()
        res = {"deriv": {"ms": round(ms, 4), "evals_per_s": a.n / (ms * 1e-3),
                         "nodes_per_entry": float(st[api.STAT_NODES]) / max(1, int(st[api.STAT_ENTRIES]))},
               "plain_k": {"ms": round(ms_k, 4), "evals_per_s": a.n / (ms_k * 1e-3)},
               "cost_ratio_vs_k": ms / ms_k}
        line = {"metric": "K_nu with dK/dx and dK/dnu, evals/s", "workload": a.workload, "n": a.n,
                "dtype": "f64", "results": res}
    else:
        c = workloads.MATERN_MEDIUM
        xy = workloads.uniform_locations(c["n"], c["seed"])
        n, ts, beta = xy.shape[0], c["tile"], c["beta"]
        lx = torch.from_numpy(np.ascontiguousarray(xy[:, 0])).to(dev)
        ly = torch.from_numpy(np.ascontiguousarray(xy[:, 1])).to(dev)
        elems = api.matern_out_elems(n, ts, 1)
        bufs = {k: torch.empty(elems, dtype=torch.float64, device=dev) for k in ("c", "dbeta", "dnu")}
        steps = max(1, min(a.steps, 3))
        for nu in c["nus"]:
            ms = _event_ms(torch, lambda: api.matern_grad_tiles(lx, ly, 1.0, beta, nu, ts, 1, out=bufs), steps,
                           a.warmup)
            ms_c = _event_ms(torch, lambda: api.matern_tiles(lx, ly, 1.0, beta, nu, ts, 1, out=bufs["c"]), steps,
                             a.warmup)
            res["nu=%g" % nu] = {"ms": round(ms, 3), "entries_per_s": elems / (ms * 1e-3),
                                 "write_gbps": 3 * 8 * elems / (ms * 1e-3) / 1e9,
                                 "plain_tiles_ms": round(ms_c, 3), "cost_ratio_vs_tiles": ms / ms_c}
        line = {"metric": "Matern entries/s with dC/dbeta and dC/dnu", "workload": a.workload, "n": n, "tile": ts,
                "entries": elems, "beta": beta, "dtype": "f64", "results": res}
    print(json.dumps(line), flush=True)


def paper_bench(a, torch, api, workloads):
    """The paper's refined algorithm (Temme's series below x = 0.1, the fixed window
    [0, 9] with b = 40 bins above) on the 2^24-pair grid, beside plain FP64, plus its
    accuracy against the oracle on a 2^16 sample (the b-versus-x trade-off shows as
    large errors at large x; the RE metric of Sec. IV-C is reported per x range)."""
    dev = torch.device("cuda:0")
    nu_h, x_h, _ = workloads.grid_pairs(a.n, seed=2)
    nu = torch.from_numpy(nu_h).to(dev)
    x = torch.from_numpy(x_h).to(dev)
    out = torch.empty_like(x)
    steps = max(1, a.steps)
    ms_p = _event_ms(torch, lambda: api.besselk(nu, x, out=out, mode="paper"), steps, a.warmup)
    ms_k = _event_ms(torch, lambda: api.besselk(nu, x, out=out, mode="plain"), steps, a.warmup)
    res = {"paper_refined_b40": {"ms": round(ms_p, 4), "evals_per_s": a.n / (ms_p * 1e-3)},
           "plain_f64": {"ms": round(ms_k, 4), "evals_per_s": a.n / (ms_k * 1e-3)},
           "temme_fraction": float(np.mean(x_h < 0.1))}
    if not a.no_cpu:
        import oracle
        idx = np.random.default_rng(98).permutation(a.n)[:1 << 16]
        _, lk, _ = oracle.besselk(nu_h[idx], x_h[idx])
        sel = torch.from_numpy(idx).to(dev)
        lg = api.besselk(nu[sel].contiguous(), x[sel].contiguous(), mode="paper", result=api.RESULT_LOG)
        torch.cuda.synchronize()
        re = np.log10(1.0 + np.abs(lg.cpu().numpy() - lk) / 2.0 ** -52)
        xs = x_h[idx]
        res["max_RE"] = {"x < 0.1 (Temme)": float(re[xs < 0.1].max()),
                         "0.1 <= x <= 10": float(re[(xs >= 0.1) & (xs <= 10)].max()),
                         "10 < x <= 140": float(re[(xs > 10) & (xs <= 140)].max()),
                         "x > 140": float(re[xs > 140].max())}
    line = {"metric": "K_nu evals/s, the paper's refined algorithm", "workload": a.workload, "n": a.n,
            "dtype": "f64", "results": res}
    print(json.dumps(line), flush=True)


def small_x_bench(a, torch, api, workloads):
    """Small arguments, x in [1e-4, 0.1) (the paper's Temme region, Sec. IV-A):
    2^24 pairs, nu ~ U[0.01, 10], x log-uniform (seed 8). The paper's refined
    algorithm (Temme's series and the forward recurrence here) against the plain
    FP64 windowed quadrature: time per evaluation and accuracy on a 2^16 sample."""
    dev = torch.device("cuda:0")
    nu_h, x_h = workloads.pairs_loguniform(a.n, 8, 0.01, 10.0, -4.0, -1.0)
    nu = torch.from_numpy(nu_h).to(dev)
    x = torch.from_numpy(x_h).to(dev)
    out = torch.empty_like(x)
    steps = max(1, a.steps)
    res = {}
    for name, mode in (("temme_series", "paper"), ("windowed_quadrature_f64", "plain")):
        ms = _event_ms(torch, lambda: api.besselk(nu, x, out=out, mode=mode, result=api.RESULT_SCALED), steps,
                       a.warmup)
        res[name] = {"ms": round(ms, 4), "evals_per_s": a.n / (ms * 1e-3)}
    if not a.no_cpu:
        import oracle
        idx = np.random.default_rng(97).permutation(a.n)[:1 << 16]
        _, _, ks = oracle.besselk(nu_h[idx], x_h[idx])
        sel = torch.from_numpy(idx).to(dev)
        for name, mode in (("temme_series", "paper"), ("windowed_quadrature_f64", "plain")):
            o = api.besselk(nu[sel].contiguous(), x[sel].contiguous(), mode=mode, result=api.RESULT_SCALED)
            torch.cuda.synchronize()
            e = np.abs(o.cpu().numpy() - ks) / ks
            res[name]["max_rel_err"] = float(e.max())
            res[name]["max_RE"] = float(np.log10(1.0 + e.max() / 2.0 ** -52))
    line = {"metric": "K_nu evals/s at x in [1e-4, 0.1)", "workload": a.workload, "n": a.n, "dtype": "f64",
            "results": res, "quadrature_over_temme": res["temme_series"]["ms"] / res["windowed_quadrature_f64"]["ms"]}
    print(json.dumps(line), flush=True)


def matern_order_bench(a, torch, api, workloads):
    """Morton order against the generator's order (Sec. IV-D sorts locations along a
    Morton curve): n = 40,000 uniform points (seed 3), beta = 0.05, nu in {0.8, 2.3},
    lower 960-tiles, FP64 output, the three forms, both orders."""
    dev = torch.device("cuda:0")
    c = workloads.MATERN_MEDIUM
    model = api.Model(a.model) if os.path.exists(a.model) else None
    elems = api.matern_out_elems(c["n"], c["tile"], 1)
    out = torch.empty(elems, dtype=torch.float64, device=dev)
    ws = torch.empty(api.matern_workspace_bytes(c["n"], c["tile"], 1), dtype=torch.uint8, device=dev)
    res = {}
    for order in ("morton", "unsorted"):
        xy = workloads.uniform_locations(c["n"], c["seed"], morton=(order == "morton"))
        lx = torch.from_numpy(np.ascontiguousarray(xy[:, 0])).to(dev)
        ly = torch.from_numpy(np.ascontiguousarray(xy[:, 1])).to(dev)
        for nu in c["nus"]:
            for f in ("plain", "mixed", "learned"):
                if f == "learned" and model is None:
                    continue
                ms = _event_ms(torch, lambda: api.matern_tiles(lx, ly, 1.0, c["beta"], nu, c["tile"], 1, mode=f,
                                                               out=out, model=model, workspace=ws),
                               max(1, min(a.steps, 3)), a.warmup)
                res["%s/nu=%g/%s" % (order, nu, f)] = round(ms, 3)
    ratio = {k.replace("unsorted/", ""): res[k] / res[k.replace("unsorted", "morton")] for k in res if
             k.startswith("unsorted")}
    line = {"metric": "Matern ms per build, Morton vs unsorted locations", "workload": a.workload, "n": c["n"],
            "tile": c["tile"], "beta": c["beta"], "ms": res, "unsorted_over_morton": ratio}
    print(json.dumps(line), flush=True)


def loglik_bench(a, torch, api, workloads):
    """Gaussian log-likelihood of one GP draw under the Matern covariance, with and
    without its gradient: n = 8,192 uniform points (seed 11), beta = 0.05,
    nu = 0.8, sigma2 = 1, observations from the exponential-correlation generator
    (seed 12). Each call builds the dense covariance (and its derivative matrices),
    factorises it and reduces; the call synchronises, so it is timed by the clock."""
    dev = torch.device("cuda:0")
    c = workloads.LOGLIK
    xy = workloads.uniform_locations(c["n"], c["seed"])
    z = workloads.gp_observations(xy, c["obs_seed"], length=c["beta"])
    n = xy.shape[0]
    lx = torch.from_numpy(np.ascontiguousarray(xy[:, 0])).to(dev)
    ly = torch.from_numpy(np.ascontiguousarray(xy[:, 1])).to(dev)
    zd = torch.from_numpy(z).to(dev)
    ws = torch.empty(api.matern_loglik_workspace_bytes(n, True), dtype=torch.uint8, device=dev)
    res = {}
    for grad in (False, True):
        f = lambda: api.matern_loglik(lx, ly, zd, c["sigma2"], c["beta"], c["nu"], grad=grad, workspace=ws)
        for _ in range(max(1, a.warmup)):
            f()
        steps = max(1, min(a.steps, 3))
        t0 = time.perf_counter()
        for _ in range(steps):
            v = f()
        ms = (time.perf_counter() - t0) / steps * 1e3
        res["with_grad" if grad else "value"] = {"ms": round(ms, 3), "result": v}
    line = {"metric": "Matern Gaussian log-likelihood evaluations/s", "workload": a.workload, "n": n,
            "beta": c["beta"], "nu": c["nu"], "dtype": "f64",
            "evals_per_s": 1e3 / res["value"]["ms"], "results": res}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
