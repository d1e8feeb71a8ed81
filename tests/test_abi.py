"""CPU-side checks of the C ABI: the library loads, exports every function that
include/besselk.h declares, validates arguments before touching the device, and
computes the tile layout on the host."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "besselk.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(bk_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    path = os.path.join(ROOT, "paper_2502_00356_amd", "libbesselk.so")
    if not os.path.exists(path):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(path)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_binding_loads():
    from paper_2502_00356_amd import api
    assert api.version() == 10000
    assert api.status_str(0) == "BK_OK"
    assert "invalid" in api.status_str(1)


def test_argument_validation_is_host_side(lib):
    """Invalid calls return BK_EINVAL before any device work (runs without a GPU)."""
    from paper_2502_00356_amd import api
    p = api.Params(mode=0)
    f = lib.bk_besselk_ex
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.POINTER(api.Params), ctypes.c_void_p]
    assert f(None, None, None, -1, ctypes.byref(p), None) == 1
    assert f(None, None, None, 5, ctypes.byref(p), None) == 1          # null arrays
    assert f(None, None, None, 0, ctypes.byref(p), None) == 0          # n == 0 is a no-op
    assert f(None, None, None, 5, None, None) == 1                     # null params
    p.result = 9
    assert f(ctypes.c_void_p(16), ctypes.c_void_p(16), ctypes.c_void_p(16), 5, ctypes.byref(p), None) == 1
    g = lib.bk_window
    g.restype = ctypes.c_int
    g.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
    assert g(None, None, None, None, None, 3, 16.0, 15.0, None) == 1
    assert g(None, None, None, None, None, -3, 16.0, 15.0, None) == 1
    m = lib.bk_matern_tiles
    m.restype = ctypes.c_int
    m.argtypes = [ctypes.POINTER(api.Locs), ctypes.POINTER(api.Params), ctypes.c_int32, ctypes.c_int32,
                  ctypes.c_void_p, ctypes.c_void_p]
    locs = api.Locs(x=None, y=None, n=10)
    for kw in (dict(beta=0.0, nu=1.0), dict(beta=0.1, nu=0.0), dict(beta=0.1, nu=1.0, sigma2=-1.0),
               dict(beta=0.1, nu=1.0, out_dtype=5)):
        q = api.Params(mode=0, sigma2=kw.get("sigma2", 1.0), beta=kw["beta"], nu=kw["nu"],
                       out_dtype=kw.get("out_dtype", 0))
        assert m(ctypes.byref(locs), ctypes.byref(q), 4, 1, ctypes.c_void_p(16), None) == 1
    q = api.Params(mode=0, sigma2=1.0, beta=0.1, nu=1.0)
    assert m(ctypes.byref(locs), ctypes.byref(q), 0, 1, ctypes.c_void_p(16), None) == 1     # tile size 0
    assert m(ctypes.byref(locs), ctypes.byref(q), 4, 1, None, None) == 1                   # null out
    locs0 = api.Locs(x=None, y=None, n=0)
    assert m(ctypes.byref(locs0), ctypes.byref(q), 4, 1, None, None) == 0


def test_noalloc_entry_point_validates_on_host(lib):
    """bk_matern_tiles_noalloc: the argument checks of bk_matern_tiles, and a call
    whose learned-form workspace would not fit the static scratch returns BK_ENOMEM
    before any device work (runs without a GPU)."""
    from paper_2502_00356_amd import api
    f = lib.bk_matern_tiles_noalloc
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.POINTER(api.Locs), ctypes.POINTER(api.Params), ctypes.c_int32, ctypes.c_int32,
                  ctypes.c_void_p, ctypes.c_void_p]
    q = api.Params(mode=api.LEARNED, sigma2=1.0, beta=0.1, nu=1.0)
    locs = api.Locs(x=ctypes.c_void_p(16), y=ctypes.c_void_p(16), n=10)
    assert f(None, ctypes.byref(q), 4, 1, ctypes.c_void_p(16), None) == 1                  # null locs
    assert f(ctypes.byref(locs), None, 4, 1, ctypes.c_void_p(16), None) == 1               # null params
    assert f(ctypes.byref(locs), ctypes.byref(q), 0, 1, ctypes.c_void_p(16), None) == 1    # tile size 0
    assert f(ctypes.byref(api.Locs(x=None, y=None, n=0)), ctypes.byref(q), 4, 1, None, None) == 0
    n, ts = 2_000_000, 64
    assert api.matern_workspace_bytes(n, ts, 1) > api.NOALLOC_SCRATCH_BYTES
    big = api.Locs(x=ctypes.c_void_p(16), y=ctypes.c_void_p(16), n=n)
    assert f(ctypes.byref(big), ctypes.byref(q), ts, 1, ctypes.c_void_p(16), None) == 3    # BK_ENOMEM
    # the 316 x 316-point lower 1,024-tile build fits
    assert api.matern_workspace_bytes(316 * 316, 1024, 1) <= api.NOALLOC_SCRATCH_BYTES
    src = open(HEADER).read()
    assert re.search(r"#define BK_NOALLOC_SCRATCH_BYTES \(4u << 20\)", src)
    assert api.NOALLOC_SCRATCH_BYTES == 4 << 20


def test_model_handle_host_calls(lib):
    """Model calls that need no device memory: create/destroy, the prediction-cell
    dimensions, and the argument checks of the cell copy (runs without a GPU)."""
    vp = ctypes.c_void_p
    lib.bk_model_create.argtypes = [ctypes.POINTER(vp)]
    lib.bk_model_create.restype = ctypes.c_int
    lib.bk_model_destroy.argtypes = [vp]
    lib.bk_model_get_cells.argtypes = [vp, vp, ctypes.c_int64, vp]
    lib.bk_model_get_cells.restype = ctypes.c_int
    lib.bk_model_set_margins.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.bk_model_set_margins.restype = ctypes.c_int
    h = vp()
    assert lib.bk_model_create(ctypes.byref(h)) == 0
    try:
        dims = (ctypes.c_int32 * 2)()
        assert lib.bk_model_get_cells(h, None, 0, dims) == 0
        assert dims[0] > 0 and dims[1] > 0
        buf = (ctypes.c_float * 4)()
        assert lib.bk_model_get_cells(h, buf, 4, dims) == 1                     # capacity too small
        big = (ctypes.c_float * (4 * dims[0] * dims[1]))()
        assert lib.bk_model_get_cells(h, big, 4 * dims[0] * dims[1], dims) == 4  # BK_ENOMODEL: no parameters yet
        assert lib.bk_model_get_cells(None, None, 0, dims) == 1
        assert lib.bk_model_get_cells(h, None, 0, None) == 1
        assert lib.bk_model_set_margins(h, -1.0, 0.0, 0.0, 0.0) == 1
        assert lib.bk_model_set_margins(h, 0.05, 0.05, 0.0, 0.0) == 0           # no parameters: host only
    finally:
        lib.bk_model_destroy(h)


def test_derivative_entry_points_validate_on_host(lib):
    from paper_2502_00356_amd import api
    d = lib.bk_besselk_deriv
    d.restype = ctypes.c_int
    d.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_int64, ctypes.POINTER(api.Params), ctypes.c_void_p]
    a = ctypes.c_void_p(16)
    assert d(a, a, a, a, a, -1, None, None) == 1
    assert d(a, a, None, None, None, 4, None, None) == 1              # no output requested
    assert d(None, a, a, None, None, 4, None, None) == 1              # null input
    assert d(None, None, None, None, None, 0, None, None) == 0        # n == 0
    for kw in (dict(mode=1), dict(mode=2), dict(result=2), dict(L_window=-1.0)):
        p = api.Params(**kw)
        assert d(a, a, a, a, a, 4, ctypes.byref(p), None) == 1, kw
    g = lib.bk_matern_grad_tiles
    g.restype = ctypes.c_int
    g.argtypes = [ctypes.POINTER(api.Locs), ctypes.POINTER(api.Params), ctypes.c_int32, ctypes.c_int32,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    locs = api.Locs(x=a, y=a, n=10)
    ok = dict(sigma2=1.0, beta=0.1, nu=1.2)
    for kw in (dict(ok, mode=1), dict(ok, beta=0.0), dict(ok, nu=0.0), dict(ok, out_dtype=7)):
        p = api.Params(**kw)
        assert g(ctypes.byref(locs), ctypes.byref(p), 4, 1, a, a, a, None) == 1, kw
    p = api.Params(**ok)
    assert g(ctypes.byref(locs), ctypes.byref(p), 4, 1, None, None, None, None) == 1
    assert g(ctypes.byref(locs), ctypes.byref(p), 0, 1, a, None, None, None) == 1
    locs0 = api.Locs(x=None, y=None, n=0)
    assert g(ctypes.byref(locs0), ctypes.byref(p), 4, 1, None, None, None, None) == 0


@pytest.mark.parametrize("n,ts,lower", [(40000, 960, 1), (99856, 1024, 1), (1024, 1024, 0), (350, 100, 1),
                                        (350, 100, 0), (1, 5, 1), (7, 7, 1)])
def test_tile_layout(n, ts, lower):
    """Offsets follow J-major order with each tile m_I x n_J contiguous, and the
    last offset plus the last tile's size is the total element count."""
    from paper_2502_00356_amd import api
    T = (n + ts - 1) // ts
    expect = 0
    for J in range(T):
        for I in range(T):
            off = api.matern_tile_offset(n, ts, lower, I, J)
            if lower and J > I:
                assert off == -1
                continue
            assert off == expect, (I, J)
            expect += min(ts, n - I * ts) * min(ts, n - J * ts)
    assert api.matern_out_elems(n, ts, lower) == expect
    if lower:
        assert expect == sum(min(ts, n - I * ts) * min(ts, n - J * ts) for J in range(T) for I in range(J, T))


def test_workload_sizes():
    """Sizes of the Matern workloads: 819,097,600 entries for n = 40,000 in lower
    960-tiles, 5,036,605,696 for the 316 x 316 grid in lower 1,024-tiles."""
    from paper_2502_00356_amd import api
    assert api.matern_out_elems(40000, 960, 1) == 819097600
    assert api.matern_out_elems(99856, 1024, 1) == 5036605696
    assert api.matern_out_elems(1024, 1024, 0) == 1024 * 1024


def test_struct_layouts_match_the_header(tmp_path):
    """The ctypes mirrors of bk_params, bk_locs and bk_train_cfg have the sizes and
    field offsets the C compiler gives the header's structs."""
    import ctypes
    import subprocess
    from paper_2502_00356_amd import api
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    checks = [("bk_params", api.Params), ("bk_locs", api.Locs), ("bk_train_cfg", api.TrainCfg)]
    lines = ['#include "besselk.h"', "#include <stdio.h>", "#include <stddef.h>", "int main(void) {"]
    for cname, cls in checks:
        lines.append('printf("%%zu\\n", sizeof(%s));' % cname)
        for fname, _ in cls._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (cname, fname))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(root, "include"), "-I", "/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    want = []
    for _, cls in checks:
        want.append(ctypes.sizeof(cls))
        want.extend(getattr(cls, f).offset for f, _ in cls._fields_)
    assert got == want


def test_binding_rejects_bad_caller_buffers():
    """Every caller buffer is checked for dtype, contiguity, size and device before
    its pointer reaches the library (these checks run without a GPU: the device test
    comes last, so each case below raises on the property it breaks)."""
    import torch
    from paper_2502_00356_amd import api
    f64 = torch.zeros(8, dtype=torch.float64)
    with pytest.raises(ValueError, match="device"):          # host tensors
        api.besselk(f64, f64, out=f64.clone())
    with pytest.raises(ValueError, match="float64"):         # an FP32 buffer for FP64 output
        api.besselk_deriv(f64, f64, want=("k",), out={"k": torch.zeros(8, dtype=torch.float32)})
    with pytest.raises(ValueError, match="needed"):          # too short for the outputs
        api.besselk_deriv(f64, f64, want=("dx",), out={"dx": torch.zeros(4, dtype=torch.float64)})
    with pytest.raises(ValueError, match="needed"):          # statistics array shorter than STATS_LEN
        api.besselk(f64, f64, out=f64.clone(), stats=torch.zeros(4, dtype=torch.int64))
    with pytest.raises(ValueError, match="int64"):
        api.besselk(f64, f64, out=f64.clone(), stats=torch.zeros(8, dtype=torch.int32))
    with pytest.raises(ValueError, match="contiguous"):
        api.besselk(f64, f64, out=torch.zeros(16, dtype=torch.float64)[::2])
    with pytest.raises(ValueError, match="needed"):          # learned workspace too small
        api.besselk(f64, f64, out=f64.clone(), mode="learned", workspace=torch.zeros(16, dtype=torch.uint8))
    with pytest.raises(ValueError, match="float32"):         # Matern output of the wrong element type
        api.matern_tiles(f64, f64, 1.0, 0.1, 1.0, 8, 1, out_dtype=api.OUT_F32, out=torch.zeros(64, dtype=torch.float64))
    with pytest.raises(ValueError, match="needed"):
        api.matern_tiles(f64, f64, 1.0, 0.1, 1.0, 8, 1, out=torch.zeros(10, dtype=torch.float64))
    with pytest.raises(ValueError, match="needed"):
        api.matern_tiles(f64, f64, 1.0, 0.1, 1.0, 4, 1, mode="learned", out=torch.zeros(64, dtype=torch.float64),
                         workspace=torch.zeros(64, dtype=torch.uint8))
    with pytest.raises(ValueError, match="needed"):
        api.matern_grad_tiles(f64, f64, 1.0, 0.1, 1.0, 8, 1, want=("c",), out={"c": torch.zeros(10, dtype=torch.float64)})
    with pytest.raises(ValueError, match="needed"):
        api.adam_step(torch.zeros(8), torch.zeros(4), torch.zeros(8), torch.zeros(8), 1, 1e-3)


def test_matern_workspace_size():
    """Learned Matern workspace: 128 KiB of tables plus one bit per wave of 64 x 32
    entries, in 256-byte units."""
    from paper_2502_00356_amd import api
    assert api.matern_workspace_bytes(0, 64, 1) == 0
    assert api.matern_workspace_bytes(10, 0, 1) == 0
    # n = 1024 full matrix in one 1024-tile: 16 x 8 workgroups of 4 waves = 512 bits, one 256-byte unit
    assert api.matern_workspace_bytes(1024, 1024, 0) == 131072 + 256
    # 316^2 grid, lower 1024-tiles: 98 tile rows, 4851 tiles of 16 x 8 workgroups
    waves = 4851 * 16 * 8 * 4
    assert api.matern_workspace_bytes(99856, 1024, 1) == 131072 + ((waves + 31) // 32 * 4 + 255) // 256 * 256
