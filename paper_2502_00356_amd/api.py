"""ctypes binding of libbesselk.so (include/besselk.h).

Argument marshalling only: every step of the computation runs in the HIP
library. Tensors are torch CUDA (HIP) tensors; the work is enqueued on torch's
current stream unless a stream is given. If the library is missing this module
raises at import: there is no CPU fallback.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbesselk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libbesselk.so is not built (run __graft_entry__.build() or "
                      "python paper_2502_00356_amd/build.py); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

PLAIN_F64, MIXED_F32C, LEARNED, PAPER_REFINED = 0, 1, 2, 3
RESULT_K, RESULT_SCALED, RESULT_LOG = 0, 1, 2
OUT_F64, OUT_F32 = 0, 1
STAT_ENTRIES, STAT_NODES, STAT_FB_RANGE, STAT_FB_TAIL, STAT_NODE_RAISED, STAT_FB_NONFINITE, STAT_FB_NODES, \
    STAT_LANE_SLOTS = range(8)
STATS_LEN = 8
MLP_NPARAM = 4547
TABLE_NETWORK, TABLE_SOLVER = 0, 1
MODES = {"plain": PLAIN_F64, "mixed": MIXED_F32C, "learned": LEARNED, "paper": PAPER_REFINED}

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double


class Params(ctypes.Structure):
    _fields_ = [("mode", _i32), ("result", _i32), ("out_dtype", _i32), ("bins", _i32),
                ("L_window", _dbl), ("L_quad", _dbl), ("sigma2", _dbl), ("beta", _dbl), ("nu", _dbl),
                ("model", _vp), ("stats", _vp), ("workspace", _vp), ("workspace_bytes", ctypes.c_size_t),
                ("t_upper", _dbl), ("kernel_events", _vp * 2)]


class Locs(ctypes.Structure):
    _fields_ = [("x", _vp), ("y", _vp), ("n", _i64)]


class TrainCfg(ctypes.Structure):
    _fields_ = [("epochs", _i32), ("batch", _i32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("tau_lo", ctypes.c_float),
                ("tau_hi", ctypes.c_float), ("tau_n", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("L_window", _dbl), ("L_quad", _dbl)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_status_str = _sig("bk_status_str", ctypes.c_char_p, [ctypes.c_int])
_version = _sig("bk_version", ctypes.c_int, [])
_besselk = _sig("bk_besselk", ctypes.c_int, [_vp, _vp, _vp, _i64, _vp])
_besselk_ex = _sig("bk_besselk_ex", ctypes.c_int, [_vp, _vp, _vp, _i64, ctypes.POINTER(Params), _vp])
_ws_bytes = _sig("bk_workspace_bytes", ctypes.c_size_t, [_i64])
_mws_bytes = _sig("bk_matern_workspace_bytes", ctypes.c_size_t, [_i64, _i32, _i32])
_matern = _sig("bk_matern_tiles", ctypes.c_int, [ctypes.POINTER(Locs), ctypes.POINTER(Params), _i32, _i32, _vp, _vp])
_matern_noalloc = _sig("bk_matern_tiles_noalloc", ctypes.c_int,
                      [ctypes.POINTER(Locs), ctypes.POINTER(Params), _i32, _i32, _vp, _vp])
_out_elems = _sig("bk_matern_out_elems", _i64, [_i64, _i32, _i32])
_tile_off = _sig("bk_matern_tile_offset", _i64, [_i64, _i32, _i32, _i32, _i32])
_window = _sig("bk_window", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _dbl, _dbl, _vp])
_loglik = _sig("bk_matern_loglik", ctypes.c_int, [ctypes.POINTER(Locs), _vp, ctypes.POINTER(Params), _i32, _vp,
                                                  _vp, ctypes.c_size_t, _vp])
_loglik_ws = _sig("bk_matern_loglik_workspace_bytes", ctypes.c_size_t, [_i64, _i32])
_deriv = _sig("bk_besselk_deriv", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, ctypes.POINTER(Params), _vp])
_matern_grad = _sig("bk_matern_grad_tiles", ctypes.c_int, [ctypes.POINTER(Locs), ctypes.POINTER(Params), _i32, _i32,
                                                           _vp, _vp, _vp, _vp])
_m_create = _sig("bk_model_create", ctypes.c_int, [ctypes.POINTER(_vp)])
_m_destroy = _sig("bk_model_destroy", None, [_vp])
_m_load = _sig("bk_model_load", ctypes.c_int, [_vp, ctypes.c_char_p])
_m_save = _sig("bk_model_save", ctypes.c_int, [_vp, ctypes.c_char_p])
_m_train = _sig("bk_model_train", ctypes.c_int, [_vp, _vp, _vp, _i64, ctypes.POINTER(TrainCfg),
                                                 ctypes.POINTER(ctypes.c_float), _vp])
_m_margins = _sig("bk_model_set_margins", ctypes.c_int, [_vp, _dbl, _dbl, _dbl, _dbl])
_m_get_margins = _sig("bk_model_get_margins", ctypes.c_int, [_vp, ctypes.POINTER(_dbl)])
_m_table_source = _sig("bk_model_set_table_source", ctypes.c_int, [_vp, _i32])
_m_getp = _sig("bk_model_get_params", ctypes.c_int, [_vp, _vp])
_m_setp = _sig("bk_model_set_params", ctypes.c_int, [_vp, _vp])
_m_getn = _sig("bk_model_get_norm", ctypes.c_int, [_vp, _vp])
_m_setn = _sig("bk_model_set_norm", ctypes.c_int, [_vp, _vp])
_m_getb = _sig("bk_model_get_box", ctypes.c_int, [_vp, _vp])
_m_setb = _sig("bk_model_set_box", ctypes.c_int, [_vp, _vp])
_m_cells = _sig("bk_model_get_cells", ctypes.c_int, [_vp, _vp, _i64, _vp])
_mlp_infer = _sig("bk_mlp_infer", ctypes.c_int, [_vp, _vp, _vp, _i64, _vp])
_mlp_grad = _sig("bk_mlp_grad", ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, ctypes.c_size_t, _vp])
_mlp_grad_scratch = _sig("bk_mlp_grad_scratch_bytes", ctypes.c_size_t, [_i64])
_adam = _sig("bk_adam_step", ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _i32, ctypes.c_float, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_float, _vp])


class BkError(RuntimeError):
    def __init__(self, status):
        self.status = status
        super().__init__(_status_str(status).decode())


def _check(st):
    if st != 0:
        raise BkError(st)


def status_str(st):
    return _status_str(st).decode()


def version():
    return _version()


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _dev(t, dtype, numel=None):
    """Device pointer of a caller buffer after checking that it is a contiguous
    device tensor of the given dtype with at least numel elements."""
    if not isinstance(t, torch.Tensor):
        raise ValueError("expected a tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError("expected a contiguous %s tensor" % dtype)
    if numel is not None and t.numel() < numel:
        raise ValueError("buffer holds %d elements, %d needed" % (t.numel(), numel))
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return t.data_ptr()


def _stats(stats):
    return _dev(stats, torch.int64, STATS_LEN) if stats is not None else None


def _ws(ws, need):
    """Workspace pointer and size (a device uint8 tensor of at least need bytes)."""
    if ws is None:
        return None, 0
    _dev(ws, torch.uint8, need)
    return ws.data_ptr(), ws.numel()


def _mode(mode):
    return MODES[mode] if isinstance(mode, str) else int(mode)


def workspace_bytes(n):
    return int(_ws_bytes(int(n)))


def matern_workspace_bytes(n, tile_size, lower_only):
    """Workspace of bk_matern_tiles in the learned form (bytes)."""
    return int(_mws_bytes(int(n), int(tile_size), int(lower_only)))


def besselk(nu, x, out=None, mode="plain", result=RESULT_K, L_window=0.0, L_quad=0.0,
            stats=None, model=None, workspace=None, stream=None, bins=0, t_upper=0.0, kernel_events=None):
    """K_nu(x) (or e^x K, log K) for device float64 tensors nu, x of equal size.
    kernel_events: optional pair of torch.cuda.Event (timing enabled, recorded once
    already so that they exist), recorded around the form's main kernel."""
    n = x.numel()
    if nu.numel() != n:
        raise ValueError("nu and x differ in size")
    if out is None:
        out = torch.empty_like(x)
    if out.numel() != n:
        raise ValueError("out has the wrong size")
    m = _mode(mode)
    if m == LEARNED and workspace is None and n > 0:
        workspace = torch.empty(workspace_bytes(n), dtype=torch.uint8, device=x.device)
    wp, wb = _ws(workspace, workspace_bytes(n) if m == LEARNED else 0)
    sp = _stats(stats)
    op = _dev(out, torch.float64, n)
    p = Params(mode=m, result=int(result), L_window=float(L_window), L_quad=float(L_quad),
               bins=int(bins), t_upper=float(t_upper),
               model=(model.handle if model is not None else None),
               stats=sp, workspace=wp, workspace_bytes=wb)
    if kernel_events is not None:
        p.kernel_events[0] = kernel_events[0].cuda_event
        p.kernel_events[1] = kernel_events[1].cuda_event
    _check(_besselk_ex(_dev(nu, torch.float64), _dev(x, torch.float64), op, n, ctypes.byref(p), _stream(stream)))
    return out


def besselk_plain(nu, x, out, stream=None):
    """The fixed-signature entry point bk_besselk (plain FP64, default window)."""
    n = x.numel()
    if nu.numel() != n:
        raise ValueError("nu and x differ in size")
    _check(_besselk(_dev(nu, torch.float64), _dev(x, torch.float64), _dev(out, torch.float64, n), n, _stream(stream)))
    return out


def window(nu, x, L_window=0.0, L_quad=0.0, stream=None):
    """Plain-solver window (t_lo, t_hi, N) per pair (training targets of the MLP)."""
    n = x.numel()
    tlo = torch.empty_like(x)
    thi = torch.empty_like(x)
    nodes = torch.empty(n, dtype=torch.int32, device=x.device)
    _check(_window(_dev(nu, torch.float64), _dev(x, torch.float64), tlo.data_ptr(), thi.data_ptr(),
                   nodes.data_ptr(), n, float(L_window), float(L_quad), _stream(stream)))
    return tlo, thi, nodes


def matern_out_elems(n, tile_size, lower_only):
    return int(_out_elems(int(n), int(tile_size), int(lower_only)))


def matern_tile_offset(n, tile_size, lower_only, I, J):
    return int(_tile_off(int(n), int(tile_size), int(lower_only), int(I), int(J)))


def matern_tiles(lx, ly, sigma2, beta, nu, tile_size, lower_only, mode="plain", out_dtype=OUT_F64,
                 out=None, model=None, L_window=0.0, L_quad=0.0, stream=None, bins=0, t_upper=0.0,
                 workspace=None, stats=None, kernel_events=None):
    """Tiled Matern covariance (packed tiles, see bk_matern_tiles). The learned form
    takes a workspace of matern_workspace_bytes(n, tile_size, lower_only) bytes
    (allocated here when not given)."""
    n = lx.numel()
    if ly.numel() != n:
        raise ValueError("lx and ly differ in size")
    elems = matern_out_elems(n, tile_size, lower_only)
    dt = torch.float32 if int(out_dtype) == OUT_F32 else torch.float64
    if out is None:
        out = torch.empty(max(elems, 0), dtype=dt, device=lx.device)
    m = _mode(mode)
    need = matern_workspace_bytes(n, tile_size, lower_only) if m == LEARNED else 0
    if m == LEARNED and workspace is None and n > 0:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=lx.device)
    wp, wb = _ws(workspace, need)
    op = _dev(out, dt, max(elems, 0))
    locs = Locs(x=_dev(lx, torch.float64), y=_dev(ly, torch.float64), n=n)
    p = Params(mode=m, out_dtype=int(out_dtype), sigma2=float(sigma2), beta=float(beta), nu=float(nu),
               L_window=float(L_window), L_quad=float(L_quad), bins=int(bins), t_upper=float(t_upper),
               model=(model.handle if model is not None else None), stats=_stats(stats),
               workspace=wp, workspace_bytes=wb)
    if kernel_events is not None:
        p.kernel_events[0] = kernel_events[0].cuda_event
        p.kernel_events[1] = kernel_events[1].cuda_event
    _check(_matern(ctypes.byref(locs), ctypes.byref(p), int(tile_size), int(lower_only), op, _stream(stream)))
    return out


NOALLOC_SCRATCH_BYTES = 4 << 20


def matern_tiles_noalloc(lx, ly, sigma2, beta, nu, tile_size, lower_only, out, mode="learned", out_dtype=OUT_F32,
                         model=None, L_window=0.0, L_quad=0.0, stream=None, stats=None):
    """bk_matern_tiles_noalloc: tiled Matern covariance into the caller's packed
    output, the learned form's workspace taken from the library's static device
    scratch (no allocation in the library or here)."""
    n = lx.numel()
    if ly.numel() != n:
        raise ValueError("lx and ly differ in size")
    elems = matern_out_elems(n, tile_size, lower_only)
    dt = torch.float32 if int(out_dtype) == OUT_F32 else torch.float64
    op = _dev(out, dt, max(elems, 0))
    locs = Locs(x=_dev(lx, torch.float64), y=_dev(ly, torch.float64), n=n)
    p = Params(mode=_mode(mode), out_dtype=int(out_dtype), sigma2=float(sigma2), beta=float(beta), nu=float(nu),
               L_window=float(L_window), L_quad=float(L_quad),
               model=(model.handle if model is not None else None), stats=_stats(stats))
    _check(_matern_noalloc(ctypes.byref(locs), ctypes.byref(p), int(tile_size), int(lower_only), op,
                           _stream(stream)))
    return out


def besselk_deriv(nu, x, want=("k", "dx", "dnu"), result=RESULT_K, L_window=0.0, L_quad=0.0, stats=None,
                  stream=None, out=None):
    """K_nu(x), dK/dx and dK/dnu (bk_besselk_deriv) for device float64 tensors.
    Returns a dict with the requested outputs among "k", "dx", "dnu"; out may give
    preallocated tensors for them."""
    n = x.numel()
    if nu.numel() != n:
        raise ValueError("nu and x differ in size")
    if any(k not in ("k", "dx", "dnu") for k in want):
        raise ValueError("unknown output")
    outs = {k: (out[k] if out is not None and k in out else torch.empty_like(x)) for k in want}
    ptrs = {k: _dev(t, torch.float64, n) for k, t in outs.items()}
    p = Params(mode=PLAIN_F64, result=int(result), L_window=float(L_window), L_quad=float(L_quad),
               stats=_stats(stats))
    ptr = lambda k: ptrs.get(k)
    _check(_deriv(_dev(nu, torch.float64), _dev(x, torch.float64), ptr("k"), ptr("dx"), ptr("dnu"), n,
                  ctypes.byref(p), _stream(stream)))
    return outs


def matern_grad_tiles(lx, ly, sigma2, beta, nu, tile_size, lower_only, out_dtype=OUT_F64,
                      want=("c", "dbeta", "dnu"), L_window=0.0, L_quad=0.0, stream=None, out=None):
    """Matern tiles and their beta and nu derivatives (bk_matern_grad_tiles), packed
    like matern_tiles. Returns a dict with the requested outputs among "c", "dbeta",
    "dnu"; out may give preallocated buffers for them."""
    n = lx.numel()
    if ly.numel() != n:
        raise ValueError("lx and ly differ in size")
    if any(k not in ("c", "dbeta", "dnu") for k in want):
        raise ValueError("unknown output")
    elems = matern_out_elems(n, tile_size, lower_only)
    dt = torch.float32 if int(out_dtype) == OUT_F32 else torch.float64
    outs = {k: (out[k] if out is not None and k in out else torch.empty(max(elems, 0), dtype=dt, device=lx.device))
            for k in want}
    ptrs = {k: _dev(t, dt, max(elems, 0)) for k, t in outs.items()}
    locs = Locs(x=_dev(lx, torch.float64), y=_dev(ly, torch.float64), n=n)
    p = Params(mode=PLAIN_F64, out_dtype=int(out_dtype), sigma2=float(sigma2), beta=float(beta), nu=float(nu),
               L_window=float(L_window), L_quad=float(L_quad))
    ptr = lambda k: ptrs.get(k)
    _check(_matern_grad(ctypes.byref(locs), ctypes.byref(p), int(tile_size), int(lower_only), ptr("c"),
                        ptr("dbeta"), ptr("dnu"), _stream(stream)))
    return outs


def matern_loglik(lx, ly, z, sigma2, beta, nu, grad=False, mode="plain", model=None, workspace=None,
                  L_window=0.0, L_quad=0.0, stream=None):
    """Gaussian log-likelihood of z under the Matern covariance (bk_matern_loglik).
    Returns l, or (l, [dl/dsigma2, dl/dbeta, dl/dnu]) with grad=True. Synchronises."""
    n = lx.numel()
    if ly.numel() != n or z.numel() != n:
        raise ValueError("lx, ly and z differ in size")
    need = int(_loglik_ws(n, 1 if grad else 0))
    if need == 0:
        raise ValueError("n out of range")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=lx.device)
    wp, wb = _ws(workspace, need)
    locs = Locs(x=_dev(lx, torch.float64), y=_dev(ly, torch.float64), n=n)
    p = Params(mode=_mode(mode), sigma2=float(sigma2), beta=float(beta), nu=float(nu), L_window=float(L_window),
               L_quad=float(L_quad), model=(model.handle if model is not None else None))
    res = (ctypes.c_double * 4)()
    _check(_loglik(ctypes.byref(locs), _dev(z, torch.float64), ctypes.byref(p), 1 if grad else 0, res,
                   wp, wb, _stream(stream)))
    if grad:
        return res[0], [res[1], res[2], res[3]]
    return res[0]


def matern_loglik_workspace_bytes(n, grad=False):
    return int(_loglik_ws(int(n), 1 if grad else 0))


def unpack_tiles(packed, n, tile_size, lower_only):
    """Host helper: rebuild the dense n x n matrix (torch CPU tensor) from the packed
    tile buffer; tiles not stored (upper part when lower_only) are filled by symmetry."""
    packed = packed.cpu()
    A = torch.zeros((n, n), dtype=packed.dtype)
    T = (n + tile_size - 1) // tile_size
    for J in range(T):
        for I in range(T):
            off = matern_tile_offset(n, tile_size, lower_only, I, J)
            if off < 0:
                continue
            m = min(tile_size, n - I * tile_size)
            w = min(tile_size, n - J * tile_size)
            blk = packed[off:off + m * w].reshape(w, m).T
            A[I * tile_size:I * tile_size + m, J * tile_size:J * tile_size + w] = blk
            if lower_only and I != J:
                A[J * tile_size:J * tile_size + w, I * tile_size:I * tile_size + m] = blk.T
    return A


class Model:
    """Handle of a window-predicting MLP (bk_model)."""

    def __init__(self, path=None):
        h = _vp()
        _check(_m_create(ctypes.byref(h)))
        self.handle = h.value
        if path is not None:
            self.load(path)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            _m_destroy(h)
            self.handle = None

    def load(self, path):
        _check(_m_load(self.handle, os.fsencode(path)))

    def save(self, path):
        _check(_m_save(self.handle, os.fsencode(path)))

    def train(self, nu, x, epochs=40, batch=4096, lr=2e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              tau=(0.1, 0.9, 0.9), seed=1234, L_window=0.0, L_quad=0.0, stream=None):
        cfg = TrainCfg(epochs=epochs, batch=batch, lr=lr, beta1=beta1, beta2=beta2, eps=eps,
                       tau_lo=tau[0], tau_hi=tau[1], tau_n=tau[2], seed=seed,
                       L_window=float(L_window), L_quad=float(L_quad))
        loss = ctypes.c_float(0.0)
        _check(_m_train(self.handle, _dev(nu, torch.float64), _dev(x, torch.float64), x.numel(),
                        ctypes.byref(cfg), ctypes.byref(loss), _stream(stream)))
        return loss.value

    def set_margins(self, d_lo, d_hi, eta, n_add):
        _check(_m_margins(self.handle, float(d_lo), float(d_hi), float(eta), float(n_add)))

    def get_margins(self):
        m4 = (_dbl * 4)()
        _check(_m_get_margins(self.handle, m4))
        return tuple(m4)

    def set_table_source(self, source):
        """TABLE_NETWORK or TABLE_SOLVER (bk_model_set_table_source); rebuilds the cells."""
        _check(_m_table_source(self.handle, int(source)))

    def get_params(self):
        t = torch.empty(MLP_NPARAM, dtype=torch.float32)
        _check(_m_getp(self.handle, t.data_ptr()))
        return t

    def set_params(self, params):
        t = params.detach().to("cpu", torch.float32).contiguous()
        _check(_m_setp(self.handle, t.data_ptr()))

    def get_norm(self):
        t = torch.empty(8, dtype=torch.float64)
        _check(_m_getn(self.handle, t.data_ptr()))
        return t

    def set_norm(self, norm8):
        t = torch.as_tensor(norm8, dtype=torch.float64).contiguous()
        _check(_m_setn(self.handle, t.data_ptr()))

    def get_box(self):
        t = torch.empty(4, dtype=torch.float64)
        _check(_m_getb(self.handle, t.data_ptr()))
        return t

    def set_box(self, box4):
        t = torch.as_tensor(box4, dtype=torch.float64).contiguous()
        _check(_m_setb(self.handle, t.data_ptr()))

    def get_cells(self):
        """Prediction cells of the learned K_nu form: float32 (cells along log10 x,
        cells along nu, 4) = smallest t_lo, largest t_hi and N (normalised) that the
        network predicts at the cell's four corners, then 0."""
        dims = (ctypes.c_int32 * 2)()
        _check(_m_cells(self.handle, None, 0, dims))
        t = torch.empty((dims[0], dims[1], 4), dtype=torch.float32)
        _check(_m_cells(self.handle, t.data_ptr(), t.numel(), dims))
        return t

    def infer(self, u, stream=None):
        """Raw MLP forward (FP16 matrix cores) on normalised inputs u (n x 2 float32)."""
        n = u.shape[0]
        y = torch.empty((n, 3), dtype=torch.float32, device=u.device)
        _check(_mlp_infer(self.handle, _dev(u, torch.float32, 2 * n), y.data_ptr(), n, _stream(stream)))
        return y


def mlp_grad(params, u, target, tau, stream=None):
    """FP32 loss and gradient of one batch with the training kernels."""
    B = u.shape[0]
    grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=u.device)
    loss = torch.empty(1, dtype=torch.float32, device=u.device)
    sb = int(_mlp_grad_scratch(B))
    scratch = torch.empty(max(sb, 1), dtype=torch.uint8, device=u.device)
    _check(_mlp_grad(_dev(params, torch.float32, MLP_NPARAM), _dev(u, torch.float32, 2 * B),
                     _dev(target, torch.float32, 3 * B), _dev(tau, torch.float32, 3), B, grad.data_ptr(), loss.data_ptr(), scratch.data_ptr(), sb,
                     _stream(stream)))
    return loss, grad


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    n = p.numel()
    gp, mp, vp = (_dev(t, torch.float32, n) for t in (g, m, v))
    _check(_adam(_dev(p, torch.float32), gp, mp, vp, n, int(step), float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))
