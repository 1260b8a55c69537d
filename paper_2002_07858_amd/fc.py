"""Thin ctypes binding of libfc.so (include/fc.h), same names as the C ABI.

Argument marshalling only: host arrays are numpy, device arrays are torch CUDA
tensors (PyTorch-ROCm supplies device memory and streams), and every step of
the computation runs in the library's HIP kernels.  There is no CPU fallback:
if libfc.so is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfc.so")

FC_OK = 0
FC_ERR_INVALID_ARG = -1
FC_ERR_NOT_PD = -2
FC_ERR_NOMEM = -3
FC_ERR_DEVICE = -4
FC_ERR_STATE = -5
FC_ERR_UNSUPPORTED = -6

FC_FORM_FP64 = 1
FC_FORM_FP32 = 2
FC_FORM_SPLIT_BF16 = 4
FC_FORM_SPLIT_FP16 = 8

FC_STAT_PEARSON = 0
FC_STAT_FIXED = 1

FC_MAX_BINS = 64
FC_NO_ALLOC_SCRATCH_BYTES = 32 << 20

FC_SCHED_FAIR = 0
FC_SCHED_FIFO = 1

FC_REQ_QUEUED = 0
FC_REQ_RUNNING = 1
FC_REQ_DONE = 2
FC_REQ_FAILED = -1

EXPORTED = ("fc_build_grid", "fc_build_covariance", "fc_scan", "fc_scan_points",
            "fc_scan_points_workspace", "fc_scan_state_init", "fc_scan_slice",
            "fc_scan_points_slice", "fc_scan_points_slice_workspace", "fc_scan_state_finalize",
            "fc_critical_value",
            "fc_scan_fixed_m", "fc_generate_universes", "fc_region", "fc_data_scan",
            "fc_acceptance",
            "fc_grid_inverse_cov", "fc_grid_info",
            "fc_grid_device_bytes", "fc_grid_destroy", "fc_last_error", "fc_server_create", "fc_server_submit",
            "fc_server_submit_drawn", "fc_server_poll",
            "fc_server_stats", "fc_server_destroy", "fc_profile_enable", "fc_profile_read",
            "fc_scan_no_alloc")


class FCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None
_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_dbl = ctypes.c_double


def lib():
    """Load libfc.so (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2002_07858_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.fc_build_grid.argtypes = [ctypes.POINTER(_p), _i32, _p, _p, _i32, _p, _p, _p]
        L.fc_build_covariance.argtypes = [_p, _p, _i32, _p, _u32, _p, _p]
        L.fc_scan.argtypes = [_p, _i32, _i64, _p, _p, _p, _p, _p, _p, _p]
        L.fc_scan_no_alloc.argtypes = [_p, _i32, _i64, _p, _p, _p, _p, _p, _p, _p]
        L.fc_scan_no_alloc.restype = ctypes.c_int
        L.fc_scan_points.argtypes = [_p, _i32, _i64, _p, _p, _i64, _p, _p, ctypes.c_size_t, _p,
                                     _p, _p, _p, _p]
        L.fc_scan_points_workspace.argtypes = [_p, _i32, _i64, _i64, _p]
        L.fc_scan_state_init.argtypes = [_i64, _p, _p, _p]
        L.fc_scan_slice.argtypes = [_p, _i32, _i64, _p, _p, _i64, _i64, _p, _p, _p]
        L.fc_scan_points_slice.argtypes = [_p, _i32, _i64, _p, _p, _i64, _p, _i64, _i64, _p,
                                           ctypes.c_size_t, _p, _p, _p]
        L.fc_scan_points_slice_workspace.argtypes = [_p, _i32, _i64, _i64, _i64, _p]
        L.fc_scan_state_finalize.argtypes = [_p, _i64, _p, _p, _p, _p, _p, _p, _p]
        L.fc_critical_value.argtypes = [_i64, _p, _p, _i32, _p, _p, _i32, _dbl, _p, _p]
        L.fc_generate_universes.argtypes = [_p, _i64, _p, _p, _p, ctypes.c_uint64, _i64, _p, _p,
                                            _p, _p]
        L.fc_scan_fixed_m.argtypes = [_p, _i64, _p, _p, _i32, _p, _p, _p, _p, _p, _p, _p]
        L.fc_region.argtypes = [_p, _i32, _i64, _p, _i64, _i64, _dbl, ctypes.c_uint64, _i32, _p,
                                _p, _p, _p, _p, _p, _p, _p]
        L.fc_data_scan.argtypes = [_p, _p, _p, _p, _p, _p]
        L.fc_acceptance.argtypes = [_p, _i64, _p, _p, _i64, _p, _p, _p]
        L.fc_grid_inverse_cov.argtypes = [_p, _i64, _i64, _p, _p]
        L.fc_grid_info.argtypes = [_p, _p, _p, _p, _p]
        L.fc_grid_device_bytes.argtypes = [_p]
        L.fc_grid_device_bytes.restype = ctypes.c_size_t
        L.fc_grid_destroy.argtypes = [_p]
        L.fc_grid_destroy.restype = None
        L.fc_last_error.argtypes = []
        L.fc_last_error.restype = ctypes.c_char_p
        L.fc_server_create.argtypes = [ctypes.POINTER(_p), _p, _i32, _i32, ctypes.c_size_t,
                                       ctypes.c_size_t, _i32, _p, _i32, _dbl, _dbl, _i32]
        L.fc_server_submit.argtypes = [_p, _i32, _i64, _i64, _p, _p]
        L.fc_server_submit_drawn.argtypes = [_p, _i32, _i64, _i64, ctypes.c_uint64, _i64, _p]
        L.fc_server_poll.argtypes = [_p, _i64, _p, _p, _p, _p, _p, _p, _p, _p, _i32]
        L.fc_server_stats.argtypes = [_p, _p, _p, _p, _p]
        L.fc_server_destroy.argtypes = [_p]
        L.fc_server_destroy.restype = None
        L.fc_profile_enable.argtypes = [_i32]
        L.fc_profile_enable.restype = ctypes.c_int
        L.fc_profile_read.argtypes = [ctypes.c_char_p, _p, _p]
        L.fc_profile_read.restype = ctypes.c_int
        for name in ("fc_server_create", "fc_server_submit", "fc_server_submit_drawn",
                     "fc_server_poll", "fc_server_stats"):
            getattr(L, name).restype = ctypes.c_int
        for name in ("fc_build_grid", "fc_build_covariance", "fc_scan", "fc_scan_points",
                     "fc_scan_points_workspace", "fc_scan_state_init", "fc_scan_slice",
                     "fc_scan_points_slice", "fc_scan_points_slice_workspace",
                     "fc_scan_state_finalize", "fc_critical_value",
                     "fc_scan_fixed_m", "fc_generate_universes", "fc_region", "fc_data_scan",
            "fc_acceptance",
            "fc_grid_inverse_cov", "fc_grid_info"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def fc_last_error() -> str:
    return lib().fc_last_error().decode()


def _check(rc: int):
    if rc != FC_OK:
        raise FCError(rc, fc_last_error())


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _hp(a):
    return None if a is None else a.ctypes.data_as(_p)


def _dev(t, dtype_name: str, name: str):
    """Device pointer of a contiguous torch CUDA tensor of the given dtype (or None)."""
    if t is None:
        return None
    import torch
    want = {"f64": torch.float64, "i64": torch.int64, "u8": torch.uint8,
            "i32": torch.int32}[dtype_name]
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch CUDA tensor")
    if t.dtype != want:
        raise TypeError(f"{name} must have dtype {want}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return _p(t.data_ptr()) if t.numel() else None


def _need(t, n: int, name: str):
    """Size check before a device pointer goes to the library: a tensor that
    is too short would be read or written past its end by the kernels."""
    if t is not None and int(t.numel()) < int(n):
        raise ValueError(f"{name} holds {int(t.numel())} elements, the call needs {int(n)}")


def _rows(d, N: int, name: str = "d") -> int:
    """K of a [K][N] universe tensor (checked against the grid's bin count)."""
    if d is None:
        return 0
    if d.dim() != 2 or int(d.shape[1]) != int(N):
        raise ValueError(f"{name} must be [K][{N}] for this grid, got {tuple(d.shape)}")
    return int(d.shape[0])


def _stream(stream):
    if stream is None:
        import torch
        return _p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _p(stream)
    return _p(stream.cuda_stream)


class Grid:
    """Owning wrapper of an fc_grid handle."""

    def __init__(self, handle: int):
        self.handle = handle
        self._shape = None

    @property
    def N(self) -> int:
        return self._sizes()[0]

    @property
    def G(self) -> int:
        return self._sizes()[1]

    def _sizes(self):
        if self._shape is None:
            i = fc_grid_info(self)
            self._shape = (i["N"], i["G"])
        return self._shape

    @property
    def _h(self):
        if not self.handle:
            raise FCError(FC_ERR_STATE, "grid was destroyed")
        return _p(self.handle)

    def info(self):
        return fc_grid_info(self)

    def device_bytes(self) -> int:
        return fc_grid_device_bytes(self)

    def destroy(self):
        if self.handle:
            lib().fc_grid_destroy(_p(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def fc_build_grid(axes, signal, central=None, stream=None) -> Grid:
    """Make a grid resident: ``axes`` is a list of D 1-D arrays, ``signal`` [G][N]."""
    lens = _host([len(a) for a in axes], np.int64)
    vals = _host(np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in axes]),
                 np.float64)
    S = _host(signal, np.float64)
    if S.ndim != 2:
        raise ValueError("signal must be [G][N]")
    c = None if central is None else _host(central, np.float64)
    out = _p()
    _check(lib().fc_build_grid(ctypes.byref(out), len(axes), _hp(lens), _hp(vals),
                               int(S.shape[1]), _hp(S), _hp(c), _stream(stream)))
    return Grid(out.value)


def fc_build_covariance(grid: Grid, frac_cov, stat_mode=FC_STAT_PEARSON, stat_diag=None,
                        forms=FC_FORM_FP32 | FC_FORM_FP64, stream=None) -> int:
    """Build every requested form; returns -1, raises FCError (with .bad_q) if not PD."""
    F = _host(frac_cov, np.float64)
    sd = None if stat_diag is None else _host(stat_diag, np.float64)
    bad = np.full(1, -1, dtype=np.int64)
    rc = lib().fc_build_covariance(grid._h, _hp(F), int(stat_mode), _hp(sd), int(forms),
                                   _hp(bad), _stream(stream))
    if rc != FC_OK:
        err = FCError(rc, fc_last_error())
        err.bad_q = int(bad[0])
        raise err
    return int(bad[0])


def fc_scan(grid: Grid, form: int, d, p_idx, dchi2, chi2_min=None, argmin=None, chi2_p=None,
            stream=None):
    """Enqueue the scan of K = d.shape[0] universes (all arrays torch CUDA
    tensors; chi2_min, argmin and chi2_p are optional outputs)."""
    K = _rows(d, grid.N)
    for t, n in ((p_idx, "p_idx"), (dchi2, "dchi2"), (chi2_min, "chi2_min"), (argmin, "argmin"),
                 (chi2_p, "chi2_p")):
        _need(t, K, n)
    _check(lib().fc_scan(grid._h, int(form), K, _dev(d, "f64", "d"), _dev(p_idx, "i64", "p_idx"),
                         _dev(dchi2, "f64", "dchi2"), _dev(chi2_min, "f64", "chi2_min"),
                         _dev(argmin, "i64", "argmin"), _dev(chi2_p, "f64", "chi2_p"),
                         _stream(stream)))


def fc_scan_no_alloc(grid: Grid, form: int, d, p_idx, dchi2, chi2_min=None, argmin=None,
                     chi2_p=None, stream=None):
    """fc_scan without any device allocation in the call: its scratch lives in
    the library's static per-device array (calls on one device must not
    overlap in time)."""
    K = _rows(d, grid.N)
    for t, n in ((p_idx, "p_idx"), (dchi2, "dchi2"), (chi2_min, "chi2_min"), (argmin, "argmin"),
                 (chi2_p, "chi2_p")):
        _need(t, K, n)
    _check(lib().fc_scan_no_alloc(grid._h, int(form), K, _dev(d, "f64", "d"),
                                  _dev(p_idx, "i64", "p_idx"), _dev(dchi2, "f64", "dchi2"),
                                  _dev(chi2_min, "f64", "chi2_min"), _dev(argmin, "i64", "argmin"),
                                  _dev(chi2_p, "f64", "chi2_p"), _stream(stream)))


def fc_scan_points_workspace(grid: Grid, form: int, n_pts: int, K: int) -> int:
    """Bytes of workspace fc_scan_points needs."""
    b = ctypes.c_size_t()
    _check(lib().fc_scan_points_workspace(grid._h, int(form), int(n_pts), int(K),
                                          ctypes.byref(b)))
    return b.value


def fc_scan_points(grid: Grid, form: int, p, seg_off, d, dchi2, chi2_min=None, argmin=None,
                   chi2_p=None, workspace=None, stream=None):
    """Enqueue the scan of universes grouped by true point: segment i of
    seg_off (n_pts + 1 offsets) holds universes of true point p[i].  The
    workspace (a uint8 CUDA tensor) is allocated here when not given."""
    import torch
    K = _rows(d, grid.N)
    n_pts = int(p.numel())
    _need(seg_off, n_pts + 1, "seg_off")
    for t, n in ((dchi2, "dchi2"), (chi2_min, "chi2_min"), (argmin, "argmin"), (chi2_p, "chi2_p")):
        _need(t, K, n)
    need = fc_scan_points_workspace(grid, form, n_pts, K)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=d.device)
    _check(lib().fc_scan_points(grid._h, int(form), n_pts, _dev(p, "i64", "p"),
                                _dev(seg_off, "i64", "seg_off"), K, _dev(d, "f64", "d"),
                                _dev(workspace, "u8", "workspace"), int(workspace.numel()),
                                _dev(dchi2, "f64", "dchi2"), _dev(chi2_min, "f64", "chi2_min"),
                                _dev(argmin, "i64", "argmin"), _dev(chi2_p, "f64", "chi2_p"),
                                _stream(stream)))
    return workspace


def fc_scan_state_init(keys, chi2_p, stream=None):
    """Enqueue keys = none, chi2_p = 0 for a grid-sliced scan.  keys is an
    int64 CUDA tensor holding the uint64 keys bit for bit."""
    K = int(keys.numel())
    _need(chi2_p, K, "chi2_p")
    _check(lib().fc_scan_state_init(K, _dev(keys, "i64", "keys"), _dev(chi2_p, "f64", "chi2_p"),
                                    _stream(stream)))


def fc_scan_slice(grid: Grid, form: int, d, p_idx, q0: int, nq: int, keys, chi2_p, stream=None):
    """Enqueue the scan of grid points [q0, q0 + nq), merged into (keys, chi2_p)."""
    K = _rows(d, grid.N)
    for t, n in ((p_idx, "p_idx"), (keys, "keys"), (chi2_p, "chi2_p")):
        _need(t, K, n)
    _check(lib().fc_scan_slice(grid._h, int(form), K, _dev(d, "f64", "d"),
                               _dev(p_idx, "i64", "p_idx"), int(q0), int(nq),
                               _dev(keys, "i64", "keys"), _dev(chi2_p, "f64", "chi2_p"),
                               _stream(stream)))


def fc_scan_points_slice_workspace(grid: Grid, form: int, n_pts: int, K: int, nq: int) -> int:
    """Bytes of workspace fc_scan_points_slice needs for nq grid points."""
    b = ctypes.c_size_t()
    _check(lib().fc_scan_points_slice_workspace(grid._h, int(form), int(n_pts), int(K), int(nq),
                                                ctypes.byref(b)))
    return b.value


def fc_scan_points_slice(grid: Grid, form: int, p, seg_off, d, q0: int, nq: int, keys, chi2_p,
                         workspace=None, stream=None):
    """Enqueue the points scan of grid points [q0, q0 + nq), merged into
    (keys, chi2_p).  The workspace is allocated here when not given."""
    import torch
    K = _rows(d, grid.N)
    n_pts = int(p.numel())
    _need(seg_off, n_pts + 1, "seg_off")
    for t, n in ((keys, "keys"), (chi2_p, "chi2_p")):
        _need(t, K, n)
    need = fc_scan_points_slice_workspace(grid, form, n_pts, K, nq)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=d.device)
    _check(lib().fc_scan_points_slice(grid._h, int(form), n_pts, _dev(p, "i64", "p"),
                                      _dev(seg_off, "i64", "seg_off"), K, _dev(d, "f64", "d"),
                                      int(q0), int(nq), _dev(workspace, "u8", "workspace"),
                                      int(workspace.numel()), _dev(keys, "i64", "keys"),
                                      _dev(chi2_p, "f64", "chi2_p"), _stream(stream)))
    return workspace


def fc_scan_state_finalize(grid: Grid, p_idx, keys, chi2_p, dchi2, chi2_min, argmin,
                           stream=None):
    """Enqueue the decoding of a merged sliced-scan state into fc_scan's outputs."""
    K = int(keys.numel())
    for t, n in ((p_idx, "p_idx"), (chi2_p, "chi2_p"), (dchi2, "dchi2"), (chi2_min, "chi2_min"),
                 (argmin, "argmin")):
        _need(t, K, n)
    _check(lib().fc_scan_state_finalize(grid._h, K, _dev(p_idx, "i64", "p_idx"),
                                        _dev(keys, "i64", "keys"), _dev(chi2_p, "f64", "chi2_p"),
                                        _dev(dchi2, "f64", "dchi2"),
                                        _dev(chi2_min, "f64", "chi2_min"),
                                        _dev(argmin, "i64", "argmin"), _stream(stream)))


def fc_critical_value(seg_off, dchi2, alpha, crit, n_bins=200, hist_hi=50.0, hist=None,
                      stream=None):
    """Enqueue critical values (and histograms) for n_seg = seg_off.numel()-1 segments."""
    a = _host(np.atleast_1d(alpha), np.float64)
    n_seg = int(seg_off.numel()) - 1
    _need(crit, max(n_seg, 0) * a.shape[0], "crit")
    _need(hist, max(n_seg, 0) * (int(n_bins) + 1), "hist")
    _check(lib().fc_critical_value(n_seg, _dev(seg_off, "i64", "seg_off"),
                                   _dev(dchi2, "f64", "dchi2"), int(a.shape[0]), _hp(a),
                                   _dev(crit, "f64", "crit"), int(n_bins), float(hist_hi),
                                   _dev(hist, "i64", "hist"), _stream(stream)))


def fc_scan_fixed_m(grid: Grid, d, p_idx, dchi2, chi2_min, argmin, chi2_p, max_iter=0,
                    m_final=None, iters=None, stream=None):
    """One matrix per universe scan (M = Sigma_m^-1, m = p, iterated up to
    max_iter times at the minimiser); synchronous; torch CUDA tensors."""
    K = _rows(d, grid.N)
    for t, n in ((p_idx, "p_idx"), (dchi2, "dchi2"), (chi2_min, "chi2_min"), (argmin, "argmin"),
                 (chi2_p, "chi2_p"), (m_final, "m_final"), (iters, "iters")):
        _need(t, K, n)
    _check(lib().fc_scan_fixed_m(grid._h, K, _dev(d, "f64", "d"), _dev(p_idx, "i64", "p_idx"),
                                 int(max_iter), _dev(dchi2, "f64", "dchi2"),
                                 _dev(chi2_min, "f64", "chi2_min"), _dev(argmin, "i64", "argmin"),
                                 _dev(chi2_p, "f64", "chi2_p"), _dev(m_final, "i64", "m_final"),
                                 _dev(iters, "i32", "iters"), _stream(stream)))


def fc_generate_universes(grid: Grid, p, seg_off, seed: int, d, p_idx=None, counts=None,
                          u_first=None, stream=None):
    """Enqueue universes of true points p[k] into rows seg_off[k]..seg_off[k+1]-1 of d.

    p, seg_off, u_first: int64 CUDA tensors; d: float64 [K][N]; p_idx int64 [K]
    and counts int32 [K][N] optional outputs.
    """
    K = _rows(d, grid.N)
    _need(seg_off, int(p.numel()) + 1, "seg_off")
    _need(u_first, int(p.numel()), "u_first")
    _need(p_idx, K, "p_idx")
    _need(counts, K * grid.N, "counts")
    _check(lib().fc_generate_universes(grid._h, int(p.numel()), _dev(p, "i64", "p"),
                                       _dev(seg_off, "i64", "seg_off"),
                                       _dev(u_first, "i64", "u_first"),
                                       ctypes.c_uint64(int(seed) % 2**64), K,
                                       _dev(d, "f64", "d"), _dev(p_idx, "i64", "p_idx"),
                                       _dev(counts, "i32", "counts"), _stream(stream)))


def fc_region(grid: Grid, form: int, dchi2_data, crit, accepted, pts=None, K0=256, K_max=4096,
              z=2.0, seed=0, alpha=(0.6827, 0.9, 0.95), stream=None):
    """Feldman-Cousins region with per-point universe counts (synchronous).

    pts: host grid indices or None (every point); dchi2_data float64 CUDA [G];
    crit float64 CUDA [n_pts][n_alpha]; accepted uint8 CUDA [n_pts][n_alpha].
    Returns dict(K_used=np.ndarray, rounds=int, evals=float).
    """
    G = fc_grid_info(grid)["G"]
    pa = None if pts is None else _host(pts, np.int64)
    n_pts = G if pa is None else int(pa.shape[0])
    a = _host(np.atleast_1d(alpha), np.float64)
    _need(dchi2_data, G, "dchi2_data")
    _need(crit, n_pts * a.shape[0], "crit")
    _need(accepted, n_pts * a.shape[0], "accepted")
    K_used = np.zeros(n_pts, dtype=np.int64)
    rounds = ctypes.c_int32()
    evals = ctypes.c_double()
    _check(lib().fc_region(grid._h, int(form), n_pts, _hp(pa), int(K0), int(K_max), float(z),
                           ctypes.c_uint64(int(seed) % 2**64), int(a.shape[0]), _hp(a),
                           _dev(dchi2_data, "f64", "dchi2_data"), _dev(crit, "f64", "crit"),
                           _dev(accepted, "u8", "accepted"), _hp(K_used), ctypes.byref(rounds),
                           ctypes.byref(evals), _stream(stream)))
    return dict(K_used=K_used, rounds=rounds.value, evals=evals.value)


def fc_data_scan(grid: Grid, dchi2_data, central=None, stream=None):
    """Delta chi2 of the data vector at every grid point (synchronous).

    ``dchi2_data`` is a float64 CUDA tensor [G]; ``central`` a host vector [N]
    or None for the grid's own.  Returns (chi2_min, argmin).
    """
    c = None if central is None else _host(central, np.float64)
    if c is not None and c.shape != (grid.N,):
        raise ValueError(f"central must hold {grid.N} bins")
    _need(dchi2_data, grid.G, "dchi2_data")
    m = ctypes.c_double()
    a = ctypes.c_int64()
    _check(lib().fc_data_scan(grid._h, _hp(c), _dev(dchi2_data, "f64", "dchi2_data"),
                              ctypes.byref(m), ctypes.byref(a), _stream(stream)))
    return m.value, a.value


def fc_acceptance(grid: Grid, p, crit, dchi2_data, accepted, crit_stride=1, stream=None):
    """Enqueue accepted[k] = dchi2_data[p[k]] <= crit[k * crit_stride] (CUDA tensors)."""
    n = int(p.numel())
    _need(accepted, n, "accepted")
    _need(crit, (n - 1) * int(crit_stride) + 1 if n else 0, "crit")
    _need(dchi2_data, grid.G, "dchi2_data")
    _check(lib().fc_acceptance(grid._h, n, _dev(p, "i64", "p"), _dev(crit, "f64", "crit"),
                               int(crit_stride), _dev(dchi2_data, "f64", "dchi2_data"),
                               _dev(accepted, "u8", "accepted"), _stream(stream)))


def fc_grid_inverse_cov(grid: Grid, q0: int, nq: int, out, stream=None):
    _need(out, int(nq) * grid.N * grid.N, "out")
    _check(lib().fc_grid_inverse_cov(grid._h, int(q0), int(nq), _dev(out, "f64", "out"),
                                     _stream(stream)))


def fc_grid_info(grid: Grid):
    D = ctypes.c_int32()
    N = ctypes.c_int32()
    G = ctypes.c_int64()
    forms = ctypes.c_uint32()
    _check(lib().fc_grid_info(grid._h, ctypes.byref(D), ctypes.byref(N), ctypes.byref(G),
                              ctypes.byref(forms)))
    return dict(D=D.value, N=N.value, G=G.value, forms=forms.value)


def fc_profile_enable(on: bool = True):
    """Start (clearing earlier records) or stop kernel timing with HIP events."""
    _check(lib().fc_profile_enable(1 if on else 0))


def fc_profile_read(kernel: str):
    """(launches, total ms) of one kernel's timed launches since fc_profile_enable(True)."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(lib().fc_profile_read(kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def fc_grid_device_bytes(grid: Grid) -> int:
    return int(lib().fc_grid_device_bytes(grid._h))


def fc_grid_destroy(grid: Grid):
    grid.destroy()


class Server:
    """Owning wrapper of an fc_server (FC request serving with continuous batching).

    The grids passed in must stay alive while the server exists; the server
    keeps references to their wrappers for that reason.
    """

    def __init__(self, grids, form=FC_FORM_FP32, hbm_budget=8 << 30, host_budget=2 << 30,
                 alpha=(0.6827, 0.9, 0.95), n_bins=200, hist_hi=50.0, launch_evals=0.0,
                 policy=FC_SCHED_FAIR):
        self.grids = list(grids)
        self.alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        self.n_bins = int(n_bins)
        self.N = [fc_grid_info(g)["N"] for g in self.grids]
        handles = (_p * len(self.grids))(*[g.handle for g in self.grids])
        out = _p()
        _check(lib().fc_server_create(ctypes.byref(out), handles, len(self.grids), int(form),
                                      int(hbm_budget), int(host_budget), len(self.alpha),
                                      _hp(self.alpha), self.n_bins, float(hist_hi),
                                      float(launch_evals), int(policy)))
        self.handle = out.value
        self.K = {}

    def submit(self, grid: int, p: int, d) -> int:
        """Queue a request; d is host [K][N] FP64.  Returns the request id."""
        d = _host(d, np.float64)
        if d.ndim != 2 or d.shape[1] != self.N[grid]:
            raise ValueError("d must be [K][N] for the chosen grid")
        req = ctypes.c_int64()
        _check(lib().fc_server_submit(_p(self.handle), int(grid), int(p), int(d.shape[0]),
                                      _hp(d), ctypes.byref(req)))
        self.K[req.value] = int(d.shape[0])
        return req.value

    def submit_drawn(self, grid: int, p: int, K: int, seed: int, u_first: int = 0) -> int:
        """Queue a request whose K universes (u_first .. u_first+K-1 of point p,
        stream `seed`) are drawn on the device.  Returns the request id."""
        req = ctypes.c_int64()
        _check(lib().fc_server_submit_drawn(_p(self.handle), int(grid), int(p), int(K),
                                            int(seed) & (2**64 - 1), int(u_first),
                                            ctypes.byref(req)))
        self.K[req.value] = int(K)
        return req.value

    def poll(self, req: int, release: bool = True):
        """(state, results or None).  Results: dict of numpy arrays + latency (s)."""
        state = ctypes.c_int32()
        K = self.K[req]
        dchi2 = np.empty(K)
        cmin = np.empty(K)
        am = np.empty(K, dtype=np.int64)
        cp = np.empty(K)
        crit = np.empty(len(self.alpha))
        hist = np.empty(self.n_bins + 1, dtype=np.int64)
        lat = ctypes.c_double()
        _check(lib().fc_server_poll(_p(self.handle), int(req), ctypes.byref(state), _hp(dchi2),
                                    _hp(cmin), _hp(am), _hp(cp), _hp(crit), _hp(hist),
                                    ctypes.byref(lat), 1 if release else 0))
        if state.value != FC_REQ_DONE:
            return state.value, None
        if release:
            del self.K[req]
        return state.value, dict(dchi2=dchi2, chi2_min=cmin, argmin=am, chi2_p=cp, crit=crit,
                                 hist=hist, latency=lat.value)

    def stats(self):
        done = ctypes.c_int64()
        launches = ctypes.c_int64()
        evals = ctypes.c_double()
        used = ctypes.c_size_t()
        _check(lib().fc_server_stats(_p(self.handle), ctypes.byref(done), ctypes.byref(launches),
                                     ctypes.byref(evals), ctypes.byref(used)))
        return dict(done=done.value, launches=launches.value, evals=evals.value,
                    hbm_in_use=used.value)

    def destroy(self):
        if getattr(self, "handle", None):
            lib().fc_server_destroy(_p(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
