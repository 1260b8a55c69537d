"""FP64 CPU oracle of the Feldman-Cousins grid scan (TEST INFRASTRUCTURE ONLY).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg import this package.  The GPU library never does, and the two share no
code: they meet only through the seeded generator in ``fcgen``.

The arithmetic lives in ``fc_oracle.c`` (plain C, FP64, no FP contraction);
this module only marshals numpy arrays through ctypes and walks very large
grids in consecutive q ranges (the running minimum carries over exactly).

Functions follow arXiv:2002.07858:
  covariance / cholesky  -- the SPD covariance whose inverse is M in Eq. (1)
  chi2                   -- Eq. (1) / Algorithm 2, as ||L^{-1}(a-b)||^2
  scan                   -- Algorithm 1 (strict-< running minimum, Delta chi^2)
  critical_value         -- Section 1 / Figure 1 (quantiles of Delta chi^2)
  data_scan / acceptance -- Section 1 (Delta chi^2 of the observed data at every
                            point, accepted where it is within the critical value)
  scan_fixed_m           -- Algorithm 1 as printed (one matrix M for the whole grid,
                            M = Sigma_p^{-1}) and its iteration (Section 2, step 5)
  region                 -- Section 2's construction for a set of true points with
                            per-point universe counts, refined near the contour
                            (the closing section's proposal)
  universes              -- Section 2, steps 1-2 (the prediction at p fluctuated:
                            Poisson counts plus correlated fractional systematics),
                            from a counter-based stream (Philox4x64-10) and
                            Hormann's PTRS Poisson sampler
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STAT_PEARSON = 0
STAT_FIXED = 1

CFLAGS = ["-O3", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-pthread"]


def build(force: bool = True) -> str:
    """Compile fc_oracle.c into liboracle.so next to it (gcc)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_p = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.fco_grid_coords.argtypes = [_i32, _p, _p, _i64, _p]
        L.fco_covariance.argtypes = [_i32, _p, _p, _i32, _p, _p]
        L.fco_cholesky.argtypes = [_i32, _p, _p]
        L.fco_chi2.argtypes = [_i32, _p, _p, _p]
        L.fco_chi2.restype = _dbl
        L.fco_factor_range.argtypes = [_i64, _i32, _p, _p, _i32, _p, _i64, _i64, _p, _p, _i32]
        L.fco_scan.argtypes = [_i64, _i32, _p, _p, _i64, _p, _p, _p, _p, _p, _p, _p, _i32]
        L.fco_scan_init.argtypes = [_i64, _p, _p, _p, _p, _p]
        L.fco_scan_range.argtypes = [_i64, _i32, _p, _i64, _i64, _p, _i64, _p, _p, _p, _p,
                                     _p, _p, _i32]
        L.fco_scan_finish.argtypes = [_i64, _p, _p, _p]
        L.fco_chi2_table.argtypes = [_i64, _i32, _p, _p, _i64, _p, _p, _i32]
        L.fco_critical_value.argtypes = [_i64, _p, _p, _i32, _p, _p, _i32, _dbl, _p]
        _u64 = ctypes.c_uint64
        L.fco_philox4x64.argtypes = [_p, _p, _p]
        L.fco_philox4x64.restype = None
        L.fco_uniform.argtypes = [_u64]
        L.fco_uniform.restype = _dbl
        L.fco_poisson.argtypes = [_dbl, _u64, _i64, _i64, _i32]
        L.fco_poisson.restype = _i64
        L.fco_normal.argtypes = [_u64, _i64, _i64, _i32]
        L.fco_normal.restype = _dbl
        L.fco_universes.argtypes = [_i64, _i32, _p, _p, _i64, _p, _p, _p, _u64, _p, _p, _i32]
        L.fco_scan_fixed_m.argtypes = [_i64, _i32, _p, _p, _i32, _p, _i64, _p, _p, _i32, _p, _p,
                                       _p, _p, _p, _p, _i32]
        for name in ("fco_grid_coords", "fco_covariance", "fco_cholesky", "fco_factor_range",
                     "fco_scan", "fco_scan_init", "fco_scan_range", "fco_scan_finish",
                     "fco_chi2_table", "fco_critical_value", "fco_universes",
                     "fco_scan_fixed_m"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def default_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    n = int(env) if env and env.isdigit() else (os.cpu_count() or 1)
    return max(1, min(n, 64))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64a(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def grid_coords(axes, q: int) -> np.ndarray:
    """Coordinates of linear grid index q (row-major, last axis fastest)."""
    lens = _i64a([len(a) for a in axes])
    vals = _f64(np.concatenate([np.asarray(a, dtype=np.float64) for a in axes]))
    out = np.zeros(len(axes))
    if lib().fco_grid_coords(len(axes), _ptr(lens), _ptr(vals), int(q), _ptr(out)) != 0:
        raise OracleError("bad grid index")
    return out


def covariance(s, F, stat_mode=STAT_PEARSON, stat_diag=None) -> np.ndarray:
    s = _f64(s)
    F = _f64(F)
    N = s.shape[0]
    sd = None if stat_diag is None else _f64(stat_diag)
    out = np.zeros((N, N))
    if lib().fco_covariance(N, _ptr(s), _ptr(F), int(stat_mode), _ptr(sd), _ptr(out)) != 0:
        raise OracleError("bad covariance arguments")
    return out


def cholesky(A) -> np.ndarray:
    A = _f64(A)
    N = A.shape[0]
    L = np.zeros((N, N))
    if lib().fco_cholesky(N, _ptr(A), _ptr(L)) != 0:
        raise OracleError("matrix is not positive definite")
    return L


def chi2(L, a, b) -> float:
    L = _f64(L)
    a = _f64(a)
    b = _f64(b)
    return float(lib().fco_chi2(L.shape[0], _ptr(L), _ptr(a), _ptr(b)))


def factor_range(S, F, stat_mode=STAT_PEARSON, stat_diag=None, q0=0, nq=None, nthreads=None):
    """Cholesky factors of Sigma_q for q in [q0, q0+nq): [nq][N][N]."""
    S = _f64(S)
    F = _f64(F)
    G, N = S.shape
    nq = G - q0 if nq is None else nq
    sd = None if stat_diag is None else _f64(stat_diag)
    L = np.empty((nq, N, N))
    bad = np.zeros(1, dtype=np.int64)
    rc = lib().fco_factor_range(G, N, _ptr(S), _ptr(F), int(stat_mode), _ptr(sd), int(q0),
                                int(nq), _ptr(L), _ptr(bad), nthreads or default_threads())
    if rc == -2:
        raise OracleError("covariance not positive definite at q=%d" % int(bad[0]))
    if rc != 0:
        raise OracleError("bad factor arguments")
    return L


def scan(S, F, d, p_idx, stat_mode=STAT_PEARSON, stat_diag=None, nthreads=None,
         block_bytes=1 << 30):
    """Algorithm 1 over every universe: returns a dict of per-universe arrays.

    Keys: dchi2, chi2_min, argmin, chi2_p, chi2_2nd.  The grid is walked in
    consecutive ranges of q so that at most ``block_bytes`` of factors exist at
    a time; the running minimum carries across ranges unchanged.
    """
    S = _f64(S)
    F = _f64(F)
    d = _f64(d)
    p_idx = _i64a(p_idx)
    G, N = S.shape
    K = d.shape[0]
    nt = nthreads or default_threads()
    out = dict(dchi2=np.empty(K), chi2_min=np.empty(K), argmin=np.empty(K, dtype=np.int64),
               chi2_p=np.empty(K), chi2_2nd=np.empty(K))
    L_ = lib()
    if L_.fco_scan_init(K, _ptr(p_idx), _ptr(out["chi2_min"]), _ptr(out["argmin"]),
                        _ptr(out["chi2_p"]), _ptr(out["chi2_2nd"])) != 0:
        raise OracleError("bad scan arguments")
    if K and (p_idx.min() < 0 or p_idx.max() >= G):
        raise OracleError("true point out of range")
    step = max(1, int(block_bytes // (8 * N * N)))
    for q0 in range(0, G, step):
        nq = min(step, G - q0)
        Lb = factor_range(S, F, stat_mode, stat_diag, q0, nq, nt)
        rc = L_.fco_scan_range(G, N, _ptr(S), q0, nq, _ptr(Lb), K, _ptr(d), _ptr(p_idx),
                               _ptr(out["chi2_min"]), _ptr(out["argmin"]), _ptr(out["chi2_p"]),
                               _ptr(out["chi2_2nd"]), nt)
        if rc != 0:
            raise OracleError("bad scan arguments")
    L_.fco_scan_finish(K, _ptr(out["chi2_p"]), _ptr(out["chi2_min"]), _ptr(out["dchi2"]))
    return out


def chi2_table(S, F, d, stat_mode=STAT_PEARSON, stat_diag=None, nthreads=None) -> np.ndarray:
    """chi^2 of every universe against every grid point: [K][G]."""
    S = _f64(S)
    d = _f64(d)
    G, N = S.shape
    K = d.shape[0]
    nt = nthreads or default_threads()
    Lall = factor_range(S, F, stat_mode, stat_diag, 0, G, nt)
    out = np.empty((K, G))
    if lib().fco_chi2_table(G, N, _ptr(S), _ptr(Lall), K, _ptr(d), _ptr(out), nt) != 0:
        raise OracleError("bad table arguments")
    return out


def data_scan(S, F, c, stat_mode=STAT_PEARSON, stat_diag=None, nthreads=None):
    """Delta chi^2 of one data vector c at every grid point (Section 1).

    chi^2(c, q) by Eq. (1) for every q, the minimum over the grid with
    Algorithm 1's tie rule (the lowest q among equal values; NaN never wins),
    and dchi2[q] = chi^2(c, q) - minimum.  Returns (dchi2 [G], chi2_min,
    argmin); with every chi^2 NaN there is no minimum: NaN, NaN and -1.
    """
    t = chi2_table(S, F, _f64(c)[None, :], stat_mode, stat_diag, nthreads)[0]
    ok = ~np.isnan(t)
    if not ok.any():
        return np.full_like(t, np.nan), float("nan"), -1
    m = float(t[ok].min())
    arg = int(np.flatnonzero(t == m)[0])
    return t - m, m, arg


def acceptance(dchi2_data, p, crit):
    """Feldman-Cousins acceptance (Section 1): true point p[k] is in the region
    when the data's Delta chi^2 there is not above its critical value crit[k].
    Points outside the grid, and NaN on either side, are not accepted."""
    dd = _f64(dchi2_data)
    p = np.asarray(p, dtype=np.int64)
    crit = _f64(crit)
    out = np.zeros(p.shape[0], dtype=np.uint8)
    for k in range(p.shape[0]):
        if 0 <= p[k] < dd.shape[0] and dd[p[k]] <= crit[k]:
            out[k] = 1
    return out


def scan_fixed_m(S, F, d, p_idx, max_iter=0, stat_mode=STAT_PEARSON, stat_diag=None,
                 nthreads=None) -> dict:
    """Algorithm 1 with one M per universe: M = Sigma_m^{-1}, m = the true point,
    re-scanned with m = q_min up to max_iter times while q_min != m."""
    S = _f64(S)
    d = _f64(d)
    p_idx = _i64a(p_idx)
    G, N = S.shape
    K = d.shape[0]
    out = {k: np.empty(K) for k in ("dchi2", "chi2_min", "chi2_p")}
    out["argmin"] = np.empty(K, dtype=np.int64)
    out["m_final"] = np.empty(K, dtype=np.int64)
    out["iters"] = np.empty(K, dtype=np.int32)
    sd = None if stat_diag is None else _f64(stat_diag)
    rc = lib().fco_scan_fixed_m(G, N, _ptr(S), _ptr(_f64(F)), int(stat_mode), _ptr(sd), K,
                                _ptr(d), _ptr(p_idx), int(max_iter), _ptr(out["dchi2"]),
                                _ptr(out["chi2_min"]), _ptr(out["argmin"]), _ptr(out["chi2_p"]),
                                _ptr(out["m_final"]), _ptr(out["iters"]),
                                nthreads or default_threads())
    if rc != 0:
        raise OracleError("bad arguments or covariance not positive definite")
    return out


def philox4x64(ctr, key) -> list:
    """Philox4x64-10 block for a 4-word counter and 2-word key."""
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().fco_philox4x64(_ptr(c), _ptr(k), _ptr(out))
    return [int(x) for x in out]


def uniform(w: int) -> float:
    return float(lib().fco_uniform(int(w)))


def poisson(lam: float, seed: int, p: int, j: int, i: int) -> int:
    """Poisson draw for (true point p, universe j, bin i); -1 for an invalid mean."""
    return int(lib().fco_poisson(float(lam), int(seed), int(p), int(j), int(i)))


def normal(seed: int, p: int, j: int, i: int) -> float:
    return float(lib().fco_normal(int(seed), int(p), int(j), int(i)))


def universes(S, F, p, seg_off, seed, u_first=None, nthreads=None):
    """Universes of true points p[k] into rows seg_off[k]..seg_off[k+1]-1.

    d_i = Poisson(S_p[i]) + S_p[i] * (chol(F) g)_i; returns (d [K][N],
    counts [K][N] int32).
    """
    S = _f64(S)
    G, N = S.shape
    LF = cholesky(F)
    p = _i64a(p)
    seg_off = _i64a(seg_off)
    uf = None if u_first is None else _i64a(u_first)
    K = int(seg_off[-1]) if seg_off.shape[0] else 0
    d = np.empty((K, N))
    counts = np.empty((K, N), dtype=np.int32)
    rc = lib().fco_universes(G, N, _ptr(S), _ptr(_f64(LF)), p.shape[0], _ptr(p), _ptr(seg_off),
                             _ptr(uf), int(seed), _ptr(d), _ptr(counts),
                             nthreads or default_threads())
    if rc != 0:
        raise OracleError("bad universe arguments")
    return d, counts


def region(S, F, pts, K0, K_max, z, seed, alpha, dchi2_data, stat_mode=STAT_PEARSON,
           stat_diag=None, nthreads=None):
    """Feldman-Cousins region over true points pts with per-point universe counts.

    Section 2 builds each point's Delta chi^2 distribution from universes drawn
    at it; the closing section proposes spending universes only near the
    contour.  Rounds: every point starts with universes 0..K0-1; after each
    round a point's critical values are x_(j), j = ceil(alpha K), over its K
    values, and its band is [x_(j - delta), x_(j + delta)] with delta =
    ceil(z sqrt(K alpha (1 - alpha))) (ranks clamped to [1, K]); a point whose
    data value dchi2_data[p] falls inside a band, and has K < K_max, draws
    universes K..2K-1 (at most K_max) for the next round.  Returns crit
    [n][n_alpha], accepted [n][n_alpha] (dchi2_data[p] <= crit), K_used,
    rounds and evals (universe x grid-point evaluations).
    """
    S = _f64(S)
    G = S.shape[0]
    pts = _i64a(pts)
    n = pts.shape[0]
    alpha = _f64(np.atleast_1d(alpha))
    dd = _f64(dchi2_data)[pts]
    vals = [np.empty(0) for _ in range(n)]
    K = np.zeros(n, dtype=np.int64)
    K_new = np.full(n, K0, dtype=np.int64)
    crit = np.full((n, alpha.shape[0]), np.nan)
    rounds, evals = 0, 0.0
    while True:
        act = np.flatnonzero(K_new > K)
        if act.shape[0] == 0:
            break
        rounds += 1
        seg = np.concatenate([[0], np.cumsum(K_new[act] - K[act])]).astype(np.int64)
        d, _ = universes(S, F, pts[act], seg, seed, u_first=K[act], nthreads=nthreads)
        r = scan(S, F, d, np.repeat(pts[act], np.diff(seg)), stat_mode, stat_diag, nthreads)
        for i, k in enumerate(act):
            vals[k] = np.concatenate([vals[k], r["dchi2"][seg[i]:seg[i + 1]]])
        evals += float(seg[-1]) * G
        K = K_new.copy()
        off = np.concatenate([[0], np.cumsum(K)]).astype(np.int64)
        crit, _ = critical_value(np.concatenate(vals), off, alpha, with_hist=False)
        for k in range(n):
            xs = np.sort(vals[k])                       # NaN last
            undecided = False
            for a in range(alpha.shape[0]):
                j = min(max(int(math.ceil(alpha[a] * K[k])), 1), int(K[k]))
                delta = int(math.ceil(z * math.sqrt(K[k] * alpha[a] * (1.0 - alpha[a]))))
                lo_r, hi_r = max(1, j - delta), min(int(K[k]), j + delta)
                if xs[lo_r - 1] <= dd[k] <= xs[hi_r - 1]:
                    undecided = True
            if undecided and K[k] < K_max:
                K_new[k] = min(2 * K[k], K_max)
    accepted = (dd[:, None] <= crit).astype(np.uint8)
    return dict(crit=crit, accepted=accepted, K_used=K, rounds=rounds, evals=evals)


def critical_value(x, seg_off, alpha, n_bins=200, hist_hi=50.0, with_hist=True):
    """Per-segment type-1 quantiles crit[n_seg][n_alpha] and histograms [n_seg][n_bins+1]."""
    x = _f64(x)
    seg_off = _i64a(seg_off)
    alpha = _f64(np.atleast_1d(alpha))
    n_seg = seg_off.shape[0] - 1
    crit = np.empty((n_seg, alpha.shape[0]))
    hist = np.empty((n_seg, n_bins + 1), dtype=np.int64) if with_hist else None
    rc = lib().fco_critical_value(n_seg, _ptr(seg_off), _ptr(x), alpha.shape[0], _ptr(alpha),
                                  _ptr(crit), int(n_bins), float(hist_hi), _ptr(hist))
    if rc != 0:
        raise OracleError("bad critical-value arguments")
    return crit, hist
