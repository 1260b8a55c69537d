"""Seeded synthetic inputs for the Feldman-Cousins grid scan.

This module is the one input generator shared by the FP64 oracle and the GPU
library.  It holds none of the scan's arithmetic (no covariance, no chi^2, no
minimum): it only draws a toy oscillation model, evaluates the signal table
S(q) on a rectangular grid, picks true points and fluctuates universes.

The paper's own inputs (SBN ROOT histograms and covariance matrices) are not
available, so a short-baseline toy model stands in for them:

* three detectors at baselines L = 0.11, 0.47, 0.60 km, with uniform energy
  bins on [0.2, 3.0] GeV (bin centre E_i);
* background per bin ~ LogNormal(ln 300, 0.5), flux per bin ~ LogNormal(ln 50, 0.3);
* fractional systematic covariance F = diag(sigma) C diag(sigma) with
  sigma_i ~ U(0.05, 0.20) and C the correlation matrix of a Wishart draw
  W = A A^T, A an N x 2N standard normal matrix;
* appearance signal S_i = bkg_i + flux_i * sin^2(2theta) * sin^2(1.27 dm2 L_i / E_i),
  with optional disappearance factor (D = 3) and normalisation / energy-scale
  nuisance axes (D = 5);
* universes d = Poisson(S(p)) + diag(S(p)) chol(F) g with g ~ N(0, I), which
  has covariance diag(S(p)) + F o S(p)S(p)^T, the Pearson statistical plus
  fractional systematic covariance at the true point.  No clamping.

Every random stream comes from ``numpy.random.SeedSequence(20020785,
spawn_key=(config, stream, index))`` with stream 0 = model parameters,
1 = true-point choice, 2 = universes of true point ``index``,
3 = serving arrivals.  The universes of one true point therefore do not depend
on how many other points or requests are generated.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 20020785
BASELINES_KM = (0.11, 0.47, 0.60)
E_LO, E_HI = 0.2, 3.0

STAT_PEARSON = 0
STAT_FIXED = 1


def rng_for(config: int, stream: int, index: int = 0) -> np.random.Generator:
    """PCG64 generator for one (config, stream, index) triple."""
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(int(config), int(stream), int(index)))
    return np.random.Generator(np.random.PCG64(ss))


@dataclass
class ToyModel:
    bins_per_det: tuple
    L: np.ndarray       # [N] baseline of each bin's detector (km)
    E: np.ndarray       # [N] bin-centre energy (GeV)
    bkg: np.ndarray     # [N]
    flux: np.ndarray    # [N]
    sigma: np.ndarray   # [N] fractional systematic per bin
    C: np.ndarray       # [N][N] correlation
    F: np.ndarray       # [N][N] fractional systematic covariance

    @property
    def N(self) -> int:
        return int(self.bkg.shape[0])


def toy_model(config: int, bins_per_det=(19, 19, 19)) -> ToyModel:
    """Draw the model parameters of one configuration (stream 0)."""
    rng = rng_for(config, 0, 0)
    Ls, Es = [], []
    for L, nb in zip(BASELINES_KM, bins_per_det):
        edges = np.linspace(E_LO, E_HI, nb + 1)
        Es.append(0.5 * (edges[:-1] + edges[1:]))
        Ls.append(np.full(nb, L))
    L = np.concatenate(Ls)
    E = np.concatenate(Es)
    N = L.shape[0]
    bkg = rng.lognormal(mean=math.log(300.0), sigma=0.5, size=N)
    flux = rng.lognormal(mean=math.log(50.0), sigma=0.3, size=N)
    sigma = rng.uniform(0.05, 0.20, size=N)
    A = rng.standard_normal((N, 2 * N))
    W = A @ A.T
    W = 0.5 * (W + W.T)          # exactly symmetric
    dw = np.sqrt(np.diag(W))
    C = W / np.outer(dw, dw)
    np.fill_diagonal(C, 1.0)
    F = C * np.outer(sigma, sigma)
    return ToyModel(tuple(bins_per_det), L, E, bkg, flux, sigma, C, F)


def axis_points(lo: float, hi: float, n: int, log10: bool = False) -> np.ndarray:
    """Inclusive linspace (in log10 space when asked; values are returned as log10)."""
    return np.linspace(lo, hi, n)


def grid_points(axes) -> np.ndarray:
    """All grid points as a [G][D] array, row-major with the last axis fastest."""
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def signal_table(model: ToyModel, axes, kind: str) -> np.ndarray:
    """Evaluate the toy signal S(q) for every grid point q: returns [G][N] float64.

    kind = "app2": axes (log10 dm2, log10 sin^2 2theta)
    kind = "app3": adds log10 |U_mu4|^2 (disappearance factor folded into the flux)
    kind = "app5": app3 plus normalisation n and energy scale e
    """
    P = grid_points(axes)
    dm2 = 10.0 ** P[:, 0:1]
    s22t = 10.0 ** P[:, 1:2]
    if kind == "app2":
        phase = 1.27 * dm2 * model.L[None, :] / model.E[None, :]
        s2 = np.sin(phase) ** 2
        return model.bkg[None, :] + model.flux[None, :] * s22t * s2
    u = 10.0 ** P[:, 2:3]
    if kind == "app3":
        phase = 1.27 * dm2 * model.L[None, :] / model.E[None, :]
        s2 = np.sin(phase) ** 2
        surv = 1.0 - 4.0 * u * (1.0 - u) * s2
        return model.bkg[None, :] + model.flux[None, :] * surv * s22t * s2
    if kind == "app5":
        n = P[:, 3:4]
        e = P[:, 4:5]
        phase = 1.27 * dm2 * model.L[None, :] / (e * model.E[None, :])
        s2 = np.sin(phase) ** 2
        surv = 1.0 - 4.0 * u * (1.0 - u) * s2
        return n * (model.bkg[None, :] + model.flux[None, :] * surv * s22t * s2)
    raise ValueError(kind)


def true_points(config: int, G: int, n_true: int) -> np.ndarray:
    """n_true distinct grid indices, sorted ascending (stream 1)."""
    rng = rng_for(config, 1, 0)
    return np.sort(rng.choice(G, size=n_true, replace=False)).astype(np.int64)


def universes(config: int, j: int, s_p: np.ndarray, F: np.ndarray, K: int) -> np.ndarray:
    """K universes around the prediction s_p (stream 2, index j): [K][N] float64.

    d = Poisson(s_p) + diag(s_p) chol(F) g.  All Poisson draws come first, then
    all normal draws.
    """
    rng = rng_for(config, 2, j)
    N = s_p.shape[0]
    pois = rng.poisson(s_p, size=(K, N)).astype(np.float64)
    g = rng.standard_normal((K, N))
    LF = np.linalg.cholesky(F)
    return pois + (g @ LF.T) * s_p[None, :]


@dataclass
class Problem:
    """One complete scan problem: grid, signal, covariance recipe and universes."""
    name: str
    config: int
    axes: list                 # D arrays of axis values
    S: np.ndarray              # [G][N] float64
    F: np.ndarray              # [N][N] float64
    stat_mode: int
    stat_diag: np.ndarray | None
    true_pts: np.ndarray       # [P] int64 grid indices
    seg_off: np.ndarray        # [P+1] int64 universe offsets per true point
    d: np.ndarray              # [K_tot][N] float64
    p_idx: np.ndarray          # [K_tot] int64
    central: np.ndarray | None = None
    alpha: tuple = (0.6827, 0.9, 0.95)
    meta: dict = field(default_factory=dict)

    @property
    def G(self) -> int:
        return int(self.S.shape[0])

    @property
    def N(self) -> int:
        return int(self.S.shape[1])

    @property
    def D(self) -> int:
        return len(self.axes)

    @property
    def K(self) -> int:
        return int(self.d.shape[0])


# Configurations: (config id, grid kind, axis specs, bins per detector, true points, K per point)
_AX_DM2 = (-2.0, 2.0)
_AX_S22T = (-4.0, 0.0)
_AX_U = (-4.0, 0.0)
_AX_NORM = (0.8, 1.2)
_AX_ESCALE = (0.95, 1.05)

CONFIGS = {
    # small FP64 case: D=2 20x20, N=38, one true point x 1000 universes
    "c1": dict(config=1, kind="app2", n=(20, 20), bins=(12, 12, 14), n_true=1, K=1000),
    # FP32 scan: D=2 100x100, N=57, 256 true points x 2000 universes
    "c2": dict(config=2, kind="app2", n=(100, 100), bins=(19, 19, 19), n_true=256, K=2000),
    # split precision: D=3 60^3, N=57, 64 true points x 4000 universes
    "c3": dict(config=3, kind="app3", n=(60, 60, 60), bins=(19, 19, 19), n_true=64, K=4000),
    # large grid: D=5 16^5, N=57, 16 true points x 10000 universes
    "c5": dict(config=5, kind="app5", n=(16, 16, 16, 16, 16), bins=(19, 19, 19), n_true=16, K=10000),
}


def _axes_for(kind: str, n) -> list:
    specs = [_AX_DM2, _AX_S22T]
    if kind in ("app3", "app5"):
        specs.append(_AX_U)
    if kind == "app5":
        specs += [_AX_NORM, _AX_ESCALE]
    return [axis_points(lo, hi, k) for (lo, hi), k in zip(specs, n)]


def make_problem(name: str, n_true: int | None = None, K: int | None = None,
                 n_axis=None, true_subset=None) -> Problem:
    """Build one named configuration.

    ``n_true`` / ``K`` / ``n_axis`` override the configuration's sizes (smaller
    cases for tests); ``true_subset`` keeps only those positions of the
    configuration's true-point list (their universes are unchanged, because each
    point has its own stream).
    """
    spec = CONFIGS[name]
    c = spec["config"]
    model = toy_model(c, spec["bins"])
    axes = _axes_for(spec["kind"], n_axis or spec["n"])
    S = signal_table(model, axes, spec["kind"])
    G = S.shape[0]
    nt = spec["n_true"] if n_true is None else n_true
    Kp = spec["K"] if K is None else K
    tp = true_points(c, G, spec["n_true"] if n_true is None else nt)
    idx = np.arange(tp.shape[0]) if true_subset is None else np.asarray(true_subset)
    ds, ps, off = [], [], [0]
    for j in idx:
        p = int(tp[j])
        ds.append(universes(c, int(j), S[p], model.F, Kp))
        ps.append(np.full(Kp, p, dtype=np.int64))
        off.append(off[-1] + Kp)
    d = np.concatenate(ds, axis=0) if ds else np.zeros((0, S.shape[1]))
    p_idx = np.concatenate(ps) if ps else np.zeros(0, dtype=np.int64)
    return Problem(name=name, config=c, axes=axes, S=S, F=model.F,
                   stat_mode=STAT_PEARSON, stat_diag=None,
                   true_pts=tp[idx].astype(np.int64),
                   seg_off=np.asarray(off, dtype=np.int64), d=np.ascontiguousarray(d),
                   p_idx=p_idx, central=None,
                   meta=dict(kind=spec["kind"], bins=spec["bins"], K_per_point=Kp))


def serving_requests(n_req: int, grid_sizes, rate_hz: float, k_lo=500, k_hi=20000):
    """Seeded request stream (stream 3): arrival times, grid choice, K per request.

    Arrivals are Poisson at ``rate_hz``; the grid is uniform over ``grid_sizes``
    (a list of G per resident grid), the true point uniform on that grid, and
    K = floor(exp(U(ln k_lo, ln k_hi))).
    """
    rng = rng_for(4, 3, 0)
    gaps = rng.exponential(1.0 / rate_hz, size=n_req)
    t = np.cumsum(gaps)
    gsel = rng.integers(0, len(grid_sizes), size=n_req)
    p = np.array([rng.integers(0, grid_sizes[g]) for g in gsel], dtype=np.int64)
    K = np.floor(np.exp(rng.uniform(math.log(k_lo), math.log(k_hi), size=n_req))).astype(np.int64)
    return t, gsel, p, K
