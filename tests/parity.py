"""Parity report of a device scan against the FP64 oracle (test helper).

e_rel  = max_k |dchi2_dev - dchi2_64| / max(1, chi2_p_64)
         (Delta chi^2 is a difference of two chi^2 values of size ~N, so its
         attainable precision scales with chi^2 at the true point)
argmin agreement is counted over universes that are not near-ties:
         universe k is a near-tie if (chi2_2nd - chi2_min) / max(1, chi2_min) <= tau
         with chi2_2nd the smallest chi^2 at a grid point other than the
         oracle's argmin.  tau is twice the form's tolerance: two chi^2
         values within 2 tol of each other can swap order under per-value
         errors <= tol.
argmin validity covers every compared universe, near-ties included: the
         oracle evaluates Eq. (1) at the device's argmin q_dev, and q_dev is
         valid when that value is a minimum up to the form's error,
             chi2_64(d, q_dev) <= chi2_min_64 + 2 tol max(1, chi2_min_64),
         and the device's reported minimum is chi2 at q_dev up to it,
             |chi2_64(d, q_dev) - chi2_min_dev| <= tol max(1, chi2_p_64).
         (A wrong q packed beside a correct chi^2 fails the second test; a
         q that is not a minimiser fails the first.)
"""
from __future__ import annotations

import numpy as np

TOL = {"fp64": 1e-11, "fp32": 1e-6, "split_bf16": 1e-4, "split_fp16": 1e-4}


def split_bf16_tol(S, d, p) -> float:
    """The split-BF16 form's error bound on a given input.

    The split forms contract z = W_q (d - o) - W_q (S_q - o) with o the grid's
    mean signal per bin, so their products see d - o, not d - S_q.  A BF16
    hi + lo pair carries x to 2^-18 |x|, and each of the three products
    hi*hi + hi*lo + lo*hi of W_ij x_j is off by at most about 3 * 2^-18
    |W_ij x_j|; with R = max_j |d_j - o_j| / sqrt(S_p,j), the universe's
    reach from the offset in its own standard deviations, a row of z is off
    by a few 2^-18 R, and chi^2 = |z|^2 by about 2^-14 R relative to
    max(1, chi^2_p) (a few 2^-16 R sqrt(N) absolute against chi^2 ~ N).
    The 1e-4 target holds while R stays within about 15 (the c1-c5
    configurations: R <= 25 and N >= 38, measured 2e-5); few bins on a wide
    grid reach 1e-4 to 4e-4 (FP16, with 5 more bits in each half, stays
    below 1e-5 on the same inputs)."""
    S = np.asarray(S, dtype=np.float64)
    o = S.mean(axis=0)
    R = float(np.max(np.abs(np.asarray(d) - o) / np.sqrt(S[np.asarray(p)])))
    return max(TOL["split_bf16"], 2.0 ** -14 * R)


def report(dev: dict, ref: dict, tol: float) -> dict:
    scale = np.maximum(1.0, ref["chi2_p"])
    e_abs = np.abs(dev["dchi2"] - ref["dchi2"])
    e_rel = e_abs / scale
    big = ref["dchi2"] >= 1.0
    tau = 2.0 * tol
    gap = (ref["chi2_2nd"] - ref["chi2_min"]) / np.maximum(1.0, ref["chi2_min"])
    clear = gap > tau
    agree = dev["argmin"][clear] == ref["argmin"][clear]
    return dict(
        n=int(ref["dchi2"].shape[0]),
        e_abs=float(e_abs.max()) if e_abs.size else 0.0,
        e_rel=float(e_rel.max()) if e_rel.size else 0.0,
        e_rel_vs_dchi2_ge1=float((e_abs[big] / ref["dchi2"][big]).max()) if big.any() else 0.0,
        chi2_min_rel=float((np.abs(dev["chi2_min"] - ref["chi2_min"]) /
                            np.maximum(1.0, ref["chi2_min"])).max()) if e_abs.size else 0.0,
        chi2_p_rel=float((np.abs(dev["chi2_p"] - ref["chi2_p"]) / scale).max())
        if e_abs.size else 0.0,
        argmin_agree=float(agree.mean()) if agree.size else 1.0,
        near_tie_frac=float(1.0 - clear.mean()) if clear.size else 0.0,
    )


def chi2_at(pr, d, q):
    """The oracle's chi^2 (Eq. (1), FP64) of universes d[k] at grid points q[k]."""
    import oracle
    d = np.asarray(d, dtype=np.float64)
    q = np.asarray(q, dtype=np.int64)
    out = np.empty(q.shape[0])
    for qq in np.unique(q):
        L = oracle.factor_range(pr.S, pr.F, pr.stat_mode, pr.stat_diag, int(qq), 1)[0]
        for k in np.flatnonzero(q == qq):
            out[k] = oracle.chi2(L, d[k], pr.S[qq])
    return out


def argmin_validity(pr, dev: dict, d, ref: dict, tol: float) -> dict:
    """Validity of the device's argmin on every compared universe (see above).
    Universes whose oracle minimum is not finite (no chi^2 < +inf) are left
    to the invariants and the NaN tests."""
    fin = np.isfinite(ref["chi2_min"])
    am = np.asarray(dev["argmin"])
    ok_range = (am >= 0) & (am < pr.G)
    sel = np.flatnonzero(fin & ok_range)
    c_at = np.full(am.shape[0], np.nan)
    if sel.size:
        c_at[sel] = chi2_at(pr, np.asarray(d)[sel], am[sel])
    cmin = ref["chi2_min"]
    gap = (c_at - cmin) / np.maximum(1.0, cmin)
    val_err = np.abs(c_at - dev["chi2_min"]) / np.maximum(1.0, ref["chi2_p"])
    valid = fin & ok_range & (gap <= 2.0 * tol) & (val_err <= tol)
    n = int(fin.sum())
    return dict(argmin_valid=float(valid[fin].mean()) if n else 1.0,
                argmin_invalid=int(n - valid[fin].sum()),
                argmin_gap_max=float(np.nanmax(gap[fin])) if n else 0.0,
                chi2_min_at_argmin_err=float(np.nanmax(val_err[fin])) if n else 0.0)


def check_invariants(dev: dict, G: int, all_finite: bool = False):
    """Properties that hold for any correct scan at any size.  With
    all_finite, every universe must have a finite Delta chi^2 (inputs with no
    NaN data and every true point on the grid)."""
    dchi2, cmin, cp, am = dev["dchi2"], dev["chi2_min"], dev["chi2_p"], dev["argmin"]
    if all_finite:
        assert np.all(np.isfinite(dchi2)), "non-finite Delta chi^2"
        assert np.all(np.isfinite(cmin)) and np.all(np.isfinite(cp))
    fin = np.isfinite(cp)
    assert np.all(cmin[fin] >= 0.0)
    assert np.all(dchi2[fin] >= 0.0), "Delta chi^2 < 0"
    assert np.all(cmin[fin] <= cp[fin]), "minimum above the true point's chi^2"
    assert np.all(dchi2[fin] == cp[fin] - cmin[fin])
    assert np.all((am >= 0) & (am < G))
