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
"""
from __future__ import annotations

import numpy as np

TOL = {"fp64": 1e-11, "fp32": 1e-6, "split_bf16": 1e-4, "split_fp16": 1e-4}


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


def check_invariants(dev: dict, G: int):
    """Properties that hold for any correct scan at any size."""
    dchi2, cmin, cp, am = dev["dchi2"], dev["chi2_min"], dev["chi2_p"], dev["argmin"]
    fin = np.isfinite(cp)
    assert np.all(cmin[fin] >= 0.0)
    assert np.all(dchi2[fin] >= 0.0), "Delta chi^2 < 0"
    assert np.all(cmin[fin] <= cp[fin]), "minimum above the true point's chi^2"
    assert np.all(dchi2[fin] == cp[fin] - cmin[fin])
    assert np.all((am >= 0) & (am < G))
