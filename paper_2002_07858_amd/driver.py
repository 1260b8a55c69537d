"""One call that runs the whole hot path on one grid (marshalling only).

    grid residency -> covariance factors -> scan -> critical values

Inputs are host numpy arrays (uploaded once); outputs are torch CUDA tensors.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import fc


@dataclass
class ScanOutputs:
    dchi2: "object"
    chi2_min: "object"
    argmin: "object"
    chi2_p: "object"
    crit: "object" = None
    hist: "object" = None


def alloc_outputs(K: int, device="cuda"):
    import torch
    return ScanOutputs(dchi2=torch.empty(K, dtype=torch.float64, device=device),
                       chi2_min=torch.empty(K, dtype=torch.float64, device=device),
                       argmin=torch.empty(K, dtype=torch.int64, device=device),
                       chi2_p=torch.empty(K, dtype=torch.float64, device=device))


def scan_problem(axes, S, F, d, p_idx, seg_off=None, form=fc.FC_FORM_FP32,
                 stat_mode=fc.FC_STAT_PEARSON, stat_diag=None, alpha=(0.6827, 0.9, 0.95),
                 n_bins=200, hist_hi=50.0, grid: fc.Grid | None = None, stream=None):
    """Run the hot path; returns (grid, ScanOutputs).  Reuses ``grid`` if given."""
    import torch
    if grid is None:
        grid = fc.fc_build_grid(axes, S, stream=stream)
        fc.fc_build_covariance(grid, F, stat_mode, stat_diag, forms=form, stream=stream)
    dev = torch.device("cuda")
    d_t = torch.as_tensor(np.ascontiguousarray(d, dtype=np.float64)).to(dev)
    p_t = torch.as_tensor(np.ascontiguousarray(p_idx, dtype=np.int64)).to(dev)
    out = alloc_outputs(d_t.shape[0])
    fc.fc_scan(grid, form, d_t, p_t, out.dchi2, out.chi2_min, out.argmin, out.chi2_p,
               stream=stream)
    if seg_off is not None:
        so = torch.as_tensor(np.ascontiguousarray(seg_off, dtype=np.int64)).to(dev)
        n_seg = so.numel() - 1
        out.crit = torch.empty((n_seg, len(alpha)), dtype=torch.float64, device=dev)
        out.hist = torch.empty((n_seg, n_bins + 1), dtype=torch.int64, device=dev)
        fc.fc_critical_value(so, out.dchi2, alpha, out.crit, n_bins, hist_hi, out.hist,
                             stream=stream)
    return grid, out
