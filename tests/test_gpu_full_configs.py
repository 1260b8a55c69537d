"""Full-size configurations on the GPU, checked against the FP64 oracle's
values for a sample of universes (written by tests/golden/
make_full_config_golden.py, which calls only the oracle) and on properties
that hold at any size, in the launch configuration the benchmark times.

c2: D=2 100^2 (10 000 points), N=57, 256 true points x 2000 universes: every
    universe of 4 true points, and the full-K critical values and histograms
    of all 256 true points (the oracle ran on every universe).
c3: D=3 60^3 (216 000 points), N=57, 64 true points x 4000 universes: the
    first 64 universes of every true point plus all 4000 of 2 true points
    (full-K critical values).
c5: D=5 16^5 (1 048 576 points), N=57, 16 true points x 10 000 universes: the
    first 16 universes of every true point.
Every form (FP64, FP32 through both entries, split BF16 and FP16) runs on the
same inputs.  Per form: the invariants on every universe (all finite: no NaN
data, every true point on the grid), e_rel within the form's tolerance,
argmin agreement on universes that are not near-ties (100 % for FP64 and
FP32), the argmin's validity on every sampled universe (near-ties included),
and the critical values of the full points within the Lipschitz bound of
the Delta chi^2 error.
"""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest

import fcgen
import parity

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_full_config_golden as golden  # noqa: E402

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FORM = {"fp64": 1, "fp32": 2, "split_bf16": 4, "split_fp16": 8}
ALPHA = (0.6827, 0.9, 0.95)


@pytest.fixture(scope="module")
def fc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_07858_amd as fc
    fc.lib()
    return fc


def scan_all(fc, pr):
    """Every form through fc_scan_points (the benchmark's entry) and the FP32
    form also through fc_scan; critical values of every segment."""
    grid = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(grid, pr.F, pr.stat_mode, pr.stat_diag, forms=1 | 2 | 4 | 8)
    K = pr.K
    d_t = torch.as_tensor(pr.d).cuda()
    p_t = torch.as_tensor(pr.p_idx).cuda()
    pts = torch.as_tensor(pr.p_idx[pr.seg_off[:-1]]).cuda()
    seg = torch.as_tensor(pr.seg_off).cuda()
    n_seg = len(pr.seg_off) - 1
    outs = {}
    for name in list(FORM) + ["fp32_universes"]:
        form = FORM[name.replace("_universes", "")]
        o = {k: torch.empty(K, dtype=torch.float64, device="cuda")
             for k in ("dchi2", "chi2_min", "chi2_p")}
        o["argmin"] = torch.empty(K, dtype=torch.int64, device="cuda")
        if name.endswith("_universes"):
            fc.fc_scan(grid, form, d_t, p_t, o["dchi2"], o["chi2_min"], o["argmin"],
                       o["chi2_p"])
        else:
            fc.fc_scan_points(grid, form, pts, seg, d_t, o["dchi2"], o["chi2_min"], o["argmin"],
                              o["chi2_p"])
        crit = torch.empty((n_seg, len(ALPHA)), dtype=torch.float64, device="cuda")
        fc.fc_critical_value(seg, o["dchi2"], ALPHA, crit)
        torch.cuda.synchronize()
        outs[name] = {k: v.cpu().numpy() for k, v in o.items()}
        outs[name]["crit"] = crit.cpu().numpy()
    grid.destroy()
    return outs


@pytest.fixture(scope="module", params=["c2", "c3", "c5"])
def config(fc, request):
    name = request.param
    pr = fcgen.make_problem(name)
    ref = golden.load(name, pr)
    print(f"\n[config] {name}: G={pr.G} K={pr.K}, {ref['idx'].shape[0]} sampled universes",
          flush=True)
    return name, pr, ref, scan_all(fc, pr)


@pytest.mark.parametrize("form", list(FORM) + ["fp32_universes"])
def test_full_config_parity(config, form):
    name, pr, ref, outs = config
    dev = outs[form]
    tol = parity.TOL[form.replace("_universes", "")]
    parity.check_invariants(dev, pr.G, all_finite=True)
    idx = ref["idx"]
    ds = {k: dev[k][idx] for k in ("dchi2", "chi2_min", "argmin", "chi2_p")}
    rep = parity.report(ds, ref, tol)
    rep.update(parity.argmin_validity(pr, ds, pr.d[idx], ref, tol))
    print(name, form, rep)
    assert rep["e_rel"] <= tol, rep
    assert rep["argmin_agree"] >= (1.0 if form in ("fp64", "fp32", "fp32_universes") else 0.99)
    assert rep["argmin_valid"] == 1.0, rep
    # full-K critical values of the points whose universes are all sampled
    # (P10: an order statistic moves by at most the largest value error)
    for j, s in enumerate(ref["full_points"]):
        lo, hi = int(pr.seg_off[s]), int(pr.seg_off[s + 1])
        bound = tol * max(1.0, float(dev["chi2_p"][lo:hi].max()))
        err = np.abs(dev["crit"][s] - ref["crit"][j])
        assert np.all(err <= bound), (name, form, int(s), err, bound)
    if "crit_all" in ref:
        # every true point's critical values (the oracle's full run)
        for s in range(len(pr.seg_off) - 1):
            lo, hi = int(pr.seg_off[s]), int(pr.seg_off[s + 1])
            bound = tol * max(1.0, float(dev["chi2_p"][lo:hi].max()))
            err = np.abs(dev["crit"][s] - ref["crit_all"][s])
            assert np.all(err <= bound), (name, form, s, err, bound)


def test_forms_agree_on_every_universe(config):
    """All universes: every form against the FP64 form on the same inputs."""
    name, pr, ref, outs = config
    base = outs["fp64"]
    scale = np.maximum(1.0, base["chi2_p"])
    for form, dev in outs.items():
        tol = parity.TOL[form.replace("_universes", "")]
        e = np.abs(dev["dchi2"] - base["dchi2"]) / scale
        assert e.max() <= tol + parity.TOL["fp64"], (name, form, e.max())
