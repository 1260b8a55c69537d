"""GPU Feldman-Cousins region with per-point universe counts (fc_region)
against the oracle's region on the same seeded inputs.

The device draws universes with its own generator, scans them, takes the
critical values and bands with its own order-statistic kernel and makes the
refinement decisions; the oracle does every step on the CPU.  In FP64 the
decisions (universe counts, rounds) must agree exactly and the critical
values to the FP64 tolerance; in FP32 a decision may differ only where the
data value sits within the FP32 error of a band edge or critical value.
"""
from __future__ import annotations

import numpy as np
import pytest

import fcgen
import oracle
import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ALPHA = (0.6827, 0.9)


@pytest.fixture(scope="module")
def fc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_07858_amd as fc
    fc.lib()
    return fc


def setup(fc, name, n_axis, forms, data_point, data_j):
    pr = fcgen.make_problem(name, K=1, true_subset=[0], n_axis=n_axis)
    c = fcgen.universes(pr.config, data_j, pr.S[data_point], pr.F, 1)[0]
    g = fc.fc_build_grid(pr.axes, pr.S, central=c)
    fc.fc_build_covariance(g, pr.F, forms=forms | fc.FC_FORM_FP64)   # FP64: the data scan
    dd = torch.empty(pr.G, dtype=torch.float64, device="cuda")
    fc.fc_data_scan(g, dd)
    return pr, g, dd


def run_region(fc, g, form, dd, n_pts, pts, K0, K_max, z, seed):
    crit = torch.full((n_pts, len(ALPHA)), -7.0, dtype=torch.float64, device="cuda")
    acc = torch.full((n_pts, len(ALPHA)), 7, dtype=torch.uint8, device="cuda")
    info = fc.fc_region(g, form, dd, crit, acc, pts=pts, K0=K0, K_max=K_max, z=z, seed=seed,
                        alpha=ALPHA)
    return crit.cpu().numpy(), acc.cpu().numpy(), info


def test_region_fp64_matches_oracle(fc):
    pr, g, dd = setup(fc, "c1", (12, 12), fc.FC_FORM_FP64 | fc.FC_FORM_FP32, 70, 40000)
    crit, acc, info = run_region(fc, g, fc.FC_FORM_FP64, dd, pr.G, None, 32, 512, 2.0, 7)
    dd_h = dd.cpu().numpy()
    g.destroy()
    ref = oracle.region(pr.S, pr.F, np.arange(pr.G), 32, 512, 2.0, 7, ALPHA, dd_h)
    np.testing.assert_array_equal(info["K_used"], ref["K_used"])
    assert info["rounds"] == ref["rounds"] and info["evals"] == ref["evals"]
    assert np.all(np.abs(crit - ref["crit"]) <= parity.TOL["fp64"] * np.maximum(1.0, ref["crit"]))
    np.testing.assert_array_equal(acc, ref["accepted"])
    # the refinement did something: several counts, a region that is not everything
    assert len(np.unique(info["K_used"])) >= 3
    assert 0 < acc[:, 0].sum() < pr.G


def test_region_subset_fp32_and_invariants(fc):
    pr, g, dd = setup(fc, "c2", (30, 30), fc.FC_FORM_FP32, 400, 40001)
    pts = np.array([3, 100, 399, 400, 401, 455, 777, 899])
    crit, acc, info = run_region(fc, g, fc.FC_FORM_FP32, dd, len(pts), pts, 64, 1024, 2.0, 11)
    dd_h = dd.cpu().numpy()
    g.destroy()
    ref = oracle.region(pr.S, pr.F, pts, 64, 1024, 2.0, 11, ALPHA, dd_h)
    K = info["K_used"]
    assert np.all(np.isin(K, [64, 128, 256, 512, 1024]))
    np.testing.assert_array_equal(acc, (dd_h[pts][:, None] <= crit).astype(np.uint8))
    same = K == ref["K_used"]
    # a count may differ only where the data value is within FP32 error of an
    # order statistic of the oracle's values
    near = np.any(np.abs(dd_h[pts][:, None] - ref["crit"]) <= 1e-4 * np.maximum(1.0, ref["crit"]),
                  axis=1)
    assert np.all(same | near)
    ok = same[:, None] & (np.abs(dd_h[pts][:, None] - ref["crit"]) > 1e-4)
    assert np.all((acc == ref["accepted"]) | ~ok)
    scale = np.maximum(1.0, np.abs(ref["crit"]))
    assert np.all((np.abs(crit - ref["crit"]) <= 1e-5 * scale) | ~same[:, None])


def test_region_errors(fc):
    pr, g, dd = setup(fc, "c1", (6, 6), fc.FC_FORM_FP32, 3, 40002)
    # outputs large enough for every alpha list below, so that each call
    # reaches the library's own argument checks
    crit = torch.empty((pr.G, 5), dtype=torch.float64, device="cuda")
    acc = torch.empty((pr.G, 5), dtype=torch.uint8, device="cuda")
    for kw in (dict(K0=0), dict(K0=64, K_max=32), dict(z=-1.0), dict(pts=[pr.G]),
               dict(alpha=(0.1, 0.2, 0.3, 0.4, 0.5))):
        args = dict(K0=16, K_max=64, z=2.0)
        args.update(kw)
        with pytest.raises(fc.FCError):
            fc.fc_region(g, fc.FC_FORM_FP32, dd, crit, acc, **args)
    with pytest.raises(fc.FCError) as ei:              # form not built
        fc.fc_region(g, fc.FC_FORM_SPLIT_BF16, dd, crit, acc, K0=16, K_max=64)
    assert ei.value.code == fc.FC_ERR_STATE
    g.destroy()


def test_region_split_fp16_matches_oracle_up_to_near_ties(fc):
    """The region in the split-FP16 form: counts, critical values and
    acceptance agree with the oracle except where the data value lies within
    the form's error of an order statistic."""
    pr, g, dd = setup(fc, "c1", (10, 10), fc.FC_FORM_SPLIT_FP16, 33, 40003)
    crit, acc, info = run_region(fc, g, fc.FC_FORM_SPLIT_FP16, dd, pr.G, None, 32, 256, 2.0, 13)
    dd_h = dd.cpu().numpy()
    g.destroy()
    ref = oracle.region(pr.S, pr.F, np.arange(pr.G), 32, 256, 2.0, 13, ALPHA, dd_h)
    same = info["K_used"] == ref["K_used"]
    near = np.any(np.abs(dd_h[:, None] - ref["crit"]) <= 1e-2 * np.maximum(1.0, ref["crit"]),
                  axis=1)
    assert np.all(same | near)
    assert same.mean() >= 0.9
    np.testing.assert_array_equal(acc, (dd_h[:, None] <= crit).astype(np.uint8))
    ok = same[:, None] & (np.abs(dd_h[:, None] - ref["crit"]) > 1e-2)
    assert np.all((acc == ref["accepted"]) | ~ok)
    scale = np.maximum(1.0, np.abs(ref["crit"]))
    assert np.all((np.abs(crit - ref["crit"]) <= 1e-3 * scale) | ~same[:, None])
