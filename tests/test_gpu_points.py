"""fc_scan_points: universes grouped by true point (Algorithm 1's shape).

The FP32 form's offset path (d - S_p once, W_q (S_p - S_q) from a table) is
checked against the FP64 oracle; the other forms must equal fc_scan on the
expanded per-universe true points bit for bit.  Segments are ragged (empty,
single-universe, tile-sized and longer ones), so tiles end short of 256.
"""
from __future__ import annotations

import numpy as np
import pytest

import fcgen
import oracle
import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def fc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_07858_amd as fc
    fc.lib()
    return fc


def outputs(K):
    o = {k: torch.full((K,), -7.0, dtype=torch.float64, device="cuda")
         for k in ("dchi2", "chi2_min", "chi2_p")}
    o["argmin"] = torch.full((K,), -7, dtype=torch.int64, device="cuda")
    return o


def run_points(fc, g, form, p, seg, d):
    K = d.shape[0]
    o = outputs(K)
    fc.fc_scan_points(g, form, torch.as_tensor(np.asarray(p, dtype=np.int64)).cuda(),
                      torch.as_tensor(np.asarray(seg, dtype=np.int64)).cuda(),
                      torch.as_tensor(d).cuda(), o["dchi2"], o["chi2_min"], o["argmin"],
                      o["chi2_p"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def run_scan(fc, g, form, p_idx, d):
    K = d.shape[0]
    o = outputs(K)
    fc.fc_scan(g, form, torch.as_tensor(d).cuda(), torch.as_tensor(p_idx).cuda(), o["dchi2"],
               o["chi2_min"], o["argmin"], o["chi2_p"])
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def ragged(pr, sizes, seed):
    rng = np.random.default_rng(seed)
    p = rng.choice(pr.G, len(sizes), replace=False)
    seg = np.concatenate([[0], np.cumsum(sizes)])
    d = np.concatenate([fcgen.universes(2, 100 * seed + j, pr.S[p[j]], pr.F, int(sizes[j]))
                        for j in range(len(sizes))])
    return p, seg, d, np.repeat(p, sizes)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_points_fp32_matches_oracle(fc, name):
    n_axis = {"c1": None, "c2": (40, 40)}[name]
    pr = fcgen.make_problem(name, K=1, true_subset=[0], n_axis=n_axis)
    sizes = np.array([700, 1, 0, 64, 130, 257, 3])
    p, seg, d, p_idx = ragged(pr, sizes, 1)
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=fc.FC_FORM_FP32)
    dev = run_points(fc, g, fc.FC_FORM_FP32, p, seg, d)
    g.destroy()
    ref = oracle.scan(pr.S, pr.F, d, p_idx)
    parity.check_invariants(dev, pr.G)
    rep = parity.report(dev, ref, parity.TOL["fp32"])
    assert rep["e_rel"] <= parity.TOL["fp32"], rep
    assert rep["argmin_agree"] == 1.0, rep
    assert parity.argmin_validity(pr, dev, d, ref, parity.TOL["fp32"])["argmin_valid"] == 1.0


@pytest.mark.parametrize("form_name", ["fp64", "split_bf16", "split_fp16"])
def test_points_other_forms_equal_fc_scan(fc, form_name):
    form = {"fp64": 1, "split_bf16": 4, "split_fp16": 8}[form_name]
    pr = fcgen.make_problem("c1", K=1, true_subset=[0])
    sizes = np.array([90, 0, 200, 33])
    p, seg, d, p_idx = ragged(pr, sizes, 2)
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=form)
    a = run_points(fc, g, form, p, seg, d)
    b = run_scan(fc, g, form, p_idx, d)
    g.destroy()
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("N", list(range(1, 65)))
def test_points_fp32_every_bin_count(fc, N):
    """The offset path is compiled per bin count like the residual path: every
    N, with two segments whose tiles end short of 256 universes."""
    rng = np.random.default_rng(2000 + N)
    G, sizes = 23, np.array([200, 100])
    S = rng.uniform(20, 800, size=(G, N))
    A = rng.normal(size=(N, 2 * N))
    W = A @ A.T
    dw = np.sqrt(np.diag(W))
    F = 0.5 * ((W / np.outer(dw, dw)) + (W / np.outer(dw, dw)).T) * 0.02
    p = np.array([5, 17])
    seg = np.array([0, 200, 300])
    p_idx = np.repeat(p, sizes)
    d = S[p_idx] + rng.normal(0, 1, size=(300, N)) * np.sqrt(S[p_idx])
    ref = oracle.scan(S, F, d, p_idx)
    g = fc.fc_build_grid([np.arange(float(G))], S)
    fc.fc_build_covariance(g, F, forms=2)
    dev = run_points(fc, g, 2, p, seg, d)
    g.destroy()
    parity.check_invariants(dev, G)
    rep = parity.report(dev, ref, parity.TOL["fp32"])
    assert rep["e_rel"] <= parity.TOL["fp32"], rep
    assert rep["argmin_agree"] == 1.0, rep


def test_points_unfluctuated_and_bad_points(fc):
    """d = S_p exactly: the offset path gives Delta chi2 = 0 and chi2_min = 0
    exactly (e = 0 and the table row at q = p is W (S_p - S_p) = 0); a
    segment whose true point is outside the grid gets NaN."""
    pr = fcgen.make_problem("c1", K=1, true_subset=[0])
    ps = np.array([0, 17, 382, 399, 200])
    sizes = np.array([64, 64, 64, 64, 64])
    seg = np.concatenate([[0], np.cumsum(sizes)])
    d = pr.S[np.repeat(ps, sizes)]
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=2)
    dev = run_points(fc, g, 2, ps, seg, d)
    assert np.all(dev["dchi2"] == 0.0) and np.all(dev["chi2_min"] == 0.0)
    np.testing.assert_array_equal(dev["argmin"], np.repeat(ps, sizes))
    bad = run_points(fc, g, 2, np.array([3, pr.G + 5]), np.array([0, 70, 140]),
                     pr.S[np.repeat([3, 3], 70)])
    g.destroy()
    assert np.all(bad["dchi2"][:70] == 0.0)
    assert np.all(np.isnan(bad["dchi2"][70:])) and np.all(np.isnan(bad["chi2_p"][70:]))


def test_points_workspace_errors(fc):
    pr = fcgen.make_problem("c1", K=1, true_subset=[0])
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=2)
    K = 100
    need = fc.fc_scan_points_workspace(g, 2, 1, K)
    assert need >= 8 * K + pr.G * 16 * 10           # true points + table (N = 38: ns = 10)
    p = torch.tensor([5], dtype=torch.int64, device="cuda")
    seg = torch.tensor([0, K], dtype=torch.int64, device="cuda")
    d = torch.as_tensor(pr.S[[5] * K]).cuda()
    o = outputs(K)
    small = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(fc.FCError) as ei:
        fc.fc_scan_points(g, 2, p, seg, d, o["dchi2"], o["chi2_min"], o["argmin"], o["chi2_p"],
                          workspace=small)
    assert ei.value.code == fc.FC_ERR_INVALID_ARG
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(fc.FCError) as ei:                       # misaligned
        fc.fc_scan_points(g, 2, p, seg, d, o["dchi2"], o["chi2_min"], o["argmin"], o["chi2_p"],
                          workspace=big[8:])
    assert ei.value.code == fc.FC_ERR_INVALID_ARG
    fc.fc_scan_points(g, 2, p, seg, d, o["dchi2"], o["chi2_min"], o["argmin"], o["chi2_p"],
                      workspace=big)
    torch.cuda.synchronize()
    assert bool((o["dchi2"] == 0).all())
    g.destroy()


def test_points_full_size_c2_sampled(fc):
    """The benchmark's configuration through fc_scan_points: 256 points x 2000
    universes on the 100 x 100 grid, sampled universes against the oracle."""
    pr = fcgen.make_problem("c2")
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=2)
    pts = pr.p_idx[pr.seg_off[:-1]]
    dev = run_points(fc, g, 2, pts, pr.seg_off, pr.d)
    g.destroy()
    parity.check_invariants(dev, pr.G)
    rows = np.concatenate([pr.seg_off[:-1] + k for k in (0, 1, 999, 1999)])
    rows = np.concatenate([rows, np.arange(1990, 2070)])
    ref = oracle.scan(pr.S, pr.F, pr.d[rows], pr.p_idx[rows])
    ds = {k: v[rows] for k, v in dev.items()}
    rep = parity.report(ds, ref, parity.TOL["fp32"])
    assert rep["e_rel"] <= parity.TOL["fp32"], rep
    assert rep["argmin_agree"] == 1.0, rep
    assert parity.argmin_validity(pr, ds, pr.d[rows], ref, parity.TOL["fp32"])["argmin_valid"] == 1.0


def test_points_many_segments_and_long_ones(fc):
    """2500 segments (the tile prefix sum runs over three 1024-segment chunks),
    most of them tiny, some empty, and two long ones of 20 and 9 tiles (more
    than the eight tiles that share an XCD)."""
    pr = fcgen.make_problem("c1", K=1, true_subset=[0], n_axis=(12, 12))
    rng = np.random.default_rng(11)
    sizes = rng.integers(0, 4, 2500)
    sizes[100] = 5000
    sizes[2400] = 2100
    p = rng.integers(0, pr.G, sizes.size)
    seg = np.concatenate([[0], np.cumsum(sizes)])
    p_idx = np.repeat(p, sizes)
    K = int(seg[-1])
    d = pr.S[p_idx] + rng.normal(0, 1, size=(K, pr.N)) * np.sqrt(pr.S[p_idx])
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=2)
    dev = run_points(fc, g, 2, p, seg, d)
    g.destroy()
    parity.check_invariants(dev, pr.G)
    ref = oracle.scan(pr.S, pr.F, d, p_idx)
    rep = parity.report(dev, ref, parity.TOL["fp32"])
    assert rep["e_rel"] <= parity.TOL["fp32"], rep
    assert rep["argmin_agree"] == 1.0, rep
    assert parity.argmin_validity(pr, dev, d, ref, parity.TOL["fp32"])["argmin_valid"] == 1.0


def test_points_empty_inputs(fc):
    """K = 0 enqueues nothing; all-empty segments likewise; n_pts = 0 with
    universes is an argument error."""
    pr = fcgen.make_problem("c1", K=1, true_subset=[0])
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=2)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    ei = torch.empty(0, dtype=torch.int64, device="cuda")
    d0 = torch.empty((0, pr.N), dtype=torch.float64, device="cuda")
    fc.fc_scan_points(g, 2, torch.tensor([3, 4], dtype=torch.int64, device="cuda"),
                      torch.zeros(3, dtype=torch.int64, device="cuda"), d0, e, e, ei, e)
    o = outputs(5)
    with pytest.raises(fc.FCError) as ei_:
        fc.fc_scan_points(g, 2, torch.empty(0, dtype=torch.int64, device="cuda"),
                          torch.zeros(1, dtype=torch.int64, device="cuda"),
                          torch.as_tensor(pr.S[[3] * 5]).cuda(), o["dchi2"], o["chi2_min"],
                          o["argmin"], o["chi2_p"])
    assert ei_.value.code == fc.FC_ERR_INVALID_ARG
    torch.cuda.synchronize()
    g.destroy()
