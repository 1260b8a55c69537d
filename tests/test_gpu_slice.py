"""Grid-sliced scans: Algorithm 1's loop over the grid cut into slices
[q0, q0 + nq), each a call of its own (one device's share when the grid is
sharded over devices).  The per-universe state -- the packed (FP32 chi2 bits,
q) key and chi2(d, p) -- merges by a 64-bit unsigned MIN and a SUM, so slices
that cover the grid once must reproduce the one-call scan of the same form bit
for bit: with one shared state, with separate states merged on the host, and
in any order.  The one-call scans are themselves checked against the FP64
oracle elsewhere; one sliced case is also checked against it directly here.
"""
from __future__ import annotations

import numpy as np
import pytest

import fcgen
import oracle
import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FORMS = {"fp32": 2, "split_bf16": 4, "split_fp16": 8}


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


def host(o):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def new_state(fc, K):
    keys = torch.full((K,), 12345, dtype=torch.int64, device="cuda")
    chi2_p = torch.full((K,), -3.0, dtype=torch.float64, device="cuda")
    fc.fc_scan_state_init(keys, chi2_p)
    return keys, chi2_p


def finalize(fc, g, p_idx_t, keys, chi2_p):
    o = outputs(keys.numel())
    fc.fc_scan_state_finalize(g, p_idx_t, keys, chi2_p, o["dchi2"], o["chi2_min"], o["argmin"])
    o["chi2_p"] = chi2_p.clone()
    return host(o)


def merge_on_host(states):
    """The two reductions a sharded job would run as collectives."""
    keys = np.stack([k.cpu().numpy().view(np.uint64) for k, _ in states]).min(axis=0)
    chi2_p = np.stack([c.cpu().numpy() for _, c in states]).sum(axis=0)
    return (torch.as_tensor(keys.view(np.int64)).cuda(), torch.as_tensor(chi2_p).cuda())


def slices_of(G):
    """Uneven slices covering [0, G) once: a single point, an empty slice, a
    long one and the ragged rest."""
    a, b = 1, 1 + (G * 3) // 7
    return [(0, a), (a, 0), (a, b - a), (b, G - b)]


def problem(n_axis=None, sizes=(700, 1, 0, 64, 257, 300), seed=3):
    pr = fcgen.make_problem("c1", K=1, true_subset=[0], n_axis=n_axis)
    rng = np.random.default_rng(seed)
    sizes = np.asarray(sizes)
    p = rng.choice(pr.G, len(sizes), replace=False)
    seg = np.concatenate([[0], np.cumsum(sizes)])
    d = np.concatenate([fcgen.universes(2, 100 * seed + j, pr.S[p[j]], pr.F, int(sizes[j]))
                        for j in range(len(sizes))])
    return pr, p, seg, d, np.repeat(p, sizes)


@pytest.mark.parametrize("form_name", list(FORMS))
def test_slices_equal_one_call_scan(fc, form_name):
    form = FORMS[form_name]
    pr, _, _, d, p_idx = problem(n_axis=(23, 29))
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=form)
    K = d.shape[0]
    d_t, p_t = torch.as_tensor(d).cuda(), torch.as_tensor(p_idx).cuda()
    ref = outputs(K)
    fc.fc_scan(g, form, d_t, p_t, ref["dchi2"], ref["chi2_min"], ref["argmin"], ref["chi2_p"])
    ref = host(ref)
    sl = slices_of(pr.G)
    # one shared state, slices in reverse order
    keys, chi2_p = new_state(fc, K)
    for q0, nq in reversed(sl):
        fc.fc_scan_slice(g, form, d_t, p_t, q0, nq, keys, chi2_p)
    shared = finalize(fc, g, p_t, keys, chi2_p)
    # one state per slice, merged as a sharded job would
    states = []
    for q0, nq in sl:
        st = new_state(fc, K)
        fc.fc_scan_slice(g, form, d_t, p_t, q0, nq, *st)
        states.append(st)
    merged = finalize(fc, g, p_t, *merge_on_host(states))
    g.destroy()
    for out in (shared, merged):
        for k in ref:
            np.testing.assert_array_equal(out[k], ref[k], err_msg=k)


@pytest.mark.parametrize("form_name", list(FORMS))
def test_points_slices_equal_one_call_scan(fc, form_name):
    """fc_scan_points_slice (the offset form in FP32) against fc_scan_points."""
    form = FORMS[form_name]
    pr, p, seg, d, p_idx = problem(n_axis=(31, 17), seed=4)
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=form)
    K = d.shape[0]
    d_t, p_t = torch.as_tensor(d).cuda(), torch.as_tensor(p_idx).cuda()
    pts_t = torch.as_tensor(p.astype(np.int64)).cuda()
    seg_t = torch.as_tensor(seg.astype(np.int64)).cuda()
    ref = outputs(K)
    fc.fc_scan_points(g, form, pts_t, seg_t, d_t, ref["dchi2"], ref["chi2_min"], ref["argmin"],
                      ref["chi2_p"])
    ref = host(ref)
    keys, chi2_p = new_state(fc, K)
    for q0, nq in slices_of(pr.G):
        fc.fc_scan_points_slice(g, form, pts_t, seg_t, d_t, q0, nq, keys, chi2_p)
    out = finalize(fc, g, p_t, keys, chi2_p)
    g.destroy()
    for k in ref:
        np.testing.assert_array_equal(out[k], ref[k], err_msg=k)


def test_sliced_scan_matches_oracle(fc):
    """Eight slices of the 40 x 40 grid, FP32 offset form, against the FP64
    oracle over the whole grid."""
    pr, p, seg, d, p_idx = problem(n_axis=(40, 40), sizes=(300, 45, 256), seed=5)
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=2)
    K = d.shape[0]
    d_t, p_t = torch.as_tensor(d).cuda(), torch.as_tensor(p_idx).cuda()
    pts_t = torch.as_tensor(p.astype(np.int64)).cuda()
    seg_t = torch.as_tensor(seg.astype(np.int64)).cuda()
    keys, chi2_p = new_state(fc, K)
    edges = np.linspace(0, pr.G, 9).astype(int)
    for q0, q1 in zip(edges[:-1], edges[1:]):
        fc.fc_scan_points_slice(g, 2, pts_t, seg_t, d_t, int(q0), int(q1 - q0), keys, chi2_p)
    dev = finalize(fc, g, p_t, keys, chi2_p)
    g.destroy()
    ref = oracle.scan(pr.S, pr.F, d, p_idx)
    parity.check_invariants(dev, pr.G)
    rep = parity.report(dev, ref, parity.TOL["fp32"])
    assert rep["e_rel"] <= parity.TOL["fp32"], rep
    assert rep["argmin_agree"] == 1.0, rep
    assert parity.argmin_validity(pr, dev, d, ref, parity.TOL["fp32"])["argmin_valid"] == 1.0


def test_state_init_and_untouched_universes(fc):
    """After init, keys are the 'none' value and chi2_p is 0; finalizing an
    untouched state gives Algorithm 1's initial state (chi2_min = +inf,
    argmin = p, dchi2 = NaN)."""
    pr = fcgen.make_problem("c1", K=1, true_subset=[0])
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=2)
    K = 300
    keys, chi2_p = new_state(fc, K)
    torch.cuda.synchronize()
    assert np.all(keys.cpu().numpy().view(np.uint64) == np.uint64(0x7F800000FFFFFFFF))
    assert np.all(chi2_p.cpu().numpy() == 0.0)
    p_t = torch.arange(K, dtype=torch.int64, device="cuda") % pr.G
    out = finalize(fc, g, p_t, keys, chi2_p)
    g.destroy()
    assert np.all(np.isinf(out["chi2_min"])) and np.all(np.isnan(out["dchi2"]))
    np.testing.assert_array_equal(out["argmin"], np.arange(K) % pr.G)


def test_true_point_outside_grid(fc):
    """A universe whose true point is outside [0, G): the slices still find
    its minimum (as fc_scan does), no slice writes chi2_p, and finalize gives
    dchi2 = NaN; the other universes are unaffected."""
    pr, _, _, d, p_idx = problem(sizes=(200, 100), seed=6)
    p_bad = p_idx.copy()
    p_bad[200:] = pr.G + 3
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=2)
    K = d.shape[0]
    d_t, p_t = torch.as_tensor(d).cuda(), torch.as_tensor(p_bad).cuda()
    ref = outputs(K)
    fc.fc_scan(g, 2, d_t, p_t, ref["dchi2"], ref["chi2_min"], ref["argmin"], ref["chi2_p"])
    ref = host(ref)
    keys, chi2_p = new_state(fc, K)
    for q0, nq in slices_of(pr.G):
        fc.fc_scan_slice(g, 2, d_t, p_t, q0, nq, keys, chi2_p)
    out = finalize(fc, g, p_t, keys, chi2_p)
    g.destroy()
    np.testing.assert_array_equal(out["chi2_min"], ref["chi2_min"])
    np.testing.assert_array_equal(out["argmin"], ref["argmin"])
    np.testing.assert_array_equal(out["dchi2"][:200], ref["dchi2"][:200])
    assert np.all(np.isnan(out["dchi2"][200:])) and np.all(out["chi2_p"][200:] == 0.0)


def test_slice_argument_errors(fc):
    pr = fcgen.make_problem("c1", K=1, true_subset=[0])
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=1 | 2)
    K = 64
    d_t = torch.as_tensor(pr.S[[7] * K]).cuda()
    p_t = torch.full((K,), 7, dtype=torch.int64, device="cuda")
    keys, chi2_p = new_state(fc, K)
    for q0, nq in ((-1, 5), (0, pr.G + 1), (pr.G, 1), (5, -2)):
        with pytest.raises(fc.FCError) as ei:
            fc.fc_scan_slice(g, 2, d_t, p_t, q0, nq, keys, chi2_p)
        assert ei.value.code == fc.FC_ERR_INVALID_ARG, (q0, nq)
    with pytest.raises(fc.FCError) as ei:                      # FP64 minima do not pack
        fc.fc_scan_slice(g, 1, d_t, p_t, 0, pr.G, keys, chi2_p)
    assert ei.value.code == fc.FC_ERR_UNSUPPORTED
    with pytest.raises(fc.FCError) as ei:                      # form not built
        fc.fc_scan_slice(g, 8, d_t, p_t, 0, pr.G, keys, chi2_p)
    assert ei.value.code == fc.FC_ERR_STATE
    pts = torch.tensor([7], dtype=torch.int64, device="cuda")
    seg = torch.tensor([0, K], dtype=torch.int64, device="cuda")
    need = fc.fc_scan_points_slice_workspace(g, 2, 1, K, 100)
    assert need < fc.fc_scan_points_workspace(g, 2, 1, K)
    with pytest.raises(fc.FCError) as ei:
        fc.fc_scan_points_slice(g, 2, pts, seg, d_t, 50, 100, keys, chi2_p,
                                workspace=torch.empty(need - 1, dtype=torch.uint8,
                                                      device="cuda"))
    assert ei.value.code == fc.FC_ERR_INVALID_ARG
    # an exactly sized workspace for [50, 150), which does not hold p = 7; the
    # other two slices complete the grid (d = S_7: chi2 = 0 exactly at q = 7)
    fc.fc_scan_points_slice(g, 2, pts, seg, d_t, 50, 100, keys, chi2_p,
                            workspace=torch.empty(need, dtype=torch.uint8, device="cuda"))
    fc.fc_scan_points_slice(g, 2, pts, seg, d_t, 0, 50, keys, chi2_p)
    fc.fc_scan_points_slice(g, 2, pts, seg, d_t, 150, pr.G - 150, keys, chi2_p)
    out = finalize(fc, g, p_t, keys, chi2_p)
    g.destroy()
    assert np.all(out["dchi2"] == 0.0) and np.all(out["chi2_min"] == 0.0)
    assert np.all(out["argmin"] == 7)
