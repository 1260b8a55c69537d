"""GPU universes (fc_generate_universes) against the oracle's generator.

Both sides implement the same counter-based stream (Philox4x64-10), Poisson
sampler (multiplication method / PTRS) and Box-Muller normals from their
published definitions; they share no code.  The Poisson counts are integer
decisions and must agree exactly; d agrees to rounding (the two sides' log,
cos and Cholesky differ in the last bits).
"""
from __future__ import annotations

import numpy as np
import pytest

import fcgen
import oracle
import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

D_TOL = 1e-12


@pytest.fixture(scope="module")
def fc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2002_07858_amd as fc
    fc.lib()
    return fc


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def gen(fc, g, N, p, seg_off, seed, u_first=None):
    K = int(seg_off[-1])
    d = torch.full((K, N), -7.0, dtype=torch.float64, device="cuda")
    pi = torch.full((K,), -7, dtype=torch.int64, device="cuda")
    cnt = torch.full((K, N), -7, dtype=torch.int32, device="cuda")
    fc.fc_generate_universes(g, to_dev(p, torch.int64), to_dev(seg_off, torch.int64), seed, d,
                             pi, cnt, None if u_first is None else to_dev(u_first, torch.int64))
    torch.cuda.synchronize()
    return d.cpu().numpy(), pi.cpu().numpy(), cnt.cpu().numpy()


def close(a, b):
    return np.all(np.abs(a - b) <= D_TOL * np.maximum(1.0, np.abs(b)))


@pytest.mark.parametrize("name,seed", [("c1", 1), ("c2", 20020785), ("c3", 2**63 + 5)])
def test_universes_match_oracle(fc, name, seed):
    n_axis = {"c1": None, "c2": (20, 20), "c3": (8, 8, 8)}[name]
    pr = fcgen.make_problem(name, K=1, true_subset=[0], n_axis=n_axis)
    rng = np.random.default_rng(3)
    p = rng.integers(0, pr.G, 7)
    sizes = np.array([1, 0, 63, 64, 65, 300, 17])        # ragged, one empty
    seg = np.concatenate([[0], np.cumsum(sizes)])
    uf = rng.integers(0, 10**6, 7)
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=fc.FC_FORM_FP32)
    d, pi, cnt = gen(fc, g, pr.N, p, seg, seed, uf)
    g.destroy()
    d_o, c_o = oracle.universes(pr.S, pr.F, p, seg, seed, u_first=uf)
    np.testing.assert_array_equal(cnt, c_o)
    assert close(d, d_o), float(np.abs(d - d_o).max())
    np.testing.assert_array_equal(pi, np.repeat(p, sizes))


def test_universes_batching_invariance(fc):
    """Rows depend only on (seed, p, j): one call for universes 0..999 equals
    a call for 600..999 alone, bit for bit."""
    pr = fcgen.make_problem("c2", K=1, true_subset=[0])
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=fc.FC_FORM_FP32)
    d, _, c = gen(fc, g, pr.N, [4321, 77], [0, 1000, 1500], 9)
    d2, _, c2 = gen(fc, g, pr.N, [4321], [0, 400], 9, u_first=[600])
    d3, _, c3 = gen(fc, g, pr.N, [77, 4321], [0, 500, 600], 9, u_first=[0, 400])
    g.destroy()
    np.testing.assert_array_equal(d2, d[600:1000])
    np.testing.assert_array_equal(c2, c[600:1000])
    np.testing.assert_array_equal(d3[:500], d[1000:1500])
    np.testing.assert_array_equal(d3[500:], d[400:500])


def test_small_and_zero_means_and_bad_points(fc):
    """Means below 10 (multiplication method) and exactly 0, with a fixed
    statistical term so the covariance stays positive definite; true points
    outside the grid give NaN rows."""
    rng = np.random.default_rng(4)
    G, N = 6, 40
    S = rng.uniform(0.2, 14.0, (G, N))
    S[2, :5] = 0.0
    F = 0.01 * np.eye(N) + 0.002
    stat = np.full(N, 3.0)
    g = fc.fc_build_grid([np.arange(float(G))], S)
    fc.fc_build_covariance(g, F, fc.FC_STAT_FIXED, stat, forms=fc.FC_FORM_FP32)
    p = np.array([2, 0, 5, 9, -1])
    seg = np.array([0, 200, 400, 600, 603, 605])
    d, pi, cnt = gen(fc, g, N, p, seg, 123)
    g.destroy()
    d_o, c_o = oracle.universes(S, F, p[:3], seg[:4], 123)
    np.testing.assert_array_equal(cnt[:600], c_o)
    assert close(d[:600], d_o)
    assert np.all(cnt[:200, :5] == 0)
    assert np.all(np.isnan(d[600:])) and np.all(cnt[600:] == -1) and np.all(pi[600:] == -1)


def test_generate_errors(fc):
    pr = fcgen.make_problem("c1", K=1, true_subset=[0])
    g = fc.fc_build_grid(pr.axes, pr.S)
    d = torch.empty((4, pr.N), dtype=torch.float64, device="cuda")
    p = to_dev([0], torch.int64)
    seg = to_dev([0, 4], torch.int64)
    with pytest.raises(fc.FCError) as ei:                 # no covariance yet
        fc.fc_generate_universes(g, p, seg, 1, d)
    assert ei.value.code == fc.FC_ERR_STATE
    # F positive semidefinite only: the scan covariance is fine, F has no factor
    v = np.linspace(0.05, 0.2, pr.N)
    fc.fc_build_covariance(g, np.outer(v, v), forms=fc.FC_FORM_FP32)
    with pytest.raises(fc.FCError) as ei:
        fc.fc_generate_universes(g, p, seg, 1, d)
    assert ei.value.code == fc.FC_ERR_NOT_PD
    fc.fc_build_covariance(g, pr.F, forms=fc.FC_FORM_FP32)
    fc.fc_generate_universes(g, p, to_dev([0, 0], torch.int64), 1, d[:0])   # K = 0
    torch.cuda.synchronize()
    g.destroy()


def test_generated_universes_scan_matches_oracle(fc):
    """The whole device chain -- draw universes, FP32 scan -- against the
    oracle's universes scanned by the oracle."""
    pr = fcgen.make_problem("c2", K=1, true_subset=[0], n_axis=(30, 30))
    p = np.array([10, 455, 899])
    seg = np.array([0, 150, 300, 450])
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=fc.FC_FORM_FP32)
    K = int(seg[-1])
    d = torch.empty((K, pr.N), dtype=torch.float64, device="cuda")
    pi = torch.empty(K, dtype=torch.int64, device="cuda")
    fc.fc_generate_universes(g, to_dev(p, torch.int64), to_dev(seg, torch.int64), 5, d, pi)
    o = {k: torch.empty(K, dtype=torch.float64, device="cuda") for k in ("dchi2", "chi2_min",
                                                                       "chi2_p")}
    o["argmin"] = torch.empty(K, dtype=torch.int64, device="cuda")
    fc.fc_scan(g, fc.FC_FORM_FP32, d, pi, o["dchi2"], o["chi2_min"], o["argmin"], o["chi2_p"])
    torch.cuda.synchronize()
    dev = {k: v.cpu().numpy() for k, v in o.items()}
    g.destroy()
    d_o, _ = oracle.universes(pr.S, pr.F, p, seg, 5)
    ref = oracle.scan(pr.S, pr.F, d_o, np.repeat(p, np.diff(seg)))
    rep = parity.report(dev, ref, parity.TOL["fp32"])
    assert rep["e_rel"] <= parity.TOL["fp32"], rep
    assert rep["argmin_agree"] == 1.0, rep
    assert parity.argmin_validity(pr, dev, d_o, ref, parity.TOL["fp32"])["argmin_valid"] == 1.0


def test_large_universe_count_indexing(fc):
    """2^26 universes drawn on the device and scanned: the universe array has
    2.5e9 elements, past 32-bit indexing; sampled rows (the last ones
    included) against the oracle, invariants on every row on the device."""
    pr = fcgen.make_problem("c1", K=1, true_subset=[0], n_axis=(3, 3))
    K = 1 << 26
    p = np.array([1, 4, 8])
    seg = np.array([0, K // 3, 2 * (K // 3), K])
    g = fc.fc_build_grid(pr.axes, pr.S)
    fc.fc_build_covariance(g, pr.F, forms=fc.FC_FORM_FP32)
    d = torch.empty((K, pr.N), dtype=torch.float64, device="cuda")
    pi = torch.empty(K, dtype=torch.int64, device="cuda")
    fc.fc_generate_universes(g, to_dev(p, torch.int64), to_dev(seg, torch.int64), 31, d, pi)
    o = {k: torch.empty(K, dtype=torch.float64, device="cuda") for k in ("dchi2", "chi2_min",
                                                                       "chi2_p")}
    o["argmin"] = torch.empty(K, dtype=torch.int64, device="cuda")
    fc.fc_scan(g, fc.FC_FORM_FP32, d, pi, o["dchi2"], o["chi2_min"], o["argmin"], o["chi2_p"])
    torch.cuda.synchronize()
    assert bool((o["dchi2"] >= 0).all()) and bool((o["argmin"] >= 0).all())
    assert bool((o["argmin"] < pr.G).all())
    rows = np.concatenate([np.arange(5), [K // 3 - 1, K // 3, K // 2], K - 1 - np.arange(5)])
    k_of = np.searchsorted(seg, rows, side="right") - 1
    d_host = d[torch.as_tensor(rows, device="cuda")].cpu().numpy()
    dev = {k: v[torch.as_tensor(rows, device="cuda")].cpu().numpy() for k, v in o.items()}
    g.destroy()
    del d
    # the oracle's rows: universe index j = row - seg[k] of point p[k]
    ref_d = np.concatenate([oracle.universes(pr.S, pr.F, [p[k]], [0, 1], 31,
                                             u_first=[r - seg[k]])[0]
                            for r, k in zip(rows, k_of)])
    assert close(d_host, ref_d)
    ref = oracle.scan(pr.S, pr.F, ref_d, p[k_of])
    rep = parity.report(dev, ref, parity.TOL["fp32"])
    assert rep["e_rel"] <= parity.TOL["fp32"], rep
