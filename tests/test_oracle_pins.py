"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every expected value is exact
rational arithmetic, a closed form, a library routine on a special case, a
distributional law (Wilks), or an exact invariant of Algorithm 1.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.stats

import exact_fc
import fcgen
import oracle


# --------------------------------------------------------------------------
# P1: exact rational brute force on a 3x3 grid with N = 4 (Eq. (1), Alg. 1)
# --------------------------------------------------------------------------
def _p1_problem():
    # integer signal rows; row 5 duplicates row 2 so that exact ties occur
    S = [[10, 12, 9, 14], [11, 12, 10, 13], [12, 11, 11, 15],
         [9, 13, 12, 12], [13, 10, 9, 16], [12, 11, 11, 15],
         [10, 10, 10, 10], [14, 14, 12, 11], [8, 12, 13, 14]]
    # F = B B^T / 100 with a small integer B: symmetric positive semidefinite
    B = [[1, 0, 2], [0, 1, 1], [1, 1, 0], [2, 0, 1]]
    F = [[Fraction(sum(B[i][k] * B[j][k] for k in range(3)), 100) for j in range(4)]
         for i in range(4)]
    d = [[12, 11, 11, 15], [11, 13, 10, 12], [7, 15, 14, 10], [13, 9, 9, 17],
         [12, 11, 12, 15]]
    p = [2, 1, 8, 4, 5]
    return S, F, d, p


def test_p1_exact_rational_bruteforce():
    S, F, d, p = _p1_problem()
    exact = exact_fc.scan(S, F, d, p)
    Sn = np.array(S, dtype=np.float64)
    Fn = np.array([[float(x) for x in row] for row in F])
    dn = np.array(d, dtype=np.float64)
    r = oracle.scan(Sn, Fn, dn, np.array(p))
    for k, (dc, cmin, am, cp, c2) in enumerate(exact):
        scale = max(1.0, float(cp))
        assert abs(r["dchi2"][k] - float(dc)) <= 1e-14 * scale
        assert abs(r["chi2_min"][k] - float(cmin)) <= 1e-14 * scale
        assert abs(r["chi2_p"][k] - float(cp)) <= 1e-14 * scale
        assert r["argmin"][k] == am
        assert abs(r["chi2_2nd"][k] - float(c2)) <= 1e-14 * scale
    # universe 0 sits exactly on row 2 == row 5: chi^2 = 0 at both, q = 2 wins
    assert r["chi2_min"][0] == 0.0 and r["argmin"][0] == 2 and r["dchi2"][0] == 0.0
    assert r["chi2_2nd"][0] == 0.0
    # universe 4 has true point 5 (the duplicate): argmin must be 2, Delta chi^2 = 0
    assert exact[4][2] == 2 and r["argmin"][4] == 2 and r["dchi2"][4] == 0.0


# --------------------------------------------------------------------------
# P2: scalar closed form (N = 1): chi^2 = (d - q)^2 / sigma^2
# --------------------------------------------------------------------------
def test_p2_scalar_closed_form():
    G = 11
    S = np.arange(G, dtype=np.float64)[:, None]        # S(q) = q
    F = np.zeros((1, 1))
    stat = np.array([4.0])                             # sigma = 2 exactly
    d = np.array([[3.25], [-1.5], [12.75], [2.5], [7.0], [0.0]])
    p = np.array([5, 0, 10, 4, 7, 3])
    r = oracle.scan(S, F, d, p, stat_mode=oracle.STAT_FIXED, stat_diag=stat)
    for k in range(d.shape[0]):
        x = Fraction(d[k, 0])
        vals = [(x - q) ** 2 / 4 for q in range(G)]
        best = min(vals)
        qbest = vals.index(best)                       # lowest q among ties
        assert r["chi2_min"][k] == float(best)
        assert r["argmin"][k] == qbest
        assert r["dchi2"][k] == float(vals[p[k]] - best)
        assert r["chi2_2nd"][k] == float(min(v for q, v in enumerate(vals) if q != qbest))
    # grid edges and the exact midpoint tie (2.5 between q=2 and q=3 -> 2)
    assert list(r["argmin"]) == [3, 0, 10, 2, 7, 0]


# --------------------------------------------------------------------------
# P3: diagonal covariance: chi^2 = sum r_i^2 / Sigma_ii
# --------------------------------------------------------------------------
def test_p3_diagonal_covariance():
    rng = np.random.default_rng(3)
    G, N = 50, 9
    S = rng.uniform(50, 400, size=(G, N))
    F = np.diag(rng.uniform(0.01, 0.04, size=N))
    d = S[rng.integers(0, G, size=20)] + rng.normal(0, 20, size=(20, N))
    tab = oracle.chi2_table(S, F, d)
    for q in range(G):
        sig = S[q] + np.diag(F) * S[q] ** 2
        ref = ((d - S[q]) ** 2 / sig).sum(axis=1)
        np.testing.assert_allclose(tab[:, q], ref, rtol=1e-13, atol=0)


# --------------------------------------------------------------------------
# Cholesky and chi^2 against LAPACK (numpy) on random SPD matrices
# --------------------------------------------------------------------------
def test_cholesky_and_chi2_match_lapack():
    rng = np.random.default_rng(11)
    for N in (1, 2, 5, 38, 57, 64):
        A = rng.standard_normal((N, 2 * N))
        Sig = A @ A.T + N * np.eye(N)
        L = oracle.cholesky(Sig)
        np.testing.assert_allclose(L, np.linalg.cholesky(Sig), rtol=1e-12, atol=1e-12)
        a = rng.normal(size=N)
        b = rng.normal(size=N)
        ref = (a - b) @ np.linalg.solve(Sig, a - b)
        assert abs(oracle.chi2(L, a, b) - ref) <= 1e-12 * max(1.0, ref)


def test_not_positive_definite_detected():
    N = 4
    S = np.full((6, N), 100.0)
    S[3] = [100.0, 200.0, 50.0, 10.0]
    F = np.diag([0.01, 0.01, 0.01, 0.01])
    F[0, 1] = F[1, 0] = 0.5                      # indefinite for large S
    with pytest.raises(oracle.OracleError, match="q=0"):
        oracle.factor_range(S, F, oracle.STAT_FIXED, np.zeros(N))
    with pytest.raises(oracle.OracleError):
        oracle.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))


def test_covariance_definition():
    rng = np.random.default_rng(5)
    N = 7
    s = rng.uniform(10, 100, size=N)
    A = rng.normal(size=(N, N))
    F = (A @ A.T) / 100
    Sig = oracle.covariance(s, F)
    np.testing.assert_array_equal(Sig, F * np.outer(s, s) + np.diag(s))
    st = rng.uniform(1, 2, size=N)
    Sig2 = oracle.covariance(s, F, oracle.STAT_FIXED, st)
    np.testing.assert_array_equal(Sig2, F * np.outer(s, s) + np.diag(st))


# --------------------------------------------------------------------------
# P4 + P5: invariants of Algorithm 1 on the toy configuration
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1_result():
    pr = fcgen.make_problem("c1")
    return pr, oracle.scan(pr.S, pr.F, pr.d, pr.p_idx)


def test_p4_invariants(c1_result):
    pr, r = c1_result
    assert np.all(r["chi2_min"] >= 0)
    assert np.all(r["dchi2"] >= 0)
    assert np.all(r["dchi2"] <= r["chi2_p"])
    assert np.all(r["chi2_2nd"] >= r["chi2_min"])
    assert np.all((r["argmin"] >= 0) & (r["argmin"] < pr.G))
    # chi2_min is the value at argmin: recompute that single entry directly
    L = oracle.factor_range(pr.S, pr.F)
    for k in range(0, pr.K, 97):
        q = r["argmin"][k]
        assert oracle.chi2(L[q], pr.d[k], pr.S[q]) == r["chi2_min"][k]


def test_p4_single_point_grid():
    pr = fcgen.make_problem("c1")
    S = pr.S[[382]]
    r = oracle.scan(S, pr.F, pr.d[:50], np.zeros(50, dtype=np.int64))
    assert np.all(r["dchi2"] == 0.0)
    assert np.all(r["argmin"] == 0)
    assert np.all(np.isinf(r["chi2_2nd"]))


def test_p5_unfluctuated_universe():
    pr = fcgen.make_problem("c1")
    ps = np.array([0, 17, 382, 399])
    d = pr.S[ps].copy()
    r = oracle.scan(pr.S, pr.F, d, ps)
    assert np.all(r["chi2_min"] == 0.0)
    assert np.all(r["dchi2"] == 0.0)
    assert np.all(r["chi2_p"] == 0.0)


def test_nan_universe_keeps_initial_minimiser():
    pr = fcgen.make_problem("c1")
    d = pr.d[:3].copy()
    d[1, 5] = np.nan
    r = oracle.scan(pr.S, pr.F, d, pr.p_idx[:3])
    assert np.isnan(r["dchi2"][1]) and np.isinf(r["chi2_min"][1])
    assert r["argmin"][1] == pr.p_idx[1]
    assert np.all(np.isfinite(r["dchi2"][[0, 2]]))


# --------------------------------------------------------------------------
# P6: constructed minimiser in a linear model
# --------------------------------------------------------------------------
def _linear_model(N, D, h, n_per_axis, rng):
    s0 = rng.uniform(100, 500, size=N)
    Q, _ = np.linalg.qr(rng.normal(size=(N, D)))
    A = np.sqrt(s0)[:, None] * Q           # A^T Sigma^{-1} A = I for Sigma = diag(s0)
    ax = [h * (np.arange(n_per_axis) - n_per_axis // 2) for _ in range(D)]
    X = fcgen.grid_points(ax)
    S = s0[None, :] + X @ A.T
    return s0, A, X, S, ax


def test_p6_constructed_minimiser():
    rng = np.random.default_rng(6)
    N, D = 8, 2
    s0, A, X, S, _ = _linear_model(N, D, 0.25, 21, rng)
    Sig = np.diag(s0)
    Sinv = np.diag(1.0 / s0)
    F = np.zeros((N, N))
    # noise n orthogonal to col(A) in the Sigma^{-1} metric
    P = A @ np.linalg.solve(A.T @ Sinv @ A, A.T @ Sinv)
    qstar = np.array([37, 220, 400, 5])
    ps = np.array([220, 221, 10, 440])
    n = (np.eye(N) - P) @ rng.normal(0, 3, size=(N, len(qstar)))
    d = (S[qstar] + n.T)
    r = oracle.scan(S, F, d, ps, stat_mode=oracle.STAT_FIXED, stat_diag=s0)
    for k in range(len(qstar)):
        dx = X[qstar[k]] - X[ps[k]]
        dchi = dx @ (A.T @ Sinv @ A) @ dx
        chimin = n[:, k] @ Sinv @ n[:, k]
        assert r["argmin"][k] == qstar[k]
        assert abs(r["chi2_min"][k] - chimin) <= 1e-11 * max(1.0, chimin)
        assert abs(r["dchi2"][k] - dchi) <= 1e-11 * max(1.0, r["chi2_p"][k])
    del Sig


# --------------------------------------------------------------------------
# P7: Wilks -- for a linear model with Gaussian data Delta chi^2 ~ chi^2_D
# --------------------------------------------------------------------------
@pytest.mark.parametrize("D,n_axis,h,K", [(1, 161, 0.1, 20000), (2, 201, 0.1, 20000),
                                           (3, 41, 0.25, 20000)])
def test_p7_wilks(D, n_axis, h, K):
    # D = 1, 2: spacing 0.1 sigma over +-8 / +-10 sigma; D = 3: spacing 0.25 sigma
    # over +-5 sigma (a wider bias band, the same statistic)
    rng = np.random.default_rng(7 + D)
    N = 6
    s0, A, X, S, _ = _linear_model(N, D, h, n_axis, rng)
    F = np.zeros((N, N))
    p = (S.shape[0] - 1) // 2                  # the grid centre, x_p = 0
    d = S[p][None, :] + rng.normal(size=(K, N)) * np.sqrt(s0)[None, :]
    r = oracle.scan(S, F, d, np.full(K, p), stat_mode=oracle.STAT_FIXED, stat_diag=s0)
    x = r["dchi2"]
    assert np.all(x >= 0)
    # the grid minimum is above the continuous one by at most D h^2 / 4
    bias = D * h * h / 4
    for a in (0.5, 0.9, 0.95):
        qa = scipy.stats.chi2.ppf(a, D)
        frac_lo = np.mean(x <= qa - bias)
        frac_hi = np.mean(x <= qa)
        tol = 3 * math.sqrt(a * (1 - a) / K)
        assert frac_lo - tol <= a <= frac_hi + tol + 1e-12, (a, frac_lo, frac_hi)


# --------------------------------------------------------------------------
# P8: moment check -- the generator's universes have covariance Sigma_p
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name,K", [("c1", 1000), ("c2", 400)])
def test_p8_mean_chi2_at_true_point(name, K):
    pr = fcgen.make_problem(name, K=K, true_subset=[0])
    p = int(pr.true_pts[0])
    L = oracle.factor_range(pr.S, pr.F, q0=p, nq=1)[0]
    vals = np.array([oracle.chi2(L, pr.d[k], pr.S[p]) for k in range(pr.K)])
    N = pr.N
    assert abs(vals.mean() - N) <= 3 * math.sqrt(2 * N / pr.K)


# --------------------------------------------------------------------------
# P9: metamorphic relations
# --------------------------------------------------------------------------
def test_p9_bin_permutation():
    pr = fcgen.make_problem("c1", K=40)
    perm = np.random.default_rng(9).permutation(pr.N)
    a = oracle.scan(pr.S, pr.F, pr.d, pr.p_idx)
    b = oracle.scan(pr.S[:, perm], pr.F[np.ix_(perm, perm)], pr.d[:, perm], pr.p_idx)
    np.testing.assert_allclose(b["chi2_p"], a["chi2_p"], rtol=1e-12)
    np.testing.assert_allclose(b["dchi2"], a["dchi2"], rtol=0, atol=1e-11 * a["chi2_p"].max())


def test_p9_power_of_two_scaling_is_exact():
    pr = fcgen.make_problem("c1", K=40)
    st = pr.S.mean(axis=0)
    a = oracle.scan(pr.S, pr.F, pr.d, pr.p_idx, stat_mode=oracle.STAT_FIXED, stat_diag=st)
    b = oracle.scan(pr.S, 4.0 * pr.F, pr.d, pr.p_idx, stat_mode=oracle.STAT_FIXED,
                    stat_diag=4.0 * st)
    np.testing.assert_array_equal(b["chi2_min"] * 4.0, a["chi2_min"])
    np.testing.assert_array_equal(b["dchi2"] * 4.0, a["dchi2"])
    np.testing.assert_array_equal(b["argmin"], a["argmin"])


def test_p9_grid_permutation():
    pr = fcgen.make_problem("c1", K=60)
    perm = np.random.default_rng(19).permutation(pr.G)
    inv = np.argsort(perm)
    a = oracle.scan(pr.S, pr.F, pr.d, pr.p_idx)
    b = oracle.scan(pr.S[perm], pr.F, pr.d, inv[pr.p_idx])
    np.testing.assert_array_equal(b["dchi2"], a["dchi2"])
    np.testing.assert_array_equal(perm[b["argmin"]], a["argmin"])


# --------------------------------------------------------------------------
# P10: quantiles and histogram
# --------------------------------------------------------------------------
def test_p10_quantile_of_integers():
    rng = np.random.default_rng(10)
    for K in (1, 2, 7, 1000, 2000, 2001):
        x = rng.permutation(np.arange(1, K + 1)).astype(np.float64)
        alphas = [0.5, 0.6827, 0.9, 0.95, 1.0, 1e-9]
        crit, hist = oracle.critical_value(x, [0, K], alphas, n_bins=10, hist_hi=5.0)
        for a, c in zip(alphas, crit[0]):
            assert c == max(1, math.ceil(a * K))
        assert hist.sum() == K


def test_p10_quantile_matches_sorted_order_statistic():
    rng = np.random.default_rng(12)
    x = rng.chisquare(2, size=5000)
    off = np.array([0, 1000, 1000, 3500, 5000])
    alphas = np.array([0.6827, 0.9, 0.95])
    crit, hist = oracle.critical_value(x, off, alphas, n_bins=50, hist_hi=10.0)
    for s in range(4):
        seg = np.sort(x[off[s]:off[s + 1]])
        K = seg.shape[0]
        for a, c in zip(alphas, crit[s]):
            if K == 0:
                assert np.isnan(c)
            else:
                assert c == seg[math.ceil(a * K) - 1]
        assert hist[s].sum() == K


def test_p10_histogram_on_unit_bins():
    rng = np.random.default_rng(13)
    x = rng.integers(0, 30, size=3000).astype(np.float64) + 0.5
    x[:7] = np.nan
    x[7:9] = -1.0
    _, hist = oracle.critical_value(x, [0, 3000], [0.5], n_bins=20, hist_hi=20.0)
    fin = x[9:]
    ref = np.bincount(np.floor(fin[fin < 20]).astype(int), minlength=20)
    np.testing.assert_array_equal(hist[0, :20], ref)
    assert hist[0, 20] == 7 + 2 + np.sum(fin >= 20)


def test_p10_nan_sorts_last():
    x = np.array([3.0, np.nan, 1.0, 2.0])
    crit, _ = oracle.critical_value(x, [0, 4], [0.25, 0.75, 1.0], with_hist=False)
    assert crit[0, 0] == 1.0 and crit[0, 1] == 3.0 and np.isnan(crit[0, 2])


def test_grid_linearisation_last_axis_fastest():
    axes = [np.array([0.0, 1.0]), np.array([10.0, 20.0, 30.0]), np.array([5.0, 6.0])]
    G = 12
    seen = [tuple(oracle.grid_coords(axes, q)) for q in range(G)]
    ref = [(a, b, c) for a in axes[0] for b in axes[1] for c in axes[2]]
    assert seen == ref
    np.testing.assert_array_equal(fcgen.grid_points(axes), np.array(ref))


# --------------------------------------------------------------------------
# P11: the observed-data statistic and the acceptance region (Section 1)
# --------------------------------------------------------------------------
def test_p11_data_scan_exact_rational():
    S, F, d, _ = _p1_problem()
    Sn = np.array(S, dtype=np.float64)
    Fn = np.array([[float(x) for x in row] for row in F])
    Minv = [exact_fc.inverse(exact_fc.covariance(Sq, F)) for Sq in S]
    for c in d:
        exact = [exact_fc.chi2(c, Sq, M) for Sq, M in zip(S, Minv)]
        best = min(exact)
        arg = exact.index(best)                 # lowest q among exact ties
        dd, cmin, am = oracle.data_scan(Sn, Fn, np.array(c, dtype=np.float64))
        assert am == arg
        assert abs(cmin - float(best)) <= 1e-14 * max(1.0, float(best))
        for q in range(len(S)):
            assert abs(dd[q] - float(exact[q] - best)) <= 1e-14 * max(1.0, float(exact[q]))
    # c on the duplicated rows 2 == 5: chi^2 = 0 at both, q = 2 is the minimiser
    dd, cmin, am = oracle.data_scan(Sn, Fn, Sn[5])
    assert am == 2 and cmin == 0.0 and dd[2] == 0.0 and dd[5] == 0.0


def test_p11_data_scan_all_nan():
    pr = fcgen.make_problem("c1", K=1, true_subset=[0], n_axis=(4, 4))
    c = pr.S[3].copy()
    c[7] = np.nan
    dd, cmin, am = oracle.data_scan(pr.S, pr.F, c)
    assert am == -1 and math.isnan(cmin) and np.isnan(dd).all()


def test_p11_acceptance_boundary_and_range():
    dd = np.array([0.0, 1.5, 2.0, np.nan])
    acc = oracle.acceptance(dd, [0, 1, 2, 3, 4, -1], [0.0, 1.4, 2.0, 10.0, 10.0, 10.0])
    # equal is accepted, above is not, NaN and points off the grid are not
    assert acc.tolist() == [1, 0, 1, 0, 0, 0]


def test_p11_coverage_of_the_acceptance_region():
    """Feldman-Cousins coverage: data drawn at the true point p fall inside the
    region (Delta chi^2_data(p) <= x_alpha(p)) with probability alpha, because
    the critical value is the alpha-quantile of the same statistic over
    universes drawn at p.  A region built on chi^2 instead of Delta chi^2, a
    wrong minimiser or the wrong quantile moves the fraction far from alpha."""
    pr = fcgen.make_problem("c1", K=2000, true_subset=[0], n_axis=(10, 10))
    p = int(pr.true_pts[0])
    alpha = (0.6827, 0.9)
    r = oracle.scan(pr.S, pr.F, pr.d, pr.p_idx)
    crit, _ = oracle.critical_value(r["dchi2"], pr.seg_off, alpha, with_hist=False)
    M = 300
    data = fcgen.universes(pr.config, 10_000, pr.S[p], pr.F, M)
    hits = np.zeros(len(alpha))
    for m in range(M):
        dd, _, _ = oracle.data_scan(pr.S, pr.F, data[m])
        for a in range(len(alpha)):
            hits[a] += oracle.acceptance(dd, [p], [crit[0, a]])[0]
    for a, al in enumerate(alpha):
        sigma = math.sqrt(al * (1 - al) / M + al * (1 - al) / 2000)
        assert abs(hits[a] / M - al) <= 4 * sigma, (al, hits[a] / M)


# --------------------------------------------------------------------------
# P12: universes (Section 2, steps 1-2) from the counter-based stream
# --------------------------------------------------------------------------
@pytest.mark.parametrize("key,ctr", [((123, 456), (6, 0, 0, 0)),
                                     ((2**64 - 1, 5), (2**64 - 2, 2**64 - 1, 3, 9)),
                                     ((0, 0), (2**64 - 1, 2**64 - 1, 0, 0))])
def test_p12_philox_matches_numpy(key, ctr):
    # numpy's Philox (4x64, 10 rounds) advances its counter before each block
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(ctr, dtype=np.uint64))
    ref = [int(x) for x in bg.random_raw(4)]
    c = list(ctr)
    for w in range(4):                       # counter + 1 with carry
        c[w] = (c[w] + 1) % 2**64
        if c[w]:
            break
    assert oracle.philox4x64(c, key) == ref


def test_p12_uniform_open_interval():
    assert oracle.uniform(0) == 2.0**-54
    assert oracle.uniform(2**64 - 1) == 1.0 - 2.0**-54
    assert oracle.uniform(2**63) == 0.5 + 2.0**-54


@pytest.mark.parametrize("lam", [0.5, 3.0, 9.99, 10.0, 37.5, 300.0, 2000.0])
def test_p12_poisson_distribution(lam):
    """Chi-square goodness of fit against the Poisson pmf (scipy), both the
    multiplication branch (lambda < 10) and PTRS (lambda >= 10)."""
    n = 20000
    x = np.array([oracle.poisson(lam, 99, 3, j, 5) for j in range(n)])
    assert x.min() >= 0
    assert abs(x.mean() - lam) <= 5 * math.sqrt(lam / n)
    lo = int(max(0, lam - 7 * math.sqrt(lam) - 2))
    hi = int(lam + 7 * math.sqrt(lam) + 3)
    ks = np.arange(lo, hi + 1)
    expct = scipy.stats.poisson.pmf(ks, lam) * n
    obs = np.array([(x == k).sum() for k in ks])
    sel = expct >= 5
    rest_o, rest_e = n - obs[sel].sum(), n - expct[sel].sum()
    chi = ((obs[sel] - expct[sel]) ** 2 / expct[sel]).sum()
    dof = int(sel.sum()) - 1
    if rest_e >= 5:
        chi += (rest_o - rest_e) ** 2 / rest_e
        dof += 1
    assert scipy.stats.chi2.sf(chi, dof) > 1e-3


def test_p12_poisson_special_means():
    assert all(oracle.poisson(0.0, 1, 0, j, 0) == 0 for j in range(50))
    for bad in (-1.0, float("nan"), float("inf")):
        assert oracle.poisson(bad, 1, 0, 0, 0) == -1


def test_p12_normal_distribution():
    g = np.array([oracle.normal(7, 1, j, 2) for j in range(20000)])
    assert scipy.stats.kstest(g, "norm").pvalue > 1e-3
    # different bins / points / seeds are different streams
    h = np.array([oracle.normal(7, 1, j, 3) for j in range(20000)])
    assert abs(np.corrcoef(g, h)[0, 1]) < 0.03


def test_p12_universes_covariance_and_batching():
    """Universes around S(p) have mean S(p) and covariance diag(S) + F o (S S^T)
    (Poisson plus fractional systematics); rows depend only on (p, j), so any
    split into batches gives the same values."""
    pr = fcgen.make_problem("c1", K=1, true_subset=[0], n_axis=(4, 4))
    p = 9
    M = 20000
    d, counts = oracle.universes(pr.S, pr.F, [p], [0, M], seed=11)
    s = pr.S[p]
    Sig = np.diag(s) + pr.F * np.outer(s, s)
    r = d - s
    se_mean = np.sqrt(np.diag(Sig) / M)
    assert np.all(np.abs(r.mean(axis=0)) <= 5 * se_mean)
    C = np.cov(r, rowvar=False)
    se = np.sqrt((np.outer(np.diag(Sig), np.diag(Sig)) + Sig ** 2) / M)
    assert np.all(np.abs(C - Sig) <= 5 * se)
    assert counts.min() >= 0 and np.all(counts == np.round(counts))
    # the Poisson part alone has variance S
    assert np.all(np.abs(counts.var(axis=0) - s) <= 5 * s * math.sqrt(2.0 / M))
    # batching: rows 300..499 drawn on their own equal the same rows of the whole
    d2, c2 = oracle.universes(pr.S, pr.F, [p], [0, 200], seed=11, u_first=[300])
    np.testing.assert_array_equal(d2, d[300:500])
    np.testing.assert_array_equal(c2, counts[300:500])


# --------------------------------------------------------------------------
# P13: the region with per-point universe counts
# --------------------------------------------------------------------------
def _region_problem():
    pr = fcgen.make_problem("c1", K=1, true_subset=[0], n_axis=(6, 6))
    c = fcgen.universes(pr.config, 40000, pr.S[14], pr.F, 1)[0]
    dd, _, _ = oracle.data_scan(pr.S, pr.F, c)
    return pr, dd


def test_p13_region_refining_everything_equals_one_draw():
    """With an unbounded band (it spans every value of the point) and a data
    value inside every point's range, each point is refined to K_max; the
    universes drawn in doubling rounds must give exactly the values of drawing
    0..K_max-1 at once (the stream depends only on (seed, p, j))."""
    pr, _ = _region_problem()
    dd = np.full(pr.G, 1.0)
    pts = np.array([0, 7, 14, 20])
    r = oracle.region(pr.S, pr.F, pts, 16, 128, 1e9, 3, (0.6827, 0.9), dd)
    assert np.all(r["K_used"] == 128) and r["rounds"] == 4
    assert r["evals"] == float((16 + 16 + 32 + 64) * len(pts) * pr.G)
    seg = np.arange(len(pts) + 1) * 128
    d, _ = oracle.universes(pr.S, pr.F, pts, seg, 3)
    s = oracle.scan(pr.S, pr.F, d, np.repeat(pts, 128))
    crit, _ = oracle.critical_value(s["dchi2"], seg, (0.6827, 0.9), with_hist=False)
    np.testing.assert_array_equal(r["crit"], crit)
    np.testing.assert_array_equal(r["accepted"], (dd[pts][:, None] <= crit).astype(np.uint8))


def test_p13_region_without_refinement():
    pr, dd = _region_problem()
    r = oracle.region(pr.S, pr.F, np.arange(pr.G), 40, 40, 0.0, 5, (0.9,), dd)
    assert r["rounds"] == 1 and np.all(r["K_used"] == 40)
    # a zero-width band still refines a point whose value equals x_(j)
    r2 = oracle.region(pr.S, pr.F, np.arange(pr.G), 40, 80, 0.0, 5, (0.9,), dd)
    hit = np.flatnonzero(r2["K_used"] == 80)
    assert np.all(np.abs(dd[hit] - r["crit"][hit, 0]) == 0.0)


def test_p13_region_coverage():
    """Data drawn at the true point are inside its region with probability
    alpha, also when the point's universe count adapts to the data."""
    pr = fcgen.make_problem("c1", K=1, true_subset=[0], n_axis=(5, 5))
    p = 12
    M = 200
    data = fcgen.universes(pr.config, 50000, pr.S[p], pr.F, M)
    alpha = (0.6827, 0.9)
    hits = np.zeros(2)
    for m in range(M):
        dd, _, _ = oracle.data_scan(pr.S, pr.F, data[m])
        r = oracle.region(pr.S, pr.F, [p], 50, 800, 2.0, 100 + m, alpha, dd)
        hits += r["accepted"][0]
    for a, al in enumerate(alpha):
        sigma = math.sqrt(al * (1 - al) / M + al * (1 - al) / 50)
        assert abs(hits[a] / M - al) <= 4 * sigma, (al, hits[a] / M)


# --------------------------------------------------------------------------
# P14: one matrix for the whole grid (Algorithm 1 as printed) and its
# iteration (Section 2, step 5)
# --------------------------------------------------------------------------
def _exact_fixed(S, F, d, p, max_iter):
    """Exact rational Algorithm 1 with M = Sigma_m^{-1} (Gauss-Jordan inverse),
    m starting at p and moved to q_min while it changes (at most max_iter)."""
    m, it = p, 0
    while True:
        Minv = exact_fc.inverse(exact_fc.covariance(S[m], F))
        vals = [exact_fc.chi2(d, Sq, Minv) for Sq in S]
        best, qmin = None, p
        for q, v in enumerate(vals):
            if best is None or v < best:
                best, qmin = v, q
        if it == max_iter or qmin == m:
            return vals[p] - best, best, qmin, vals[p], m, it
        m, it = qmin, it + 1


@pytest.mark.parametrize("max_iter", [0, 1, 10])
def test_p14_fixed_matrix_exact_rational(max_iter):
    S, F, d, p = _p1_problem()
    Sn = np.array(S, dtype=np.float64)
    Fn = np.array([[float(x) for x in row] for row in F])
    dn = np.array(d, dtype=np.float64)
    r = oracle.scan_fixed_m(Sn, Fn, dn, np.array(p), max_iter)
    n_moved = 0
    for k in range(len(d)):
        dc, cmin, am, cp, m, it = _exact_fixed(S, F, d[k], p[k], max_iter)
        scale = max(1.0, float(cp))
        assert r["argmin"][k] == am and r["m_final"][k] == m and r["iters"][k] == it
        assert abs(r["dchi2"][k] - float(dc)) <= 1e-14 * scale
        assert abs(r["chi2_min"][k] - float(cmin)) <= 1e-14 * scale
        assert abs(r["chi2_p"][k] - float(cp)) <= 1e-14 * scale
        n_moved += it > 0
    if max_iter > 0:
        assert n_moved > 0          # the iteration is exercised


def test_p14_fixed_matrix_reduces_to_per_point_scan():
    """With a covariance that does not depend on q (fixed statistical term,
    no fractional systematics) every variant is Algorithm 1 with that one
    matrix, so all must equal the per-point scan exactly."""
    pr = fcgen.make_problem("c1", K=300, true_subset=[0], n_axis=(9, 9))
    stat = np.linspace(40.0, 400.0, pr.N)
    F0 = np.zeros((pr.N, pr.N))
    ref = oracle.scan(pr.S, F0, pr.d, pr.p_idx, oracle.STAT_FIXED, stat)
    for it in (0, 3):
        r = oracle.scan_fixed_m(pr.S, F0, pr.d, pr.p_idx, it, oracle.STAT_FIXED, stat)
        for key in ("dchi2", "chi2_min", "argmin", "chi2_p"):
            np.testing.assert_array_equal(r[key], ref[key])
        assert np.all(r["iters"] <= 1)


def test_range_split_scan_equals_one_pass():
    """Algorithm 1's running minimum over the grid walked in consecutive q
    ranges (the oracle's memory-bounded path for large grids) is exactly the
    single pass: same values, same minimiser, same second-best."""
    pr = fcgen.make_problem("c1", K=40, true_subset=[0], n_axis=(12, 12))
    one = oracle.scan(pr.S, pr.F, pr.d, pr.p_idx)
    N = pr.N
    for pts_per_range in (1, 7, 50):
        many = oracle.scan(pr.S, pr.F, pr.d, pr.p_idx, block_bytes=8 * N * N * pts_per_range)
        for key in ("dchi2", "chi2_min", "argmin", "chi2_p", "chi2_2nd"):
            np.testing.assert_array_equal(many[key], one[key])
