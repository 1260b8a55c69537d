"""Exact-rational brute force of the grid scan for tiny problems (test helper).

Independent of the oracle: rational arithmetic (``fractions.Fraction``), the
covariance is inverted by Gauss-Jordan elimination rather than factored, and
chi^2 = r^T Sigma^{-1} r is taken literally as in Eq. (1).  The minimum follows
Algorithm 1 (strict "<" in grid order, starting from +inf with the minimiser
set to the true point).
"""
from __future__ import annotations

from fractions import Fraction


def covariance(s, F, stat=None):
    """Sigma = diag(stat or s) + F o (s s^T) in exact arithmetic."""
    N = len(s)
    st = s if stat is None else stat
    return [[F[i][j] * s[i] * s[j] + (st[i] if i == j else 0) for j in range(N)]
            for i in range(N)]


def inverse(A):
    """Gauss-Jordan inverse of a rational matrix (raises on a zero pivot)."""
    n = len(A)
    M = [list(map(Fraction, row)) + [Fraction(int(i == j)) for j in range(n)]
         for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        pv = M[c][c]
        M[c] = [v / pv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [row[n:] for row in M]


def chi2(a, b, Minv):
    r = [x - y for x, y in zip(a, b)]
    n = len(r)
    return sum(r[i] * Minv[i][j] * r[j] for i in range(n) for j in range(n))


def scan(S, F, d, p_idx, stat=None):
    """Return per-universe (dchi2, chi2_min, argmin, chi2_p, chi2_2nd) as Fractions.

    chi2_2nd is the smallest chi^2 over grid points other than argmin (None
    for a one-point grid)."""
    Minv = [inverse(covariance(Sq, F, stat)) for Sq in S]
    out = []
    for a, p in zip(d, p_idx):
        best, qbest = None, p          # None stands for +inf
        vals = []
        for q, Sq in enumerate(S):
            c = chi2(a, Sq, Minv[q])
            vals.append(c)
            if best is None or c < best:
                best, qbest = c, q
        others = [v for q, v in enumerate(vals) if q != qbest]
        out.append((vals[p] - best, best, qbest, vals[p], min(others) if others else None))
    return out
