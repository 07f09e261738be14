"""Exact rational evaluation of Eq. 1 (TEST INFRASTRUCTURE ONLY).

For tiny integer inputs, b_i = (X_i^T M^-1 X_i)^-1 X_i^T M^-1 y is computed
with ``fractions.Fraction`` and Gauss-Jordan elimination: no rounding at all,
no Cholesky and no whitening, so it pins the floating-point oracle from
outside.  The residual variance is the GLS residual
(y - X_i b_i)^T M^-1 (y - X_i b_i) / (n - p) and v_i = ((X_i^T M^-1 X_i)^-1)_pp,
both exact.  Pure-Python loops: keep n and p tiny.
"""
from __future__ import annotations

from fractions import Fraction


def _mat(rows):
    return [[Fraction(x) for x in r] for r in rows]


def inverse(A):
    """Gauss-Jordan inverse of a nonsingular square matrix of Fractions."""
    k = len(A)
    aug = [list(A[i]) + [Fraction(int(i == j)) for j in range(k)] for i in range(k)]
    for col in range(k):
        piv = next(r for r in range(col, k) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        pv = aug[col][col]
        aug[col] = [x / pv for x in aug[col]]
        for r in range(k):
            if r != col and aug[r][col] != 0:
                f = aug[r][col]
                aug[r] = [a - f * b for a, b in zip(aug[r], aug[col])]
    return [row[k:] for row in aug]


def matmul(A, B):
    return [[sum(A[i][t] * B[t][j] for t in range(len(B))) for j in range(len(B[0]))] for i in range(len(A))]


def transpose(A):
    return [list(r) for r in zip(*A)]


def gls_exact(M, XL, y, XR_cols):
    """M (n x n), XL (n x q), y (n), XR_cols: list of SNP columns (each n).

    Returns a list of (b, sigma2, v) per SNP, b a list of p Fractions.
    """
    M = _mat(M)
    n = len(M)
    XL = _mat(XL) if len(XL) and len(XL[0]) else [[] for _ in range(n)]
    y = [Fraction(v) for v in y]
    Mi = inverse(M)
    out = []
    for x in XR_cols:
        X = [XL[r] + [Fraction(x[r])] for r in range(n)]
        p = len(X[0])
        XtMi = matmul(transpose(X), Mi)
        A = matmul(XtMi, X)
        g = [row[0] for row in matmul(XtMi, [[v] for v in y])]
        Ai = inverse(A)
        b = [sum(Ai[i][j] * g[j] for j in range(p)) for i in range(p)]
        res = [y[r] - sum(X[r][j] * b[j] for j in range(p)) for r in range(n)]
        Mres = [sum(Mi[r][t] * res[t] for t in range(n)) for r in range(n)]
        rss = sum(res[r] * Mres[r] for r in range(n))
        out.append((b, rss / (n - p), Ai[p - 1][p - 1]))
    return out
