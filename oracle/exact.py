"""Exact rational brute force for tiny GLS problems.

TEST INFRASTRUCTURE (see gls_oracle.py).  For integer-valued inputs with n up
to about a dozen, b_i of Eq. (1) is computed with Python fractions: M^{-1} by
Gauss-Jordan elimination, then A_i = X_i^T M^{-1} X_i and r_i = X_i^T M^{-1} y,
then b_i = A_i^{-1} r_i, again by Gauss-Jordan.  No rounding happens anywhere,
so the result is the true b_i and pins the floating-point oracle.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence

Matrix = List[List[Fraction]]


def to_fractions(A) -> Matrix:
    return [[Fraction(int(v)) if float(v).is_integer() else Fraction(float(v)) for v in row]
            for row in A]


def inverse(A: Matrix) -> Matrix:
    """Gauss-Jordan inverse with a nonzero-pivot search (exact arithmetic)."""
    n = len(A)
    aug = [list(A[i]) + [Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if aug[r][c] != 0)
        aug[c], aug[piv] = aug[piv], aug[c]
        pv = aug[c][c]
        aug[c] = [v / pv for v in aug[c]]
        for r in range(n):
            if r != c and aug[r][c] != 0:
                f = aug[r][c]
                aug[r] = [a - f * b for a, b in zip(aug[r], aug[c])]
    return [row[n:] for row in aug]


def matmul(A: Matrix, B: Matrix) -> Matrix:
    return [[sum((A[i][k] * B[k][j] for k in range(len(B))), Fraction(0))
             for j in range(len(B[0]))] for i in range(len(A))]


def transpose(A: Matrix) -> Matrix:
    return [list(r) for r in zip(*A)]


def gls_exact(M, XL, XR, Y, p_R: int = 1) -> List[List[List[Fraction]]]:
    """Exact b_i for every problem; returns out[i][j] = b_i (list of p
    Fractions) for phenotype j.  Inputs are row-indexable 2-D arrays with
    M n x n, X_L n x p_L, X_R n x (m p_R), Y n x t."""
    Mf = to_fractions(M)
    XLf = to_fractions(XL)
    XRf = to_fractions(XR)
    Yf = to_fractions(Y)
    n = len(Mf)
    Minv = inverse(Mf)
    m = len(XRf[0]) // p_R
    out = []
    for i in range(m):
        Xi = [XLf[r] + XRf[r][i * p_R:(i + 1) * p_R] for r in range(n)]
        XtMinv = matmul(transpose(Xi), Minv)
        A = matmul(XtMinv, Xi)
        rhs = matmul(XtMinv, Yf)
        b = matmul(inverse(A), rhs)          # p x t
        out.append([[b[k][j] for k in range(len(b))] for j in range(len(Yf[0]))])
    return out
