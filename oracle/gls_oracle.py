"""Oracle for the sequence of generalized least-squares problems.

TEST INFRASTRUCTURE.  Plain, slow, FP64 CPU reference of what the GPU path
computes.  Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import it; the product path never does, and this module
shares no code with it.

What is computed (Sec. 1, Eq. (1)): for i = 1..m,

    b_i = (X_i^T M^{-1} X_i)^{-1} X_i^T M^{-1} y,     X_i = (X_L | X_{R_i}),

with M symmetric positive definite and every X_i of full column rank, so each
b_i is unique.  The oracle writes that definition out; it does not follow the
paper's fast algorithm (Sec. 2, Alg. "hp-gwas"), which reaches the same b_i.

Library primitives used as single steps: an LU factorization with partial
pivoting of M and its triangular solves (scipy's lu_factor / lu_solve), a
batched matrix product, and a small dense solve with partial pivoting
(numpy.linalg.solve).  Nothing is blocked, fused or reordered beyond that.

Conventions: column-major inputs as numpy arrays of shape (rows, cols); M is
n x n, X_L n x p_L, Y n x t, X_R n x (m*p_R) with problem i owning columns
i*p_R .. i*p_R+p_R-1.  Outputs have shape (m, t, p): out[i, j, :] = b_i for
phenotype j, ordered (b_L; b_R) like the columns of X_i.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _snp_chunk(n: int, p: int) -> int:
    # bound the batched arrays (chunk, n, p) to about 64 MB each
    return max(1, int((64 << 20) // (8 * n * p)))


def gls_sequence(M, XL, XR, Y, p_R: int = 1, lu=None) -> np.ndarray:
    """b_i from the definition, Eq. (1), for every problem in X_R.

    Per problem: V_i = M^{-1} X_i and v = M^{-1} y by LU solves,
    A_i = X_i^T V_i and r_i = X_i^T v formed in full (no symmetry used),
    then b_i = A_i^{-1} r_i by a partial-pivoting solve."""
    M = np.asarray(M, dtype=np.float64)
    XL = np.asarray(XL, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    if Y.ndim == 1:
        Y = Y[:, None]
    n, p_L = XL.shape
    t = Y.shape[1]
    ncols = XR.shape[1]
    assert ncols % p_R == 0
    m = ncols // p_R
    p = p_L + p_R
    if lu is None:
        lu = sla.lu_factor(M)
    VL = sla.lu_solve(lu, XL)
    Vy = sla.lu_solve(lu, Y)
    out = np.empty((m, t, p), dtype=np.float64)
    step = _snp_chunk(n, p)
    for a in range(0, m, step):
        b = min(m, a + step)
        xr = np.asarray(XR[:, a * p_R:b * p_R], dtype=np.float64)
        vr = sla.lu_solve(lu, xr)
        k = b - a
        # X_i and V_i = M^{-1} X_i for the problems of this chunk: (k, n, p)
        X = np.empty((k, n, p))
        V = np.empty((k, n, p))
        X[:, :, :p_L] = XL[None]
        V[:, :, :p_L] = VL[None]
        X[:, :, p_L:] = xr.T.reshape(k, p_R, n).transpose(0, 2, 1)
        V[:, :, p_L:] = vr.T.reshape(k, p_R, n).transpose(0, 2, 1)
        Xt = X.transpose(0, 2, 1)
        A = np.matmul(Xt, V)                  # X_i^T M^{-1} X_i   (k, p, p)
        r = np.matmul(Xt, Vy[None])           # X_i^T M^{-1} y     (k, p, t)
        bi = np.linalg.solve(A, r)            # (k, p, t)
        out[a:b] = bi.transpose(0, 2, 1)
    return out


def cholesky_lower(M) -> np.ndarray:
    """The unique lower-triangular L with positive diagonal and L L^T = M
    (the factorization that starts the paper's algorithms, Alg. 3-5)."""
    return np.linalg.cholesky(np.asarray(M, dtype=np.float64))


def whiten(L, X) -> np.ndarray:
    """L^{-1} X for lower-triangular L (the trsm / trsv steps of Alg. 5)."""
    return sla.solve_triangular(np.asarray(L, dtype=np.float64),
                                np.asarray(X, dtype=np.float64), lower=True)


def fixed_blocks(L, XL, Y):
    """Quantities shared by every problem (Alg. 5 and Fig. 1):
    W_L = L^{-1} X_L, ytil = L^{-1} y, S_TL = W_L^T W_L, C_T = W_L^T ytil."""
    WL = whiten(L, XL)
    yt = whiten(L, np.asarray(Y, dtype=np.float64).reshape(L.shape[0], -1))
    return WL, yt, WL.T @ WL, WL.T @ yt


def relative_error(b_hat, b_ref) -> np.ndarray:
    """Per problem and phenotype: ||b_hat - b_ref||_inf / ||b_ref||_inf."""
    b_hat = np.asarray(b_hat, dtype=np.float64)
    b_ref = np.asarray(b_ref, dtype=np.float64)
    num = np.max(np.abs(b_hat - b_ref), axis=-1)
    den = np.max(np.abs(b_ref), axis=-1)
    return num / den


def normal_equation_residual(M, XL, XR, Y, B, p_R: int = 1) -> np.ndarray:
    """Relative residual of the normal equations X_i^T M^{-1}(y - X_i b_i) = 0,
    per problem and phenotype, scaled by ||X_i^T M^{-1}|| ||y|| + ||X_i^T M^{-1} X_i|| ||b_i||."""
    M = np.asarray(M, dtype=np.float64)
    XL = np.asarray(XL, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64).reshape(M.shape[0], -1)
    lu = sla.lu_factor(M)
    m = B.shape[0]
    res = np.empty(B.shape[:2])
    for i in range(m):
        Xi = np.hstack([XL, np.asarray(XR[:, i * p_R:(i + 1) * p_R], dtype=np.float64)])
        Wt = sla.lu_solve(lu, Xi).T            # X_i^T M^{-1}
        S = Wt @ Xi
        for j in range(Y.shape[1]):
            r = Wt @ (Y[:, j] - Xi @ B[i, j])
            scale = np.linalg.norm(Wt, np.inf) * np.linalg.norm(Y[:, j], np.inf) \
                + np.linalg.norm(S, np.inf) * np.linalg.norm(B[i, j], np.inf)
            res[i, j] = np.linalg.norm(r, np.inf) / scale
    return res
