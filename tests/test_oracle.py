"""Pins for the CPU oracle: each checks it against something other than itself
(exact rationals, a textbook closed form, a library least-squares routine,
the paper's alternative algorithms, invariances of Eq. (1))."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import gls_oracle as orc
from oracle.exact import gls_exact

HERE = os.path.dirname(os.path.abspath(__file__))


def rand_problem(rng, n=40, p_L=3, p_R=1, m=12, t=1, cond=1.0):
    A = rng.standard_normal((n, n))
    M = A @ A.T / n + cond * np.eye(n)
    XL = np.hstack([np.ones((n, 1)), rng.standard_normal((n, p_L - 1))])
    XR = rng.integers(0, 3, (n, m * p_R)).astype(np.int8)
    Y = rng.standard_normal((n, t))
    return M, XL, XR, Y


def maxrel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


# --- exact rationals ---------------------------------------------------------
def _frac(s):
    a, b = s.split("/")
    return Fraction(int(a), int(b))


def test_golden_exact_fixtures():
    doc = json.load(open(os.path.join(HERE, "golden", "tiny_exact.json")))
    assert len(doc["cases"]) >= 5
    for c in doc["cases"]:
        M, XL, XR, Y = (np.array(c[k], dtype=np.float64) for k in ("M", "XL", "XR", "Y"))
        ref = np.array([[[float(_frac(v)) for v in bj] for bj in bi] for bi in c["b"]])
        got = orc.gls_sequence(M, XL, XR, Y, c["p_R"])
        assert got.shape == ref.shape
        assert np.max(orc.relative_error(got, ref)) < 1e-13


@pytest.mark.parametrize("seed,p_R,t", [(11, 1, 1), (12, 2, 2), (13, 1, 3)])
def test_exact_bruteforce_random(seed, p_R, t):
    rng = np.random.default_rng(seed)
    n = 9
    A = rng.integers(-4, 5, (n, n))
    M = A @ A.T + n * np.eye(n, dtype=np.int64)
    XL = np.hstack([np.ones((n, 1), np.int64), rng.integers(-3, 4, (n, 2))])
    XR = rng.integers(0, 3, (n, 3 * p_R))
    Y = rng.integers(-9, 10, (n, t))
    ex = gls_exact(M, XL, XR, Y, p_R)
    ref = np.array([[[float(v) for v in bj] for bj in bi] for bi in ex])
    got = orc.gls_sequence(M, XL, XR, Y, p_R)
    assert np.max(orc.relative_error(got, ref)) < 1e-13


# --- closed forms and library routines ----------------------------------------
def test_identity_covariance_is_ordinary_least_squares():
    rng = np.random.default_rng(3)
    n, m = 50, 10
    _, XL, XR, Y = rand_problem(rng, n=n, m=m)
    got = orc.gls_sequence(np.eye(n), XL, XR, Y)
    for i in range(m):
        Xi = np.hstack([XL, XR[:, i:i + 1].astype(np.float64)])
        ref, *_ = np.linalg.lstsq(Xi, Y[:, 0], rcond=None)
        assert maxrel(got[i, 0], ref) < 1e-12


def test_frisch_waugh_lovell_closed_form():
    """b_R = (x^T P y)/(x^T P x), P = M^-1 - M^-1 X_L (X_L^T M^-1 X_L)^-1 X_L^T M^-1."""
    rng = np.random.default_rng(4)
    M, XL, XR, Y = rand_problem(rng, n=60, m=8)
    Mi = np.linalg.inv(M)
    P = Mi - Mi @ XL @ np.linalg.inv(XL.T @ Mi @ XL) @ XL.T @ Mi
    got = orc.gls_sequence(M, XL, XR, Y)
    for i in range(8):
        x = XR[:, i].astype(np.float64)
        ref = (x @ P @ Y[:, 0]) / (x @ P @ x)
        assert abs(got[i, 0, -1] - ref) <= 1e-11 * abs(ref) + 1e-14


def test_normal_equation_residual_vanishes():
    rng = np.random.default_rng(5)
    M, XL, XR, Y = rand_problem(rng, n=80, p_L=4, p_R=2, m=6, t=2)
    B = orc.gls_sequence(M, XL, XR, Y, p_R=2)
    res = orc.normal_equation_residual(M, XL, XR, Y, B, p_R=2)
    assert res.max() < 1e-13


def _exact_norm_inf(A):
    """Max row sum of absolute values, exact (Fractions)."""
    return max(sum(abs(v) for v in row) for row in A)


def _residual_vs_exact(resid_fn):
    """Checks a normal-equation residual function against exact arithmetic on
    the golden cases; returns (largest value at the exact b, largest
    relative mismatch at perturbed and wrong-model b, smallest exact value).

    With b_i = b*_i + delta (b*_i the exact solution), the residual of the
    normal equations is X_i^T M^-1 (y - X_i b_i) = -S_i delta exactly, with
    S_i = X_i^T M^-1 X_i: its value is computed here from S_i and delta in
    rationals, not by evaluating the residual's own formula."""
    from oracle.exact import inverse, matmul, to_fractions, transpose
    doc = json.load(open(os.path.join(HERE, "golden", "tiny_exact.json")))
    rng = np.random.default_rng(21)
    at_exact, mismatch, smallest = 0.0, 0.0, np.inf
    for c in doc["cases"]:
        M, XL, XR, Y = (np.array(c[k], dtype=np.float64) for k in ("M", "XL", "XR", "Y"))
        p_R, t = c["p_R"], c["t"]
        bstar = [[[_frac(v) for v in bj] for bj in bi] for bi in c["b"]]
        B0 = np.array([[[float(v) for v in bj] for bj in bi] for bi in bstar])
        at_exact = max(at_exact, float(np.max(resid_fn(M, XL, XR, Y, B0, p_R))))
        # the wrong model: b solved with M instead of M^-1
        Bw = np.empty_like(B0)
        for i in range(B0.shape[0]):
            Xi = np.hstack([XL, XR[:, i * p_R:(i + 1) * p_R]])
            Bw[i] = np.linalg.solve(Xi.T @ M @ Xi, Xi.T @ M @ Y).T
        Bp = B0 * (1.0 + 1e-6 * rng.standard_normal(B0.shape))
        Mi = inverse(to_fractions(M))
        XLf, XRf, Yf = to_fractions(XL), to_fractions(XR), to_fractions(Y)
        n = len(XLf)
        for Bt in (Bp, Bw):
            got = resid_fn(M, XL, XR, Y, Bt, p_R)
            for i in range(Bt.shape[0]):
                Xi = [XLf[r] + XRf[r][i * p_R:(i + 1) * p_R] for r in range(n)]
                XtMi = matmul(transpose(Xi), Mi)
                S = matmul(XtMi, Xi)
                for j in range(t):
                    bt = [Fraction(float(v)) for v in Bt[i, j]]
                    delta = [[bt[r] - bstar[i][j][r]] for r in range(len(bt))]
                    res = [abs(v[0]) for v in matmul(S, delta)]
                    scale = _exact_norm_inf(XtMi) * max(abs(Yf[r][j]) for r in range(n)) \
                        + _exact_norm_inf(S) * max(abs(v) for v in bt)
                    want = float(max(res) / scale)
                    smallest = min(smallest, want)
                    mismatch = max(mismatch, abs(float(got[i, j]) - want) / want)
    return at_exact, mismatch, smallest


def test_normal_equation_residual_pinned_by_exact_rationals():
    """The exact b* (rounded to FP64) gives <= 1e-13; a perturbed b
    (relative 1e-6) and the b of the wrong model (M in place of M^-1) give
    the exact relative residual (to 1e-6 of its value), far above 1e-8."""
    at_exact, mismatch, smallest = _residual_vs_exact(orc.normal_equation_residual)
    assert at_exact <= 1e-13
    assert smallest > 1e-9
    assert mismatch <= 1e-6


def test_normal_equation_residual_planted_mistakes():
    """Plausible mistakes in the residual, planted in copies on the CPU, fail
    the exact pin: a residual that is always zero, M not inverted, and a
    scale missing its ||S|| ||b|| term."""
    import scipy.linalg as sla

    def variant(kind):
        def fn(M, XL, XR, Y, B, p_R=1):
            Y = np.asarray(Y, dtype=np.float64).reshape(M.shape[0], -1)
            lu = sla.lu_factor(M)
            res = np.empty(B.shape[:2])
            for i in range(B.shape[0]):
                Xi = np.hstack([XL, np.asarray(XR[:, i * p_R:(i + 1) * p_R], dtype=np.float64)])
                Wt = (M @ Xi).T if kind == "M_not_inverted" else sla.lu_solve(lu, Xi).T
                S = Wt @ Xi
                for j in range(Y.shape[1]):
                    r = Wt @ (Y[:, j] - Xi @ B[i, j])
                    scale = np.linalg.norm(Wt, np.inf) * np.linalg.norm(Y[:, j], np.inf)
                    if kind != "scale_term_dropped":
                        scale += np.linalg.norm(S, np.inf) * np.linalg.norm(B[i, j], np.inf)
                    res[i, j] = 0.0 if kind == "zero" else np.linalg.norm(r, np.inf) / scale
            return res
        return fn

    at_exact, mismatch, _ = _residual_vs_exact(variant("none"))
    assert at_exact <= 1e-13 and mismatch <= 1e-6
    for kind in ("zero", "M_not_inverted", "scale_term_dropped"):
        at_exact, mismatch, _ = _residual_vs_exact(variant(kind))
        assert at_exact > 1e-13 or mismatch > 1e-3, kind


# --- invariances of Eq. (1) ---------------------------------------------------
def test_invariances():
    rng = np.random.default_rng(6)
    M, XL, XR, Y = rand_problem(rng, n=50, p_L=3, m=7, t=1)
    b0 = orc.gls_sequence(M, XL, XR, Y)
    # permuting individuals
    perm = rng.permutation(50)
    b1 = orc.gls_sequence(M[np.ix_(perm, perm)], XL[perm], XR[perm], Y[perm])
    assert maxrel(b1, b0) < 1e-11
    # y -> alpha y scales b; M -> alpha M leaves b
    assert maxrel(orc.gls_sequence(M, XL, XR, 3.5 * Y), 3.5 * b0) < 1e-12
    assert maxrel(orc.gls_sequence(2.25 * M, XL, XR, Y), b0) < 1e-12
    # y -> y + X_L gamma shifts b_L by gamma
    gamma = np.array([0.5, -2.0, 1.25])
    b2 = orc.gls_sequence(M, XL, XR, Y + (XL @ gamma)[:, None])
    shifted = b0.copy()
    shifted[:, 0, :3] += gamma
    assert maxrel(b2, shifted) < 1e-11
    # scaling a genotype column by s scales b_R by 1/s
    b3 = orc.gls_sequence(M, XL, 4.0 * XR.astype(np.float64), Y)
    assert maxrel(b3[:, 0, 3], b0[:, 0, 3] / 4.0) < 1e-12
    assert maxrel(b3[:, 0, :3], b0[:, 0, :3]) < 1e-11
    # problem order permutes outputs only
    order = rng.permutation(7)
    b4 = orc.gls_sequence(M, XL, XR[:, order], Y)
    assert maxrel(b4, b0[order]) < 1e-13


# --- the paper's alternative algorithms reach the same b_i ---------------------
def _alg_gels(M, XL, xr, y):
    """Alg. 1: whiten with the Cholesky factor, then least squares (QR)."""
    L = np.linalg.cholesky(M)
    X = sla.solve_triangular(L, np.hstack([XL, xr]), lower=True)
    yt = sla.solve_triangular(L, y, lower=True)
    q, r = np.linalg.qr(X)
    return sla.solve_triangular(r, q.T @ yt)


def _alg_blackbox(M, XL, xr, y):
    """Alg. 3: potrf, trsm, trsv, syrk, gemv, posv for one problem."""
    L = np.linalg.cholesky(M)
    X = sla.solve_triangular(L, np.hstack([XL, xr]), lower=True)
    yt = sla.solve_triangular(L, y, lower=True)
    S = X.T @ X
    return sla.cho_solve(sla.cho_factor(S, lower=True), X.T @ yt)


def _alg_gwfgls(M, XL, xr, y):
    """Alg. 6: explicit inverse of M, W^T = X^T M^-1, S = W^T X, b = S^-1 W^T y."""
    Mi = np.linalg.inv(M)
    X = np.hstack([XL, xr])
    Wt = X.T @ Mi
    return np.linalg.solve(Wt @ X, Wt @ y)


def _alg_hp_gwas(M, XL, XR, y, p_R):
    """Alg. 5 on the CPU: factor once, whiten X_L, y and all of X_R once,
    assemble S_i from S_TL and per-problem products, then posv."""
    L = np.linalg.cholesky(M)
    WL = sla.solve_triangular(L, XL, lower=True)
    WR = sla.solve_triangular(L, XR.astype(np.float64), lower=True)
    yt = sla.solve_triangular(L, y, lower=True)
    STL, bT = WL.T @ WL, WL.T @ yt
    out = []
    for i in range(XR.shape[1] // p_R):
        w = WR[:, i * p_R:(i + 1) * p_R]
        SBL = w.T @ WL
        S = np.block([[STL, SBL.T], [SBL, w.T @ w]])
        out.append(sla.cho_solve(sla.cho_factor(S, lower=True), np.concatenate([bT, w.T @ yt])))
    return np.array(out)


def test_cross_routes_agree():
    rng = np.random.default_rng(7)
    M, XL, XR, Y = rand_problem(rng, n=70, p_L=3, p_R=1, m=9, t=1)
    b0 = orc.gls_sequence(M, XL, XR, Y)[:, 0]
    y = Y[:, 0]
    for i in range(9):
        xr = XR[:, i:i + 1].astype(np.float64)
        for alg in (_alg_gels, _alg_blackbox, _alg_gwfgls):
            assert maxrel(alg(M, XL, xr, y), b0[i]) < 1e-11
    assert maxrel(_alg_hp_gwas(M, XL, XR, y, 1), b0) < 1e-11


@pytest.mark.parametrize("p_R,t,block", [(1, 1, 4), (2, 3, 5), (3, 2, 100)])
def test_host_hp_gwas_matches_definition(p_R, t, block):
    """The benchmark's host version of Alg. 5 (timed as a context figure)
    reaches the definition's b_i, across block boundaries."""
    import bench
    rng = np.random.default_rng(11 + p_R)
    M, XL, XR, Y = rand_problem(rng, n=60, p_L=3, p_R=p_R, m=11, t=t)
    ref = orc.gls_sequence(M, XL, XR, Y, p_R)
    got = bench.host_alg5(M, XL, XR, Y, p_R, block=block)
    assert got.shape == ref.shape
    assert maxrel(got, ref) < 1e-11


# --- intermediate quantities ----------------------------------------------------
def test_cholesky_pins():
    rng = np.random.default_rng(8)
    M, *_ = rand_problem(rng, n=64)
    L = orc.cholesky_lower(M)
    assert np.allclose(np.triu(L, 1), 0)
    assert np.all(np.diag(L) > 0)
    assert np.linalg.norm(L @ L.T - M) / np.linalg.norm(M) < 1e-14
    d = rng.uniform(0.5, 3.0, 10)
    assert np.allclose(orc.cholesky_lower(np.diag(d)), np.diag(np.sqrt(d)), rtol=1e-15)


def test_whiten_and_fixed_blocks():
    rng = np.random.default_rng(9)
    M, XL, XR, Y = rand_problem(rng, n=64, p_L=4)
    L = orc.cholesky_lower(M)
    W = orc.whiten(L, XR)
    assert np.linalg.norm(L @ W - XR) / (np.linalg.norm(L) * np.linalg.norm(W)) < 1e-14
    WL, yt, STL, CT = orc.fixed_blocks(L, XL, Y)
    Mi = np.linalg.inv(M)
    assert maxrel(STL, XL.T @ Mi @ XL) < 1e-12
    assert maxrel(CT, XL.T @ Mi @ Y) < 1e-12


def test_relative_error_definition():
    a = np.array([[[1.0, -2.0, 4.0]]])
    b = np.array([[[1.0, -2.0, 3.0]]])
    assert orc.relative_error(a, b)[0, 0] == pytest.approx(1.0 / 3.0)


def test_planted_mistakes_are_caught():
    """Plausible oracle mistakes (dropped block, transposed operand, wrong
    sign) must fail the exact pin; they are planted in copies on the CPU."""
    doc = json.load(open(os.path.join(HERE, "golden", "tiny_exact.json")))
    c = doc["cases"][1]
    M, XL, XR, Y = (np.array(c[k], dtype=np.float64) for k in ("M", "XL", "XR", "Y"))
    ref = np.array([[[float(_frac(v)) for v in bj] for bj in bi] for bi in c["b"]])
    n, p_L = XL.shape

    def variant(kind):
        Mi = np.linalg.inv(M)
        out = []
        for i in range(XR.shape[1]):
            Xi = np.hstack([XL, XR[:, i:i + 1]])
            if kind == "transposed_factor":
                # whitening with L^-T instead of L^-1
                L = np.linalg.cholesky(M)
                W = sla.solve_triangular(L.T, Xi, lower=False)
                yt = sla.solve_triangular(L.T, Y, lower=False)
                A, r = W.T @ W, W.T @ yt
            elif kind == "M_not_inverted":
                A, r = Xi.T @ M @ Xi, Xi.T @ M @ Y
            elif kind == "dropped_cross_block":
                A = Xi.T @ Mi @ Xi
                A[:p_L, p_L:] = 0
                A[p_L:, :p_L] = 0
                r = Xi.T @ Mi @ Y
            elif kind == "sign":
                A, r = Xi.T @ Mi @ Xi, -(Xi.T @ Mi @ Y)
            else:
                A, r = Xi.T @ Mi @ Xi, Xi.T @ Mi @ Y
            out.append(np.linalg.solve(A, r).T)
        return np.array(out)

    assert np.max(orc.relative_error(variant("none"), ref)) < 1e-12
    for kind in ("transposed_factor", "M_not_inverted", "dropped_cross_block", "sign"):
        assert np.max(orc.relative_error(variant(kind), ref)) > 1e-6, kind
