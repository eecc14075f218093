"""Synthetic GWAS inputs, seeded and counter-based.

This module generates inputs only and holds none of the GLS method's
arithmetic.  It serves the HIP path, the test suite and the benchmark alike.

Shapes and distributions follow the workloads the paper targets (Sec. 1,
Eq. (1): n about 10^4 individuals, 1 <= p <= 20, millions of problems) with
a kinship-style covariance M = h*Phi + (1-h)*I + 1e-3*I, where
Phi = Z Z^T / q is built from q standardized Binomial(2, f) genotypes.

Random numbers come from a counter-based generator (the splitmix64 output
function of Steele, Lea and Flood, OOPSLA 2014, applied to a counter):

    K(seed, stream)     = mix64(mix64(seed) + stream)
    Kc(seed, stream, j) = mix64(K ^ ((j + 1) * GOLDEN))
    draw(..., i)        = mix64(Kc + (i + 1) * GOLDEN)
    uniform             = (draw >> 11) * 2**-53

so genotype column j is the same whatever block it is generated in.  The C
twin (csrc/datagen.c, loaded when built) must agree with this numpy code bit
for bit; the test suite checks that.

Streams: 1 maf of X_R, 2 genotypes of X_R, 3 maf of Z, 4 genotypes of Z,
5 covariates of X_L, 6 phenotypes Y, 7 serving arrivals and job parameters.

Matrices are returned column-major (numpy Fortran order, shape (rows, cols)).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional, Tuple

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MASTER_SEED = 12107325

S_MAF_R, S_XR, S_MAF_Z, S_Z, S_XL, S_Y, S_SERVE = 1, 2, 3, 4, 5, 6, 7


def _mix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _stream_key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        return _mix64(_mix64(np.uint64(seed)) + np.uint64(stream))


def _column_keys(skey, cols) -> np.ndarray:
    cols = np.asarray(cols, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix64(skey ^ ((cols + np.uint64(1)) * GOLDEN))


def _unit(ckeys, idx) -> np.ndarray:
    """u[j, i] for column keys ckeys[j] and draw indices idx[i]."""
    ck = np.asarray(ckeys, dtype=np.uint64)[:, None]
    ii = np.asarray(idx, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        d = _mix64(ck + (ii + np.uint64(1)) * GOLDEN)
    return (d >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


# ----------------------------------------------------------------------------
# optional C twin
_CLIB = None


def _clib():
    global _CLIB
    if _CLIB is None:
        path = os.path.join(os.path.dirname(__file__), "libglsgen.so")
        if os.path.exists(path):
            lib = ctypes.CDLL(path)
            lib.gen_maf.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_void_p]
            lib.gen_genotypes.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64]
            lib.gen_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.c_int64]
            _CLIB = lib
        else:
            _CLIB = False
    return _CLIB or None


_DLIB = None


def _dlib():
    global _DLIB
    if _DLIB is None:
        path = os.path.join(os.path.dirname(__file__), "libglsgen_dev.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built")
        lib = ctypes.CDLL(path)
        lib.gen_genotypes_dev.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p]
        lib.gen_genotypes_dev.restype = ctypes.c_int
        _DLIB = lib
    return _DLIB


def make_XR_device(w: "Workload", snp0: int, nsnp: int, out, stream: int = 0) -> None:
    """Genotypes of problems snp0.. generated in device memory: `out` is a
    device int8 column-major (n, >= nsnp*p_R) tensor; `stream` a hipStream_t.
    Bit-identical to make_XR (the device twin of the same generator)."""
    assert out.dtype.__str__() == "torch.int8" and out.stride(0) == 1
    ld = out.stride(1) if out.shape[1] > 1 else w.n
    rc = _dlib().gen_genotypes_dev(w.seed, S_MAF_R, S_XR, w.maf_R[0], w.maf_R[1], w.n,
                                   snp0 * w.p_R, nsnp * w.p_R, out.data_ptr(), ld, stream)
    if rc != 0:
        raise RuntimeError(f"gen_genotypes_dev failed ({rc})")


def maf(seed: int, stream: int, lo: float, hi: float, col0: int, ncols: int,
        use_c: Optional[bool] = None) -> np.ndarray:
    """Minor-allele frequencies f_j = lo + (hi - lo) * u_j of columns col0.."""
    lib = _clib() if use_c in (None, True) else None
    if use_c and lib is None:
        raise RuntimeError("libglsgen.so is not built")
    if lib is not None:
        out = np.empty(ncols, dtype=np.float64)
        lib.gen_maf(seed, stream, lo, hi, col0, ncols, out.ctypes.data)
        return out
    sk = _stream_key(seed, stream)
    u = _unit(_column_keys(sk, np.arange(col0, col0 + ncols)), [0])[:, 0]
    return lo + (hi - lo) * u


def genotypes(seed: int, stream_maf: int, stream_g: int, lo: float, hi: float,
              n: int, col0: int, ncols: int, use_c: Optional[bool] = None,
              out: Optional[np.ndarray] = None) -> np.ndarray:
    """Binomial(2, f_j) genotypes, int8, column-major n x ncols (Fortran order).

    If `out` is given it must be a C-contiguous int8 array of shape
    (ncols, ld) with ld >= n; column j is written to out[j, :n]."""
    lib = _clib() if use_c in (None, True) else None
    if use_c and lib is None:
        raise RuntimeError("libglsgen.so is not built")
    if out is None:
        buf = np.empty((ncols, n), dtype=np.int8)
    else:
        buf = out
        assert buf.dtype == np.int8 and buf.flags.c_contiguous and buf.shape[0] >= ncols
    ld = buf.shape[1]
    if lib is not None and ncols > 0:
        lib.gen_genotypes(seed, stream_maf, stream_g, lo, hi, n, col0, ncols,
                          buf.ctypes.data, ld)
    else:
        f = maf(seed, stream_maf, lo, hi, col0, ncols, use_c=False)
        ck = _column_keys(_stream_key(seed, stream_g), np.arange(col0, col0 + ncols))
        # chunk over columns to bound memory
        step = max(1, (1 << 22) // max(n, 1))
        for a in range(0, ncols, step):
            b = min(ncols, a + step)
            u = _unit(ck[a:b], np.arange(2 * n))
            g = (u[:, 0::2] < f[a:b, None]).astype(np.int8) + (u[:, 1::2] < f[a:b, None]).astype(np.int8)
            buf[a:b, :n] = g
    return buf[:ncols, :n].T


def normals(seed: int, stream: int, n: int, col0: int, ncols: int) -> np.ndarray:
    """N(0,1) by Box-Muller from draws 2r, 2r+1; column-major n x ncols."""
    ck = _column_keys(_stream_key(seed, stream), np.arange(col0, col0 + ncols))
    u = _unit(ck, np.arange(2 * n))
    u1, u2 = u[:, 0::2], u[:, 1::2]
    z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
    return np.asfortranarray(z.T)


# ----------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic GWAS workload (all sizes explicit)."""
    name: str
    n: int                 # individuals
    p_L: int               # fixed columns (intercept + covariates)
    p_R: int               # genotype columns per problem
    t: int                 # phenotypes sharing M
    m: int                 # problems (SNPs)
    block: int             # SNPs per solve call
    q: int                 # genotypes behind Phi
    h: float               # heritability weight of Phi
    maf_R: Tuple[float, float] = (0.05, 0.5)
    maf_Z: Tuple[float, float] = (0.05, 0.5)
    seed: int = MASTER_SEED
    diag_shift: float = 1e-3

    @property
    def p(self) -> int:
        return self.p_L + self.p_R

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# The five workloads: plain FP64 small (parity), plain FP64 at scale (the
# throughput workload), mixed precision, serving mix (per-job parameters are
# drawn by the serving driver), and streamed genotypes with 8 phenotypes.
SMALL = Workload("fp64_n1000_p4_m10k", n=1000, p_L=3, p_R=1, t=1, m=10_000, block=4096,
                 q=2000, h=0.4, seed=MASTER_SEED + 0)
SCALE = Workload("fp64_n10000_p4_m1M", n=10_000, p_L=3, p_R=1, t=1, m=1_000_000, block=4096,
                 q=20_000, h=0.5, seed=MASTER_SEED + 1)
MIXED = Workload("fp32refine_n10000_p20_m1M", n=10_000, p_L=16, p_R=4, t=1, m=1_000_000,
                 block=4096, q=20_000, h=0.5, maf_R=(0.01, 0.5), seed=MASTER_SEED + 2)
SERVE_BASE = Workload("serving_mix", n=1500, p_L=3, p_R=1, t=1, m=100_000, block=4096,
                      q=3000, h=0.5, seed=MASTER_SEED + 3)
STREAM = Workload("stream_n20000_p6_t8_m10M", n=20_000, p_L=5, p_R=1, t=8, m=10_000_000,
                  block=8192, q=40_000, h=0.5, seed=MASTER_SEED + 4)
# Phenotypes with distinct covariance matrices (the phenotype index of Eq. (1)
# with its own M_j): t = 4 phenotypes y_j, M_j = h_j Phi + (1 - h_j) I + 1e-3 I
# with the heritabilities below, one shared X_R.
PHENO = Workload("phenotypes_n10000_p4_t4_distinctM", n=10_000, p_L=3, p_R=1, t=4, m=131_072,
                 block=4096, q=20_000, h=0.5, seed=MASTER_SEED + 5)
PHENO_H = (0.2, 0.4, 0.6, 0.8)
WORKLOADS = {w.name: w for w in (SMALL, SCALE, MIXED, SERVE_BASE, STREAM, PHENO)}


def make_Z(w: Workload) -> np.ndarray:
    """Standardized genotypes z = (g - 2f)/sqrt(2f(1-f)), n x q, float64."""
    g = genotypes(w.seed, S_MAF_Z, S_Z, w.maf_Z[0], w.maf_Z[1], w.n, 0, w.q)
    f = maf(w.seed, S_MAF_Z, w.maf_Z[0], w.maf_Z[1], 0, w.q)
    sd = np.sqrt(2.0 * f * (1.0 - f))
    return (g.astype(np.float64) - 2.0 * f[None, :]) / sd[None, :]


def make_phi(w: Workload) -> np.ndarray:
    """Phi = Z Z^T / q (symmetric rank-q update of the lower triangle, then
    mirrored so that the matrix is exactly symmetric)."""
    from scipy.linalg.blas import dsyrk
    Z = np.asfortranarray(make_Z(w))
    A = dsyrk(1.0 / float(w.q), Z, lower=1)
    return _mirror_lower(A)


def _mirror_lower(A: np.ndarray) -> np.ndarray:
    L = np.tril(A)
    return np.asfortranarray(L + np.tril(L, -1).T)


def make_M(w: Workload, phi: Optional[np.ndarray] = None, h: Optional[float] = None) -> np.ndarray:
    """M = h*Phi + (1-h)*I + diag_shift*I, n x n, exactly symmetric."""
    if phi is None:
        phi = make_phi(w)
    h = w.h if h is None else h
    M = h * phi
    M[np.diag_indices_from(M)] += (1.0 - h) + w.diag_shift
    return _mirror_lower(M)


def make_XL(w: Workload) -> np.ndarray:
    """X_L: intercept column of ones, then p_L-1 N(0,1) covariates."""
    XL = np.empty((w.n, w.p_L), dtype=np.float64, order="F")
    XL[:, 0] = 1.0
    if w.p_L > 1:
        XL[:, 1:] = normals(w.seed, S_XL, w.n, 0, w.p_L - 1)
    return XL


def make_Y(w: Workload) -> np.ndarray:
    """Y: t phenotype vectors, N(0,1), n x t."""
    return normals(w.seed, S_Y, w.n, 0, w.t)


def make_XR(w: Workload, snp0: int, nsnp: int, use_c: Optional[bool] = None,
            out: Optional[np.ndarray] = None) -> np.ndarray:
    """Genotypes of problems snp0 .. snp0+nsnp-1: int8, n x (nsnp*p_R).

    Problem i owns the p_R adjacent columns i*p_R .. i*p_R+p_R-1."""
    return genotypes(w.seed, S_MAF_R, S_XR, w.maf_R[0], w.maf_R[1], w.n,
                     snp0 * w.p_R, nsnp * w.p_R, use_c=use_c, out=out)


def make_all(w: Workload, m: Optional[int] = None):
    """(M, X_L, Y, X_R) for the first m problems (default: all of w.m)."""
    m = w.m if m is None else m
    return make_M(w), make_XL(w), make_Y(w), make_XR(w, 0, m)
