"""Python binding of the solver's C ABI (include/gls.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libgls.so.  PyTorch supplies device memory and streams.  The
library must have been built (python -m paper_1210_7325_amd.build); loading
fails loudly otherwise, there is no fallback.

Two levels:
  * the raw entry points, same names and arguments as the C functions
    (pointers and streams as Python ints), returning the C return codes;
  * Cohort, a small convenience class over torch tensors.

Matrices are column-major: a (rows, cols) tensor with stride(0) == 1; other
layouts are copied first, on the handle's stream, so that the copy is ordered
before the library's kernels.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgls.so")

GLS_FP64 = 0
GLS_FP32_REFINE = 1
PRECISIONS = {"fp64": GLS_FP64, "fp32_refine": GLS_FP32_REFINE}

GLS_OK, GLS_E_NOT_SPD, GLS_E_STATE, GLS_E_OOM, GLS_E_HIP, GLS_E_UNSUPPORTED = 0, 1, 2, 3, 4, 5
GLS_E_IO, GLS_E_ABORTED, GLS_E_TOO_LARGE = 6, 7, 8
# fixed device scratch of gls_solve_block_noalloc (GLS_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 128 << 20

EXPORTS = ("gls_factor", "gls_whiten_fixed", "gls_solve_block", "gls_solve_block_noalloc",
           "gls_reserve", "gls_free",
           "gls_fork", "gls_set_stream", "gls_footprint_bytes", "gls_last_info",
           "gls_strerror", "gls_copy_factor", "gls_copy_fixed", "gls_whiten_block",
           "gls_whiten_block_f64",
           "gls_solve_multi", "gls_set_slab_cols", "gls_set_kernel_timing", "gls_kernel_time",
           "gls_kernel_launches",
           "gls_solve_stream", "gls_file_open", "gls_file_fill", "gls_file_stats",
           "gls_file_close", "gls_writer_open", "gls_writer_sink", "gls_writer_close")

_i64, _p, _int = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int


class gls_work(ctypes.Structure):
    _fields_ = [("h", _p), ("nsnp", _i64), ("p_R", _i64), ("X_R", _p), ("ldxr", _i64),
                ("B", _p), ("ldb", _i64), ("info", _p)]


class gls_stream_stats(ctypes.Structure):
    _fields_ = [("wall_ms", ctypes.c_double), ("fill_ms", ctypes.c_double),
                ("sink_ms", ctypes.c_double), ("wait_ms", ctypes.c_double),
                ("blocks", _i64), ("bytes_h2d", _i64), ("bytes_d2h", _i64)]


FILL_FN = ctypes.CFUNCTYPE(_int, _p, _i64, _i64, _p, _i64)
SINK_FN = ctypes.CFUNCTYPE(_int, _p, _i64, _i64, ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_int32))


class GLSError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where} failed: code {code} ({strerror(code)})")


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1210_7325_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "gls_factor": (_int, [ctypes.POINTER(_p), _i64, _p, _i64, _int, _p]),
            "gls_whiten_fixed": (_int, [_p, _i64, _p, _i64, _i64, _p, _i64, _i64]),
            "gls_solve_block": (_int, [_p, _i64, _i64, _p, _i64, _p, _i64, _p]),
            "gls_solve_block_noalloc": (_int, [_p, _i64, _i64, _p, _i64, _p, _i64, _p]),
            "gls_reserve": (_int, [_p, _i64]),
            "gls_free": (None, [_p]),
            "gls_fork": (_int, [_p, _p, ctypes.POINTER(_p)]),
            "gls_set_stream": (_int, [_p, _p]),
            "gls_footprint_bytes": (ctypes.c_size_t, [_i64, _i64, _i64, _i64, _i64, _int]),
            "gls_last_info": (_int, [_p]),
            "gls_strerror": (ctypes.c_char_p, [_int]),
            "gls_copy_factor": (_int, [_p, _p, _i64]),
            "gls_copy_fixed": (_int, [_p, _p, _i64, _p, _i64, _p, _p]),
            "gls_whiten_block": (_int, [_p, _i64, _p, _i64, _p, _i64]),
            "gls_whiten_block_f64": (_int, [_p, _i64, _p, _i64, _p, _i64]),
            "gls_solve_multi": (_int, [ctypes.POINTER(gls_work), _i64, _p]),
            "gls_set_slab_cols": (_int, [_p, _int]),
            "gls_set_kernel_timing": (_int, [_p, _int]),
            "gls_kernel_time": (_int, [_p, _int, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(_i64)]),
            "gls_kernel_launches": (_int, [_p, _int, _i64, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(_i64), ctypes.POINTER(_int),
                                           ctypes.POINTER(_i64)]),
            "gls_solve_stream": (_int, [_p, _i64, _i64, _i64, _i64, _p, _p, _p, _p,
                                        ctypes.POINTER(gls_stream_stats)]),
            "gls_file_open": (_int, [ctypes.POINTER(_p), ctypes.c_char_p, _i64, _i64, _i64, _int,
                                     _int]),
            "gls_file_fill": (_int, [_p, _i64, _i64, _p, _i64]),
            "gls_file_stats": (_int, [_p, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double)]),
            "gls_file_close": (None, [_p]),
            "gls_writer_open": (_int, [ctypes.POINTER(_p), ctypes.c_char_p, ctypes.c_char_p, _i64,
                                       _i64, _i64, _int]),
            "gls_writer_sink": (_int, [_p, _i64, _i64, _p, _p]),
            "gls_writer_close": (_int, [_p, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def strerror(code: int) -> str:
    try:
        return lib().gls_strerror(code).decode()
    except ImportError:
        return "?"


def _chk(rc: int, where: str) -> int:
    if rc != 0:
        raise GLSError(rc, where)
    return rc


# ---- raw entry points (same names as the C ABI) ------------------------------
def gls_factor(n: int, M: int, ldm: int, prec: int, stream: int) -> Tuple[int, int]:
    """Returns (return code, handle); GLS_E_NOT_SPD still yields a handle."""
    h = _p()
    rc = lib().gls_factor(ctypes.byref(h), n, M, ldm, prec, stream)
    return rc, (h.value or 0)


def gls_whiten_fixed(h, p_L, X_L, ldx, t, Y, ldy, intercept_col) -> int:
    return lib().gls_whiten_fixed(h, p_L, X_L, ldx, t, Y, ldy, intercept_col)


def gls_solve_block(h, nsnp, p_R, X_R, ldxr, B, ldb, info) -> int:
    return lib().gls_solve_block(h, nsnp, p_R, X_R, ldxr, B, ldb, info)


def gls_solve_block_noalloc(h, nsnp, p_R, X_R, ldxr, B, ldb, info) -> int:
    return lib().gls_solve_block_noalloc(h, nsnp, p_R, X_R, ldxr, B, ldb, info)


def gls_reserve(h, max_cols) -> int:
    return lib().gls_reserve(h, max_cols)


def gls_free(h) -> None:
    lib().gls_free(h)


def gls_fork(h, stream) -> Tuple[int, int]:
    out = _p()
    rc = lib().gls_fork(h, stream, ctypes.byref(out))
    return rc, (out.value or 0)


def gls_set_stream(h, stream) -> int:
    return lib().gls_set_stream(h, stream)


def gls_footprint_bytes(n, p_L, p_R, t, max_nsnp, prec) -> int:
    return int(lib().gls_footprint_bytes(n, p_L, p_R, t, max_nsnp, prec))


def gls_last_info(h) -> int:
    return lib().gls_last_info(h)


def gls_strerror(code) -> str:
    return strerror(code)


def gls_copy_factor(h, L, ldl) -> int:
    return lib().gls_copy_factor(h, L, ldl)


def gls_copy_fixed(h, WL, ldwl, Yt, ldyt, S_TL, C_T) -> int:
    return lib().gls_copy_fixed(h, WL, ldwl, Yt, ldyt, S_TL, C_T)


def gls_whiten_block(h, ncols, X, ldx, W, ldw) -> int:
    return lib().gls_whiten_block(h, ncols, X, ldx, W, ldw)


def gls_whiten_block_f64(h, ncols, X, ldx, W, ldw) -> int:
    return lib().gls_whiten_block_f64(h, ncols, X, ldx, W, ldw)


def gls_solve_multi(items, stream) -> int:
    arr = (gls_work * len(items))(*items)
    return lib().gls_solve_multi(arr, len(items), stream)


def gls_set_slab_cols(h, cols) -> int:
    return lib().gls_set_slab_cols(h, cols)


def gls_set_kernel_timing(h, enable) -> int:
    return lib().gls_set_kernel_timing(h, enable)


def gls_kernel_time(h, kind) -> Tuple[int, float, int]:
    ms, cnt = ctypes.c_double(), _i64()
    rc = lib().gls_kernel_time(h, kind, ctypes.byref(ms), ctypes.byref(cnt))
    return rc, ms.value, cnt.value


def gls_kernel_launches(h, kind) -> Tuple[int, list]:
    """[(ms, cols, slab)] of every recorded launch of `kind`, in launch order."""
    cnt = _i64()
    rc = lib().gls_kernel_launches(h, kind, 0, None, None, None, ctypes.byref(cnt))
    if rc or cnt.value == 0:
        return rc, []
    n = cnt.value
    ms, cols, slab = (ctypes.c_double * n)(), (_i64 * n)(), (_int * n)()
    rc = lib().gls_kernel_launches(h, kind, n, ms, cols, slab, ctypes.byref(cnt))
    return rc, [(ms[i], cols[i], slab[i]) for i in range(min(n, cnt.value))]


def gls_solve_stream(h, snp_begin, snp_end, block, p_R, fill, fill_ctx, sink, sink_ctx):
    """fill / sink: C function pointers (ints) or ctypes callbacks of types
    FILL_FN / SINK_FN.  Returns (return code, gls_stream_stats)."""
    st = gls_stream_stats()
    f = ctypes.cast(fill, _p) if not isinstance(fill, int) else fill
    k = ctypes.cast(sink, _p) if not isinstance(sink, int) else sink
    rc = lib().gls_solve_stream(h, snp_begin, snp_end, block, p_R, f, fill_ctx, k, sink_ctx,
                                ctypes.byref(st))
    return rc, st


# ---- torch convenience ---------------------------------------------------------
def gls_file_open(path: str, n: int, p_R: int, offset: int = 0, direct: bool = False,
                  threads: int = 8) -> Tuple[int, int]:
    h = _p()
    rc = lib().gls_file_open(ctypes.byref(h), os.fsencode(path), n, p_R, offset, int(direct), threads)
    return rc, h.value


def gls_file_fill(src, snp0, nsnp, buf, ld) -> int:
    return lib().gls_file_fill(src, snp0, nsnp, buf, ld)


def gls_file_stats(src) -> Tuple[int, int, float]:
    b, ms = _i64(), ctypes.c_double()
    rc = lib().gls_file_stats(src, ctypes.byref(b), ctypes.byref(ms))
    return rc, b.value, ms.value


def gls_file_close(src) -> None:
    lib().gls_file_close(src)


def gls_writer_open(b_path: str, info_path: Optional[str], t: int, p: int, snp_base: int = 0,
                    depth: int = 4) -> Tuple[int, int]:
    h = _p()
    rc = lib().gls_writer_open(ctypes.byref(h), os.fsencode(b_path),
                               os.fsencode(info_path) if info_path else None, t, p, snp_base, depth)
    return rc, h.value


def gls_writer_sink(w, snp0, nsnp, b, info) -> int:
    return lib().gls_writer_sink(w, snp0, nsnp, b, info)


def gls_writer_close(w) -> Tuple[int, int, float, float, float]:
    """Returns (return code, bytes written, ms in pwrite, ms sinks waited, ms of the close)."""
    b, wr, wa, cl = _i64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    rc = lib().gls_writer_close(w, ctypes.byref(b), ctypes.byref(wr), ctypes.byref(wa),
                                ctypes.byref(cl))
    return rc, b.value, wr.value, wa.value, cl.value


def _torch():
    import torch
    return torch


def colmajor(t):
    """Same values, column-major storage (stride(0) == 1)."""
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    if t.stride(0) == 1 and (t.shape[1] == 1 or t.stride(1) >= t.shape[0]):
        return t
    return t.t().contiguous().t()


def _ld(t) -> int:
    return max(int(t.stride(1)) if t.shape[1] > 1 else int(t.shape[0]), 1)


def _stream_ptr(stream) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Cohort:
    """One cohort: M factored once, fixed part whitened once, then any
    number of genotype blocks solved (the in-core algorithm, Sec. 2)."""

    def __init__(self, M, precision: str = "fp64", stream=None, _handle: Optional[int] = None):
        torch = _torch()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.prec = PRECISIONS[precision]
        self._keep = []
        if _handle is not None:
            self.h = _handle
            self.n = None
            return
        assert M.dtype == torch.float64 and M.is_cuda and M.dim() == 2 and M.shape[0] == M.shape[1]
        # any layout copy runs on the handle's stream, ahead of the factorization
        with torch.cuda.stream(self.stream):
            M = colmajor(M)
        self.n = int(M.shape[0])
        rc, h = gls_factor(self.n, M.data_ptr(), _ld(M), self.prec, _stream_ptr(self.stream))
        self.h = h
        if rc == GLS_E_NOT_SPD:
            self.info = gls_last_info(h)
            gls_free(h)
            self.h = 0
            raise GLSError(rc, f"gls_factor (leading minor {self.info})")
        _chk(rc, "gls_factor")
        self.info = 0
        self.p_L = self.t = None

    # the fixed part (X_L, y) -------------------------------------------------
    def whiten_fixed(self, XL, Y, intercept_col: int = 0):
        torch = _torch()
        with torch.cuda.stream(self.stream):
            XL = colmajor(XL.to(torch.float64))
            Y = colmajor(Y.to(torch.float64))
        self.p_L, self.t = int(XL.shape[1]), int(Y.shape[1])
        _chk(gls_whiten_fixed(self.h, self.p_L, XL.data_ptr(), _ld(XL), self.t, Y.data_ptr(),
                              _ld(Y), intercept_col), "gls_whiten_fixed")
        self._keep = [XL, Y]  # alive until the stream passes the call
        if self.n is None:
            self.n = int(XL.shape[0])
        return self

    def reserve(self, max_cols: int):
        _chk(gls_reserve(self.h, max_cols), "gls_reserve")

    # blocks of problems -------------------------------------------------------
    def solve_block(self, XR, p_R: int = 1, B=None, info=None):
        """XR: int8 (n, nsnp*p_R) column-major on the device.  Returns
        (B, info) with B of shape (nsnp, t, p) FP64 and info int32 (nsnp,)."""
        torch = _torch()
        assert XR.dtype == torch.int8 and XR.is_cuda
        with torch.cuda.stream(self.stream):
            XR = colmajor(XR)
            ncols = int(XR.shape[1])
            assert ncols % p_R == 0
            nsnp = ncols // p_R
            p = self.p_L + p_R
            if B is None:
                B = torch.empty((nsnp, self.t, p), dtype=torch.float64, device=XR.device)
            if info is None:
                info = torch.empty((nsnp,), dtype=torch.int32, device=XR.device)
        _chk(gls_solve_block(self.h, nsnp, p_R, XR.data_ptr(), _ld(XR), B.data_ptr(), p,
                             info.data_ptr()), "gls_solve_block")
        return B, info

    def whiten_block(self, X, W=None):
        """L^{-1} X for int8 (gls_whiten_block) or FP64 (gls_whiten_block_f64)
        X of shape (n, ncols); returns W, or writes the caller's column-major W."""
        torch = _torch()
        with torch.cuda.stream(self.stream):
            X = colmajor(X)
            if W is None:
                W = torch.empty((X.shape[1], X.shape[0]), dtype=torch.float64, device=X.device).t()
        assert W.dtype == torch.float64 and W.stride(0) == 1
        if X.dtype == torch.float64:
            _chk(gls_whiten_block_f64(self.h, int(X.shape[1]), X.data_ptr(), _ld(X), W.data_ptr(),
                                      _ld(W)), "gls_whiten_block_f64")
        else:
            assert X.dtype == torch.int8
            _chk(gls_whiten_block(self.h, int(X.shape[1]), X.data_ptr(), _ld(X), W.data_ptr(),
                                  _ld(W)), "gls_whiten_block")
        return W

    def copy_factor(self):
        torch = _torch()
        with torch.cuda.stream(self.stream):
            L = torch.empty((self.n, self.n), dtype=torch.float64, device="cuda").t()
        _chk(gls_copy_factor(self.h, L.data_ptr(), self.n), "gls_copy_factor")
        return L

    def copy_fixed(self):
        torch = _torch()
        n, pL, t = self.n, self.p_L, self.t
        with torch.cuda.stream(self.stream):
            WL = torch.empty((pL, n), dtype=torch.float64, device="cuda").t()
            Yt = torch.empty((t, n), dtype=torch.float64, device="cuda").t()
            STL = torch.empty((pL, pL), dtype=torch.float64, device="cuda").t()
            CT = torch.empty((t, pL), dtype=torch.float64, device="cuda").t()
        _chk(gls_copy_fixed(self.h, WL.data_ptr(), n, Yt.data_ptr(), n, STL.data_ptr(),
                            CT.data_ptr()), "gls_copy_fixed")
        return WL, Yt, STL, CT

    def set_slab_cols(self, cols: int):
        _chk(gls_set_slab_cols(self.h, cols), "gls_set_slab_cols")

    def set_kernel_timing(self, enable: bool):
        _chk(gls_set_kernel_timing(self.h, int(enable)), "gls_set_kernel_timing")

    def kernel_time(self, kind: int) -> Tuple[float, int]:
        rc, ms, cnt = gls_kernel_time(self.h, kind)
        _chk(rc, "gls_kernel_time")
        return ms, cnt

    def kernel_launches(self, kind: int) -> list:
        """Per-launch record of the kernel timing: [(ms, cols, slab)]."""
        rc, out = gls_kernel_launches(self.h, kind)
        _chk(rc, "gls_kernel_launches")
        return out

    def fork(self, stream=None) -> "Cohort":
        torch = _torch()
        stream = stream if stream is not None else torch.cuda.Stream()
        rc, h = gls_fork(self.h, _stream_ptr(stream))
        _chk(rc, "gls_fork")
        c = Cohort(None, stream=stream, _handle=h)
        c.n, c.p_L, c.t, c.prec = self.n, self.p_L, self.t, self.prec
        return c

    def free(self):
        if getattr(self, "h", 0):
            gls_free(self.h)
            self.h = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def solve_multi(items, stream=None):
    """items: list of (Cohort, XR, p_R, B, info) solved together on
    `stream` (one launch per kernel, or rounds of launches for one cohort's
    work beyond one work-group per compute unit)."""
    works = []
    for c, XR, p_R, B, info in items:
        # no layout copies here: the launch reads the caller's arrays as they are
        assert XR.stride(0) == 1 and B.is_contiguous(), "X_R column-major, B contiguous"
        works.append(gls_work(c.h, XR.shape[1] // p_R, p_R, XR.data_ptr(), _ld(XR), B.data_ptr(),
                              c.p_L + p_R, info.data_ptr() if info is not None else None))
    _chk(gls_solve_multi(works, _stream_ptr(stream)), "gls_solve_multi")
