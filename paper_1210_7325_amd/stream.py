"""Streamed genotypes (the out-of-core form, Sec. 4, Alg. 8) over the C ABI.

`solve_stream` runs gls_solve_stream: the library double-buffers blocks of
genotypes through pinned host memory, overlapping the host-side production
of block j+1 and its copy to the device with the solve of block j and the
copy back of block j-1.  Genotypes come from a fill callback (a reader of
the caller's storage); `workload_fill` gives the synthetic generator's C
fill function so that no Python runs per block on the input side.
"""
from __future__ import annotations

import ctypes
from typing import Callable, Optional

import numpy as np

from . import datagen as dg
from . import gls


class _GenCtx(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("stream_maf", ctypes.c_uint64),
                ("stream_g", ctypes.c_uint64), ("lo", ctypes.c_double), ("hi", ctypes.c_double),
                ("n", ctypes.c_int64), ("p_R", ctypes.c_int64)]


def workload_fill(w: dg.Workload):
    """(fill function pointer, context) producing the workload's genotypes."""
    lib = dg._clib()
    if lib is None:
        raise ImportError("libglsgen.so is not built")
    ctx = _GenCtx(w.seed, dg.S_MAF_R, dg.S_XR, w.maf_R[0], w.maf_R[1], w.n, w.p_R)
    fn = ctypes.cast(lib.gen_fill_genotypes, ctypes.c_void_p).value
    return fn, ctx


def solve_stream(cohort: "gls.Cohort", snp_begin: int, snp_end: int, block: int, p_R: int,
                 fill, fill_ctx, out: Optional[np.ndarray] = None,
                 info_out: Optional[np.ndarray] = None,
                 on_block: Optional[Callable[[int, int], bool]] = None):
    """Solve problems [snp_begin, snp_end) with streamed genotypes.

    out: host float64 array (m_total, t, p) indexed by absolute problem
    number (allocated for the range if None); on_block(snp0, nsnp) is called
    after each block lands in `out` and may return False to abort (the run
    can then resume at the next block boundary).  Returns (out, info, stats)."""
    t, p = cohort.t, cohort.p_L + p_R
    base = 0
    if out is None:
        out = np.empty((snp_end - snp_begin, t, p))
        base = snp_begin
    if info_out is None:
        info_out = np.empty(out.shape[0], dtype=np.int32)

    def sink(_ctx, snp0, nsnp, b, info):
        a = snp0 - base
        out[a:a + nsnp] = np.ctypeslib.as_array(b, shape=(nsnp * t * p,)).reshape(nsnp, t, p)
        info_out[a:a + nsnp] = np.ctypeslib.as_array(info, shape=(nsnp,))
        if on_block is not None and on_block(snp0, nsnp) is False:
            return 1
        return 0

    sink_cb = gls.SINK_FN(sink)
    fctx = ctypes.cast(ctypes.pointer(fill_ctx), ctypes.c_void_p) if isinstance(
        fill_ctx, ctypes.Structure) else fill_ctx
    if callable(fill) and not isinstance(fill, int):
        fill_ptr = fill if isinstance(fill, gls.FILL_FN) else gls.FILL_FN(fill)
    else:
        fill_ptr = fill
    rc, st = gls.gls_solve_stream(cohort.h, snp_begin, snp_end, block, p_R, fill_ptr, fctx,
                                  sink_cb, None)
    stats = {k: getattr(st, k) for k, _ in gls.gls_stream_stats._fields_}
    if rc != 0:
        raise gls.GLSError(rc, "gls_solve_stream")
    return out, info_out, stats
