"""The C-ABI library on the host (no GPU): it loads, exports every entry
point include/gls.h declares, rejects bad arguments before touching the
device, and its footprint arithmetic adds up."""
import ctypes
import os
import re

import pytest

from paper_1210_7325_amd import gls

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gls.h")

pytestmark = pytest.mark.skipif(not os.path.exists(gls.LIB_PATH), reason="libgls.so not built")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gls_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 17
    L = gls.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(gls.EXPORTS) == set(names)


def test_argument_validation_without_device():
    L = gls.lib()
    # gls_factor: out NULL, n too small, M NULL, ldm < n, bad precision
    h = ctypes.c_void_p()
    assert L.gls_factor(None, 10, 1, 10, 0, None) == -1
    assert L.gls_factor(ctypes.byref(h), 1, 1, 1, 0, None) == -2
    assert L.gls_factor(ctypes.byref(h), 10, None, 10, 0, None) == -3
    assert L.gls_factor(ctypes.byref(h), 10, 1, 9, 0, None) == -4
    assert L.gls_factor(ctypes.byref(h), 10, 1, 10, 7, None) == -5
    assert h.value is None
    # NULL handles
    assert L.gls_whiten_fixed(None, 3, 1, 10, 1, 1, 10, 0) == -1
    assert L.gls_solve_block(None, 5, 1, 1, 10, 1, 4, None) == -1
    assert L.gls_solve_block_noalloc(None, 5, 1, 1, 10, 1, 4, None) == -1
    assert L.gls_reserve(None, 10) == -1
    assert L.gls_set_stream(None, None) == -1
    assert L.gls_copy_factor(None, 1, 10) == -1
    assert L.gls_copy_fixed(None, None, 0, None, 0, None, None) == -1
    assert L.gls_whiten_block(None, 1, 1, 10, 1, 10) == -1
    assert L.gls_whiten_block_f64(None, 1, 1, 10, 1, 10) == -1
    out = ctypes.c_void_p()
    assert L.gls_fork(None, None, ctypes.byref(out)) == -1
    assert L.gls_fork(None, None, None) == -3
    assert L.gls_last_info(None) == -1
    assert L.gls_solve_multi(None, -1, None) == -2
    assert L.gls_solve_multi(None, 0, None) == 0
    assert L.gls_solve_multi(None, 3, None) == -1
    assert L.gls_set_slab_cols(None, 64) == -1
    assert L.gls_set_kernel_timing(None, 1) == -1
    assert L.gls_kernel_time(None, 0, None, None) == -1
    assert L.gls_kernel_launches(None, 0, 0, None, None, None, None) == -1
    L.gls_free(None)


def test_strerror_codes():
    for code in range(0, 9):
        assert gls.strerror(code) != "unknown error"
    assert gls.strerror(9) == "unknown error"
    assert gls.strerror(-3) == "invalid argument"
    assert "positive definite" in gls.strerror(gls.GLS_E_NOT_SPD)


def test_footprint_arithmetic():
    L = gls.lib()
    n, pL, t, cols = 10_000, 3, 1, 4096
    K = (n + 127) // 128
    npad = K * 128
    expect = (K * (K - 1) // 2 * 128 * 128 * 8 + 2 * K * 128 * 128 * 8
              + npad * npad * 8 + K * 128 * 128 * 8
              + npad * (pL + t) * 8 + (pL + t) ** 2 * 8
              + npad * 4096 * 8)
    assert L.gls_footprint_bytes(n, pL, 1, t, cols, 0) == expect
    assert L.gls_footprint_bytes(n, pL, 1, t, cols, 1) > expect
    assert L.gls_footprint_bytes(0, pL, 1, t, cols, 0) == 0
    # monotone in every size
    assert L.gls_footprint_bytes(2 * n, pL, 1, t, cols, 0) > expect
    assert L.gls_footprint_bytes(n, pL, 1, t, 2 * cols, 0) > expect
    # p_R genotype columns per problem: the workspace of nsnp p_R columns
    assert L.gls_footprint_bytes(n, pL, 2, t, cols // 2, 0) == expect
    assert L.gls_footprint_bytes(n, pL, 0, t, cols, 0) == 0
