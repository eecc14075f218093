"""Error behaviour of the C ABI on a device: calls out of order, arguments
the device path rejects, allocation failure and a handle whose factor
failed.  Every error is a return code; the handle stays usable afterwards."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1210_7325_amd import datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def G():
    from paper_1210_7325_amd import gls
    gls.lib()
    return gls


def dev(a):
    return torch.from_numpy(np.asfortranarray(a)).cuda()


@pytest.fixture(scope="module")
def problem():
    w = dg.SMALL.replace(n=300, m=20, seed=dg.MASTER_SEED + 77)
    return w, dev(dg.make_M(w)), dev(dg.make_XL(w)), dev(dg.make_Y(w)), dev(dg.make_XR(w, 0, w.m))


def test_out_of_order_and_invalid_calls(G, problem):
    say("errors: state machine")
    w, M, XL, Y, XR = problem
    L = G.lib()
    rc, h = G.gls_factor(w.n, M.data_ptr(), w.n, 0, torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    B = torch.empty((w.m, w.t, w.p), dtype=torch.float64, device="cuda")
    info = torch.empty(w.m, dtype=torch.int32, device="cuda")
    # solve and fork before the fixed part
    assert G.gls_solve_block(h, w.m, 1, XR.data_ptr(), w.n, B.data_ptr(), w.p, info.data_ptr()) == G.GLS_E_STATE
    assert G.gls_fork(h, None)[0] == G.GLS_E_STATE
    # fixed part: FP64 needs no intercept; bad intercept index, p_L, t
    assert G.gls_whiten_fixed(h, w.p_L, XL.data_ptr(), w.n, w.t, Y.data_ptr(), w.n, w.p_L) == -8
    assert G.gls_whiten_fixed(h, 0, XL.data_ptr(), w.n, w.t, Y.data_ptr(), w.n, 0) == -2
    assert G.gls_whiten_fixed(h, w.p_L, XL.data_ptr(), w.n, 9, Y.data_ptr(), w.n, 0) == -5
    assert G.gls_whiten_fixed(h, w.p_L, XL.data_ptr(), w.n, w.t, Y.data_ptr(), w.n, -1) == 0
    # block arguments: p too large, ldxr < n, ldb < p, NULL output
    assert G.gls_solve_block(h, w.m, 17, XR.data_ptr(), w.n, B.data_ptr(), 20, None) < 0
    assert G.gls_solve_block(h, w.m, 1, XR.data_ptr(), w.n - 1, B.data_ptr(), w.p, None) < 0
    assert G.gls_solve_block(h, w.m, 1, XR.data_ptr(), w.n, B.data_ptr(), w.p - 1, None) < 0
    assert G.gls_solve_block(h, w.m, 1, XR.data_ptr(), w.n, None, w.p, None) < 0
    assert G.gls_solve_block(h, 0, 1, None, w.n, None, w.p, None) == 0      # empty block
    # slab widths: 16/32/64/128 only
    assert G.gls_set_slab_cols(h, 48) == -2
    assert G.gls_set_slab_cols(h, 256) == -2
    assert G.gls_set_slab_cols(h, 128) == 0 and G.gls_set_slab_cols(h, 0) == 0
    # an impossible workspace fails cleanly and leaves the handle usable
    assert G.gls_reserve(h, 1 << 40) == G.GLS_E_OOM
    assert G.gls_solve_block(h, w.m, 1, XR.data_ptr(), w.n, B.data_ptr(), w.p, info.data_ptr()) == 0
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0) and np.all(np.isfinite(B.cpu().numpy()))
    # forks share the fixed part read-only: it cannot be replaced while shared
    rc, g = G.gls_fork(h, None)
    assert rc == 0
    assert G.gls_whiten_fixed(h, w.p_L, XL.data_ptr(), w.n, w.t, Y.data_ptr(), w.n, 0) == G.GLS_E_STATE
    G.gls_free(g)
    assert G.gls_whiten_fixed(h, w.p_L, XL.data_ptr(), w.n, w.t, Y.data_ptr(), w.n, 0) == 0
    G.gls_free(h)
    G.gls_free(None)


def test_fp32_form_needs_an_intercept(G, problem):
    say("errors: fp32 form without intercept")
    w, M, XL, Y, XR = problem
    rc, h = G.gls_factor(w.n, M.data_ptr(), w.n, 1, torch.cuda.current_stream().cuda_stream)
    assert rc == 0
    assert G.gls_whiten_fixed(h, w.p_L, XL.data_ptr(), w.n, w.t, Y.data_ptr(), w.n, -1) == G.GLS_E_UNSUPPORTED
    assert G.gls_set_slab_cols(h, 16) == G.GLS_E_UNSUPPORTED
    assert G.gls_set_slab_cols(h, 128) == 0
    G.gls_free(h)


def test_failed_factor_handle_rejects_work(G, problem):
    say("errors: not-SPD handle")
    w, M, XL, Y, XR = problem
    bad = M.clone()
    bad[7, 7] = -1.0
    rc, h = G.gls_factor(w.n, bad.data_ptr(), w.n, 0, torch.cuda.current_stream().cuda_stream)
    assert rc == G.GLS_E_NOT_SPD and G.gls_last_info(h) > 0
    assert G.gls_whiten_fixed(h, w.p_L, XL.data_ptr(), w.n, w.t, Y.data_ptr(), w.n, 0) == G.GLS_E_STATE
    G.gls_free(h)
