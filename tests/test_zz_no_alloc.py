"""gls_solve_block_noalloc, the entry point that allocates nothing: through
the C ABI it gives the same bits as gls_solve_block on the same handle, for
two calls in a row (the second smaller, so the fixed scratch still holds the
first call's larger contents), in both precisions; a block too large for the
scratch is refused before any device work."""
import sys

import numpy as np
import pytest

from oracle import gls_oracle as orc
from paper_1210_7325_amd import datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def to_dev(a):
    return torch.from_numpy(np.asfortranarray(a)).cuda()


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_noalloc_equals_solve_block(prec):
    from paper_1210_7325_amd import gls
    gls.lib()
    w = dg.SMALL.replace(n=1000, q=2000, p_L=3, t=2, m=1200, seed=dg.MASTER_SEED + 70)
    M, XL, Y = dg.make_M(w), dg.make_XL(w), dg.make_Y(w)
    c = gls.Cohort(to_dev(M), precision=prec).whiten_fixed(to_dev(XL), to_dev(Y), intercept_col=0)
    st = gls._stream_ptr(c.stream)
    # first call: 700 problems of one genotype column; second: 150 problems of
    # two columns (300 columns, fewer than the first call's 700)
    for nsnp, p_R in ((700, 1), (150, 2)):
        say("noalloc", prec, nsnp, p_R)
        XR = dg.make_XR(w.replace(p_R=p_R), 0, nsnp)
        dX = to_dev(XR)
        p = w.p_L + p_R
        Bref, inf_ref = c.solve_block(dX, p_R=p_R)
        B = torch.full((nsnp, w.t, p), -7.0, dtype=torch.float64, device="cuda")
        info = torch.full((nsnp,), -7, dtype=torch.int32, device="cuda")
        torch.cuda.current_stream().synchronize()
        rc = gls.gls_solve_block_noalloc(c.h, nsnp, p_R, dX.data_ptr(), int(dX.stride(1)),
                                         B.data_ptr(), p, info.data_ptr())
        assert rc == 0, gls.strerror(rc)
        c.stream.synchronize()
        torch.cuda.synchronize()
        assert np.array_equal(B.cpu().numpy(), Bref.cpu().numpy())
        assert np.array_equal(info.cpu().numpy(), inf_ref.cpu().numpy())
        assert np.all(info.cpu().numpy() == 0)
        ref = orc.gls_sequence(M, XL, XR, Y, p_R)
        err = orc.relative_error(B.cpu().numpy(), ref).max()
        say("max rel err vs oracle", err)
        assert err < (1e-10 if prec == "fp64" else 1e-8)
    # too large for the scratch: refused before any device work, outputs untouched
    n_pad = 1024
    per_col = 8 * n_pad + (4 * n_pad if prec == "fp32_refine" else 0)
    cols = (gls.NOALLOC_SCRATCH_BYTES // per_col) // 128 * 128 + 128
    dX = torch.zeros((cols, w.n), dtype=torch.int8, device="cuda").t()
    B = torch.full((cols, w.t, w.p_L + 1), -7.0, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    rc = gls.gls_solve_block_noalloc(c.h, cols, 1, dX.data_ptr(), w.n, B.data_ptr(), w.p_L + 1, None)
    assert rc == gls.GLS_E_TOO_LARGE
    torch.cuda.synchronize()
    assert bool((B == -7.0).all())
    c.free()
