"""Phenotypes with distinct covariance matrices M_j (the phenotype index of
Eq. (1), each y_j with its own M_j = h_j Phi + (1 - h_j) I + 1e-3 I): one
handle per M_j, and every block of genotypes solved for all phenotypes by
one gls_solve_multi launch whose items share the same X_R array.  Each
phenotype's b_ij against the oracle run with its own M_j, and bitwise
against solving that phenotype alone."""
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


@pytest.mark.parametrize("prec,n,p_R,m,block", [("fp64", 700, 1, 500, 160), ("fp64", 300, 2, 90, 90),
                                                 ("fp32_refine", 700, 1, 500, 256)])
def test_distinct_m_per_phenotype(prec, n, p_R, m, block):
    from paper_1210_7325_amd import gls
    gls.lib()
    hs = (0.2, 0.5, 0.8)
    w = dg.PHENO.replace(n=n, q=2 * n, p_R=p_R, t=len(hs), m=m, seed=dg.MASTER_SEED + 80 + n)
    say("distinct M_j", prec, n, p_R, m, block)
    phi = dg.make_phi(w)
    Ms = [dg.make_M(w, phi, h=h) for h in hs]
    XL, Y = dg.make_XL(w), dg.make_Y(w)
    XR = dg.make_XR(w, 0, m)
    dXR = to_dev(XR)
    cs = [gls.Cohort(to_dev(M), precision=prec).whiten_fixed(to_dev(XL), to_dev(Y[:, j:j + 1]))
          for j, M in enumerate(Ms)]
    p = w.p_L + p_R
    Bs = [torch.empty((m, 1, p), dtype=torch.float64, device="cuda") for _ in hs]
    infos = [torch.full((m,), -7, dtype=torch.int32, device="cuda") for _ in hs]
    torch.cuda.synchronize()
    for a in range(0, m, block):
        b = min(m, a + block)
        gls.solve_multi([(c, dXR[:, a * p_R:b * p_R], p_R, B[a:b], inf[a:b])
                         for c, B, inf in zip(cs, Bs, infos)])
    torch.cuda.synchronize()
    tol = 1e-10 if prec == "fp64" else 1e-8
    for j, (c, M) in enumerate(zip(cs, Ms)):
        assert int((infos[j] != 0).sum()) == 0
        got = Bs[j].cpu().numpy()
        ref = orc.gls_sequence(M, XL, XR, Y[:, j:j + 1], p_R)
        err = orc.relative_error(got, ref).max()
        say(f"phenotype {j} (h = {hs[j]}): max rel err {err:.3e}")
        assert err < tol
        alone, _ = c.solve_block(dXR, p_R=p_R)
        torch.cuda.synchronize()
        assert np.array_equal(alone.cpu().numpy(), got)
    for c in cs:
        c.free()
