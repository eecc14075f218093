"""Input generator: determinism, block independence, C twin == numpy twin."""
import numpy as np
import pytest

from paper_1210_7325_amd import datagen as dg


def test_numpy_twin_block_independent():
    w = dg.SMALL
    a = dg.make_XR(w, 0, 64, use_c=False)
    b = dg.make_XR(w, 17, 20, use_c=False)
    assert a.dtype == np.int8 and a.shape == (w.n, 64)
    assert np.array_equal(a[:, 17:37], b)
    assert set(np.unique(a)) <= {0, 1, 2}


@pytest.mark.skipif(dg._clib() is None, reason="libglsgen.so not built")
def test_c_twin_bitwise_equal():
    for w in (dg.SMALL, dg.MIXED):
        a = dg.make_XR(w, 3, 50, use_c=False)
        b = dg.make_XR(w, 3, 50, use_c=True)
        assert np.array_equal(a, b)
        fa = dg.maf(w.seed, dg.S_MAF_R, *w.maf_R, 0, 100, use_c=False)
        fb = dg.maf(w.seed, dg.S_MAF_R, *w.maf_R, 0, 100, use_c=True)
        assert np.array_equal(fa, fb)


def test_value_ranges_and_moments():
    w = dg.SMALL
    f = dg.maf(w.seed, dg.S_MAF_R, *w.maf_R, 0, 2000, use_c=False)
    assert f.min() >= 0.05 and f.max() < 0.5
    g = dg.make_XR(w, 0, 200, use_c=False).astype(np.float64)
    # column means close to 2 f_j (Binomial(2, f))
    assert np.max(np.abs(g.mean(axis=0) - 2 * f[:200])) < 0.15
    z = dg.normals(w.seed, dg.S_Y, 20000, 0, 1)
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1) < 0.03


def test_covariance_spd_symmetric_and_deterministic():
    w = dg.SMALL.replace(n=300, q=600)
    M = dg.make_M(w)
    assert np.array_equal(M, M.T)
    ev = np.linalg.eigvalsh(M)
    assert ev[0] > 0.4 and ev[-1] < 3.0
    assert np.array_equal(M, dg.make_M(w))
    XL = dg.make_XL(w)
    assert np.all(XL[:, 0] == 1.0) and XL.shape == (300, 3)
