"""The library's file reader for streamed genotypes (gls_file_open /
gls_file_fill), host side only: it must hand back exactly the bytes of the
requested problems, for any block, thread count and alignment, and fail
cleanly on bad requests."""
import ctypes
import os

import numpy as np
import pytest

from paper_1210_7325_amd import datagen as dg
from paper_1210_7325_amd import gls, stream


def aligned_buffer(nbytes, align=4096):
    raw = np.empty(nbytes + align, dtype=np.int8)
    off = (-raw.ctypes.data) % align
    return raw[off:off + nbytes]


@pytest.fixture(scope="module")
def lib():
    return gls.lib()


@pytest.mark.parametrize("n,p_R,m", [(1000, 2, 300), (4096, 1, 64), (129, 3, 50)])
def test_fill_returns_the_generator_bytes(lib, tmp_path, n, p_R, m):
    w = dg.SMALL.replace(n=n, p_R=p_R, seed=dg.MASTER_SEED + 900 + n)
    path = str(tmp_path / "g.bin")
    assert stream.write_genotype_file(path, w, m, chunk=37) == n * p_R * m
    assert os.path.getsize(path) == n * p_R * m
    for direct in (False, True):
        for threads in (1, 3, 8):
            with stream.FileSource(path, n, p_R, direct=direct, threads=threads) as src:
                for snp0, nsnp in ((0, m), (5, 17), (m - 1, 1), (m // 2, m - m // 2)):
                    buf = aligned_buffer(n * p_R * nsnp)
                    rc = gls.gls_file_fill(src.h, snp0, nsnp, buf.ctypes.data, n)
                    assert rc == 0
                    got = buf.reshape(nsnp * p_R, n).T
                    assert np.array_equal(got, dg.make_XR(w, snp0, nsnp, use_c=False))
                b, ms = src.stats()
                assert b == n * p_R * (m + 17 + 1 + (m - m // 2)) and ms >= 0


def test_offset_and_errors(lib, tmp_path):
    n, p_R, m = 200, 1, 40
    w = dg.SMALL.replace(n=n, p_R=p_R, seed=dg.MASTER_SEED + 901)
    path = str(tmp_path / "g.bin")
    with open(path, "wb") as f:
        f.write(b"\x07" * 123)                      # a header the reader skips
    body = str(tmp_path / "body.bin")
    stream.write_genotype_file(body, w, m)
    with open(path, "ab") as f, open(body, "rb") as g:
        f.write(g.read())
    with stream.FileSource(path, n, p_R, offset=123, threads=2) as src:
        buf = np.empty(n * 10, dtype=np.int8)
        assert gls.gls_file_fill(src.h, 30, 10, buf.ctypes.data, n) == 0
        assert np.array_equal(buf.reshape(10, n).T, dg.make_XR(w, 30, 10, use_c=False))
        # past the end of the file, wrong leading dimension, negative start
        assert gls.gls_file_fill(src.h, 35, 10, buf.ctypes.data, n) != 0
        assert gls.gls_file_fill(src.h, 0, 10, buf.ctypes.data, n + 1) != 0
        assert gls.gls_file_fill(src.h, -1, 1, buf.ctypes.data, n) != 0
        assert gls.gls_file_fill(src.h, 0, 0, buf.ctypes.data, n) == 0
    rc, h = gls.gls_file_open(str(tmp_path / "missing.bin"), n, p_R)
    assert rc == 6 and h is None                    # GLS_E_IO
    assert gls.strerror(6) == "file could not be opened or read"
    assert gls.gls_file_open(path, 0, 1)[0] == -3
    assert gls.gls_file_open(path, n, 17)[0] == -4
    assert gls.gls_file_open(path, n, 1, offset=-1)[0] == -5
    assert gls.gls_file_open(path, n, 1, threads=0)[0] == -7
    gls.gls_file_close(None)                        # no-op


# --- the asynchronous writer of results (gls_writer_*) ---------------------------
def _block(rng, nsnp, t, p):
    return rng.standard_normal((nsnp, t, p)), rng.integers(-3, 5, nsnp).astype(np.int32)


@pytest.mark.parametrize("t,p,depth", [(1, 4, 1), (8, 6, 2), (3, 20, 5)])
def test_writer_round_trip(lib, tmp_path, t, p, depth):
    """Blocks handed to the sink (in and out of order, more blocks than
    buffers) land at their own offsets of the b and info files, bit for bit."""
    rng = np.random.default_rng(t * 100 + p)
    base, m = 1000, 900
    bpath, ipath = str(tmp_path / "b.bin"), str(tmp_path / "info.bin")
    B = np.zeros((m, t, p))
    info = np.zeros(m, np.int32)
    cuts = [0, 7, 300, 301, 555, 900]
    order = [2, 0, 4, 1, 3]
    rc, w = gls.gls_writer_open(bpath, ipath, t, p, base, depth)
    assert rc == 0
    for k in order:
        a, e = cuts[k], cuts[k + 1]
        b, inf = _block(rng, e - a, t, p)
        B[a:e], info[a:e] = b, inf
        b = np.ascontiguousarray(b)
        assert gls.gls_writer_sink(w, base + a, e - a, b.ctypes.data, inf.ctypes.data) == 0
    rc, nbytes, wr, wa, cl = gls.gls_writer_close(w)
    assert rc == 0 and nbytes == m * (t * p * 8 + 4)
    got = np.fromfile(bpath, dtype=np.float64).reshape(m, t, p)
    assert np.array_equal(got, B)
    assert np.array_equal(np.fromfile(ipath, dtype=np.int32), info)


def test_writer_errors(lib, tmp_path):
    rc, w = gls.gls_writer_open(str(tmp_path / "no" / "such" / "dir" / "b.bin"), None, 1, 4, 0, 2)
    assert rc == gls.GLS_E_IO and not w
    assert gls.gls_writer_open(str(tmp_path / "b.bin"), None, 0, 4, 0, 2)[0] == -4
    assert gls.gls_writer_open(str(tmp_path / "b.bin"), None, 1, 4, 0, 0)[0] == -7
    # a block before the base problem is refused without writing
    rc, w = gls.gls_writer_open(str(tmp_path / "b.bin"), None, 1, 4, 10, 2)
    b = np.zeros((3, 1, 4))
    assert gls.gls_writer_sink(w, 9, 3, b.ctypes.data, None) != 0
    assert gls.gls_writer_close(w)[0] == 0
    # a device that refuses writes: the failure reaches the sink and the close
    if os.path.exists("/dev/full"):
        rc, w = gls.gls_writer_open("/dev/full", None, 1, 4, 0, 1)
        if rc == 0:
            gls.gls_writer_sink(w, 0, 3, b.ctypes.data, None)
            assert gls.gls_writer_close(w)[0] == gls.GLS_E_IO
