"""Streamed genotypes (Alg. 8 form) through gls_solve_stream: bitwise equal
to the in-core solve of the same problems, resumable at a block boundary,
and within the oracle tolerance."""
import sys

import numpy as np
import pytest

from oracle import gls_oracle as orc
from paper_1210_7325_amd import datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def mods():
    from paper_1210_7325_amd import gls, stream
    gls.lib()
    return gls, stream


def to_dev(a):
    return torch.from_numpy(np.asfortranarray(a)).cuda()


def cohort(gls, w, prec="fp64"):
    M, XL, Y = dg.make_M(w), dg.make_XL(w), dg.make_Y(w)
    c = gls.Cohort(to_dev(M), precision=prec).whiten_fixed(to_dev(XL), to_dev(Y), intercept_col=0)
    return c, M, XL, Y


W = dg.STREAM.replace(n=700, q=1400, m=1000, block=128, seed=dg.MASTER_SEED + 40)


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_stream_equals_in_core_bitwise(mods, prec):
    gls, stream = mods
    say("stream vs in-core", prec)
    c, M, XL, Y = cohort(gls, W, prec)
    fill, ctx = stream.workload_fill(W)
    B, info, st = stream.solve_stream(c, 0, W.m, W.block, W.p_R, fill, ctx)
    assert st["blocks"] == (W.m + W.block - 1) // W.block
    Bin, info_in = c.solve_block(to_dev(dg.make_XR(W, 0, W.m)), p_R=W.p_R)
    torch.cuda.synchronize()
    assert np.array_equal(B, Bin.cpu().numpy())
    assert np.all(info == 0) and np.all(info_in.cpu().numpy() == 0)
    ref = orc.gls_sequence(M, XL, dg.make_XR(W, 0, W.m), Y, W.p_R)
    assert orc.relative_error(B, ref).max() < (1e-10 if prec == "fp64" else 1e-8)
    c.free()


def test_stream_abort_and_resume(mods):
    gls, stream = mods
    say("stream resume")
    c, *_ = cohort(gls, W)
    fill, ctx = stream.workload_fill(W)
    full, _, _ = stream.solve_stream(c, 0, W.m, W.block, W.p_R, fill, ctx)
    out = np.full((W.m, W.t, W.p), np.nan)
    done = []

    def stop_after_three(snp0, nsnp):
        done.append(snp0 + nsnp)
        return len(done) < 3

    with pytest.raises(gls.GLSError) as e:
        stream.solve_stream(c, 0, W.m, W.block, W.p_R, fill, ctx, out=out, on_block=stop_after_three)
    assert e.value.code == 7                           # GLS_E_ABORTED
    resume = done[-1]
    assert resume == 3 * W.block
    stream.solve_stream(c, resume, W.m, W.block, W.p_R, fill, ctx, out=out)
    assert np.array_equal(out, full)
    c.free()


def test_stream_python_fill(mods):
    """Any host source works: here a numpy array read through a callback."""
    gls, stream = mods
    say("stream python fill")
    w = W.replace(m=300)
    c, M, XL, Y = cohort(gls, w)
    XR = np.ascontiguousarray(dg.make_XR(w, 0, w.m).T)  # (columns, n)

    def fill(_ctx, snp0, nsnp, buf, ld):
        dst = np.ctypeslib.as_array(ctypes_cast(buf), shape=(nsnp * w.p_R * ld,))
        dst.reshape(nsnp * w.p_R, ld)[:, :w.n] = XR[snp0 * w.p_R:(snp0 + nsnp) * w.p_R]
        return 0

    B, info, st = stream.solve_stream(c, 0, w.m, 64, w.p_R, fill, None)
    ref = orc.gls_sequence(M, XL, XR.T, Y, w.p_R)
    assert orc.relative_error(B, ref).max() < 1e-10
    c.free()


def ctypes_cast(addr):
    import ctypes
    return ctypes.cast(addr, ctypes.POINTER(ctypes.c_int8))


@pytest.mark.parametrize("direct", [False, True])
def test_stream_from_file_equals_generator(mods, tmp_path, direct):
    """Disk-backed form: the genotypes written to a file and read back by the
    library's reader (gls_file_fill) give the same bits as the in-memory
    generator; a file shorter than the run aborts the stream cleanly."""
    gls, stream = mods
    say("stream from file, direct", direct)
    c, M, XL, Y = cohort(gls, W)
    fill, ctx = stream.workload_fill(W)
    ref, _, _ = stream.solve_stream(c, 0, W.m, W.block, W.p_R, fill, ctx)
    path = str(tmp_path / "genotypes.bin")
    stream.write_genotype_file(path, W, W.m)
    with stream.FileSource(path, W.n, W.p_R, direct=direct, threads=4) as src:
        B, info, st = stream.solve_stream(c, 0, W.m, W.block, W.p_R, src.fill, src.ctx)
        nbytes, _ = src.stats()
    assert np.array_equal(B, ref) and np.all(info == 0)
    assert nbytes == W.n * W.p_R * W.m
    # the file-fed results against the oracle, every problem
    ref_o = orc.gls_sequence(M, XL, dg.make_XR(W, 0, W.m), Y, W.p_R)
    assert orc.relative_error(B, ref_o).max() < 1e-10
    short = str(tmp_path / "short.bin")
    stream.write_genotype_file(short, W, W.m - 3 * W.block)
    with stream.FileSource(short, W.n, W.p_R) as src:
        with pytest.raises(gls.GLSError) as e:
            stream.solve_stream(c, 0, W.m, W.block, W.p_R, src.fill, src.ctx)
        assert e.value.code == 7                       # GLS_E_ABORTED: the fill failed
    c.free()


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_stream_file_to_file(mods, tmp_path, prec):
    """The whole out-of-core loop of Alg. 8 through the library: genotypes
    read from a file by gls_file_fill, results written to files by the
    asynchronous writer (gls_writer_sink); the files hold the in-core
    results bit for bit, within the oracle's tolerance."""
    gls, stream = mods
    say("stream file to file", prec)
    c, M, XL, Y = cohort(gls, W, prec)
    gpath = str(tmp_path / "genotypes.bin")
    stream.write_genotype_file(gpath, W, W.m)
    bpath, ipath = str(tmp_path / "b.bin"), str(tmp_path / "info.bin")
    with stream.FileSource(gpath, W.n, W.p_R, direct=True, threads=4) as src:
        wr = stream.FileWriter(bpath, ipath, W.t, W.p, snp_base=0, depth=2)
        try:
            st = stream.solve_stream_to(c, 0, W.m, W.block, W.p_R, src.fill, src.ctx, wr.sink, wr.ctx)
        finally:
            wst = wr.close()
    assert st["blocks"] == (W.m + W.block - 1) // W.block
    assert wst["bytes"] == W.m * (W.t * W.p * 8 + 4)
    B = np.fromfile(bpath, dtype=np.float64).reshape(W.m, W.t, W.p)
    info = np.fromfile(ipath, dtype=np.int32)
    Bin, info_in = c.solve_block(to_dev(dg.make_XR(W, 0, W.m)), p_R=W.p_R)
    torch.cuda.synchronize()
    assert np.array_equal(B, Bin.cpu().numpy()) and np.all(info == 0)
    ref = orc.gls_sequence(M, XL, dg.make_XR(W, 0, W.m), Y, W.p_R)
    assert orc.relative_error(B, ref).max() < (1e-10 if prec == "fp64" else 1e-8)
    c.free()
