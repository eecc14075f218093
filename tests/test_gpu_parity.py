"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerance: 1e-10 relative error of b_i (max norm per problem) for the FP64
path; intermediate quantities (L, W = L^{-1}X, fixed blocks) within 1e-12."""
import sys

import numpy as np
import pytest

from oracle import gls_oracle as orc
from paper_1210_7325_amd import datagen as dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_B = 1e-10
TOL_MID = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def G():
    from paper_1210_7325_amd import gls
    gls.lib()
    assert torch.cuda.is_available()
    return gls


def to_dev(a):
    return torch.from_numpy(np.asfortranarray(a)).cuda()


def small_problem(n, pL=3, pR=1, m=40, t=1, seed=0, q=None):
    w = dg.SMALL.replace(n=n, p_L=pL, p_R=pR, t=t, m=m, q=q or 2 * n, seed=dg.MASTER_SEED + 100 + seed)
    M = dg.make_M(w)
    XL = dg.make_XL(w)
    Y = dg.make_Y(w)
    XR = dg.make_XR(w, 0, m)
    return w, M, XL, Y, XR


def maxrel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(np.asarray(b))))


@pytest.mark.parametrize("n", [40, 127, 128, 129, 300, 1000])
def test_factor_matches_cholesky(G, n):
    say("factor n=", n)
    w, M, *_ = small_problem(n)
    c = G.Cohort(to_dev(M))
    L = c.copy_factor().cpu().numpy()
    torch.cuda.synchronize()
    Lref = orc.cholesky_lower(M)
    assert maxrel(L, Lref) < TOL_MID
    assert np.all(np.triu(L, 1) == 0)
    c.free()


def test_factor_reports_not_spd(G):
    say("factor not SPD")
    n = 300
    M = np.eye(n)
    M[200, 200] = -1.0
    with pytest.raises(G.GLSError) as ei:
        G.Cohort(to_dev(M))
    assert ei.value.code == G.GLS_E_NOT_SPD
    rc, h = G.gls_factor(n, to_dev(M).data_ptr(), n, 0, torch.cuda.current_stream().cuda_stream)
    assert rc == G.GLS_E_NOT_SPD and G.gls_last_info(h) == 201
    G.gls_free(h)


@pytest.mark.parametrize("n,ncols", [(1000, 200), (129, 65), (300, 1), (513, 130)])
def test_whiten_block_matches_oracle(G, n, ncols):
    say("whiten n=", n, "ncols=", ncols)
    w, M, XL, Y, XR = small_problem(n, m=ncols)
    c = G.Cohort(to_dev(M))
    W = c.whiten_block(to_dev(XR)).cpu().numpy()
    Wref = orc.whiten(orc.cholesky_lower(M), XR)
    assert maxrel(W, Wref) < TOL_MID
    c.free()


@pytest.mark.parametrize("n,ncols,slab", [(1000, 200, 0), (129, 65, 16), (660, 300, 64),
                                           (513, 130, 128), (1000, 4, 0), (700, 3000, 0)])
def test_whiten_block_f64_matches_oracle(G, n, ncols, slab):
    """FP64 right-hand sides (whole design matrices: covariates, phenotypes,
    genotypes as doubles) through gls_whiten_block_f64, each slab width;
    n = 660 leaves its last row block to the last-block kernel."""
    say("whiten f64 n=", n, "ncols=", ncols, "slab", slab)
    rng = np.random.default_rng(n + ncols)
    w, M, XL, Y, XR = small_problem(n, m=4)
    X = rng.standard_normal((n, ncols))
    c = G.Cohort(to_dev(M))
    c.set_slab_cols(slab)
    W = c.whiten_block(to_dev(X)).cpu().numpy()
    Wref = orc.whiten(orc.cholesky_lower(M), X)
    assert maxrel(W, Wref) < TOL_MID
    c.free()


@pytest.mark.parametrize("pL,t", [(3, 1), (16, 1), (5, 8), (1, 2)])
def test_fixed_part_matches_oracle(G, pL, t):
    say("fixed pL=", pL, "t=", t)
    w, M, XL, Y, XR = small_problem(700, pL=pL, t=t)
    c = G.Cohort(to_dev(M)).whiten_fixed(to_dev(XL), to_dev(Y))
    WL, Yt, STL, CT = (x.cpu().numpy() for x in c.copy_fixed())
    WLr, Ytr, STLr, CTr = orc.fixed_blocks(orc.cholesky_lower(M), XL, Y)
    assert maxrel(WL, WLr) < TOL_MID and maxrel(Yt, Ytr) < TOL_MID
    assert maxrel(STL, STLr) < TOL_MID and maxrel(CT, CTr) < TOL_MID
    c.free()


def run_gpu(M, XL, Y, XR, pR, block):
    from paper_1210_7325_amd import gls
    c = gls.Cohort(to_dev(M)).whiten_fixed(to_dev(XL), to_dev(Y))
    dXR = to_dev(XR)
    nsnp = XR.shape[1] // pR
    outs, infos = [], []
    for a in range(0, nsnp, block):
        b = min(nsnp, a + block)
        B, info = c.solve_block(dXR[:, a * pR:b * pR], p_R=pR)
        outs.append(B)
        infos.append(info)
    B = torch.cat(outs).cpu().numpy()
    info = torch.cat(infos).cpu().numpy()
    c.free()
    return B, info


def test_small_workload_parity(G):
    """The n=1000, p=4, m=10,000 workload in blocks of 4096 (last one partial)."""
    w = dg.SMALL
    say("workload", w.name)
    M, XL, Y, XR = dg.make_all(w)
    B, info = run_gpu(M, XL, Y, XR, w.p_R, w.block)
    ref = orc.gls_sequence(M, XL, XR, Y, w.p_R)
    assert B.shape == ref.shape
    assert np.all(info == 0)
    err = orc.relative_error(B, ref)
    say("max rel err", err.max())
    assert err.max() < TOL_B


@pytest.mark.parametrize("n,pL,pR,t,m,block", [
    (63, 3, 1, 1, 37, 16), (64, 2, 2, 1, 20, 7), (65, 4, 3, 2, 33, 33), (129, 16, 4, 1, 50, 17),
    (200, 5, 1, 8, 70, 64), (300, 1, 1, 1, 5, 5), (1500, 3, 1, 1, 300, 256), (257, 19, 1, 3, 40, 40),
    # genotype blocks wider than one column: problems per 16-column tile
    # floor(16 / p_R) = 3, 2, 1, 1 (tiles left partly empty), two F tiles
    (300, 2, 5, 2, 45, 19), (150, 3, 7, 3, 21, 10), (333, 10, 9, 8, 13, 13), (200, 1, 16, 1, 9, 4),
    (401, 2, 3, 1, 150, 150),
])
def test_ragged_shapes_parity(G, n, pL, pR, t, m, block):
    say("ragged", n, pL, pR, t, m, block)
    w, M, XL, Y, XR = small_problem(n, pL=pL, pR=pR, m=m, t=t, seed=n + pL)
    B, info = run_gpu(M, XL, Y, XR, pR, block)
    ref = orc.gls_sequence(M, XL, XR, Y, pR)
    assert np.all(info == 0)
    assert orc.relative_error(B, ref).max() < TOL_B


def test_rank_deficient_problem_sets_info(G):
    say("rank deficient")
    w, M, XL, Y, XR = small_problem(200, m=10)
    XR = XR.copy()
    XR[:, 3] = 0  # X_i has a zero column: S_i singular
    B, info = run_gpu(M, XL, Y, XR, 1, 10)
    assert info[3] == 4 and np.all(np.isnan(B[3]))
    keep = [i for i in range(10) if i != 3]
    assert np.all(info[keep] == 0)
    ref = orc.gls_sequence(M, XL, XR[:, keep], Y)
    assert orc.relative_error(B[keep], ref).max() < TOL_B


def test_deterministic_and_block_independent(G):
    say("determinism")
    w, M, XL, Y, XR = small_problem(500, m=300)
    B1, _ = run_gpu(M, XL, Y, XR, 1, 300)
    B2, _ = run_gpu(M, XL, Y, XR, 1, 300)
    B3, _ = run_gpu(M, XL, Y, XR, 1, 64)
    assert np.array_equal(B1, B2)
    # a problem's result does not depend on the block it is solved in
    assert np.array_equal(B1, B3)


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("n", [700, 660])
def test_slab_width_choice_is_bitwise_neutral(G, prec, n):
    """Automatic per-launch slab width (the default) against every fixed
    width: the same bits, for launches small enough to pick 16 or 32,
    middling (64) and large enough to pick 128 columns per work-group.
    n = 660 leaves its last row block to the last-block kernel (in every
    width), n = 700 does not."""
    say("slab widths", prec, n)
    from paper_1210_7325_amd import gls
    w, M, XL, Y, XR = small_problem(n, m=40000)
    c = gls.Cohort(to_dev(M), precision=prec).whiten_fixed(to_dev(XL), to_dev(Y), intercept_col=0)
    dXR = to_dev(XR)
    widths = (32, 64, 128) if prec == "fp32_refine" else (16, 32, 64, 128)
    for m in (100, 5000, 20000, 40000):
        c.set_slab_cols(0)
        ref, _ = c.solve_block(dXR[:, :m])
        ref = ref.cpu().numpy()
        for C in widths:
            c.set_slab_cols(C)
            B, _ = c.solve_block(dXR[:, :m])
            assert np.array_equal(B.cpu().numpy(), ref), (m, C)
    c.free()


@pytest.mark.parametrize("n,m,block,pR", [(660, 300, 300, 1), (1000, 700, 333, 1), (64, 50, 50, 1),
                                          (129, 90, 45, 1), (200, 300, 300, 1), (300, 100, 60, 3),
                                          (450, 40, 40, 7)])
def test_wide_slabs_parity(G, n, m, block, pR):
    """128 genotype columns per work-group (operands staged through LDS):
    within the bound of the oracle and the same bits as 64.  n = 660 leaves
    its last row block of 20 rows to the last-block kernel; n = 1000 ends in
    a partial row block of the main kernel; n = 64 has one row block (no
    off-diagonal product), n = 129 two with the second left to the
    last-block kernel, n = 200 two with one stage ring pass; every block
    ends in a partial slab.  p_R = 3 and 7: problems of several genotype
    columns, several problems per 16-column tile of a 128-column slab."""
    say("128-column slabs", n, m, block, pR)
    from paper_1210_7325_amd import gls
    w, M, XL, Y, XR = small_problem(n, pR=pR, m=m, seed=n + 3)
    c = gls.Cohort(to_dev(M)).whiten_fixed(to_dev(XL), to_dev(Y))
    dXR = to_dev(XR)
    outs = {}
    for C in (128, 64):
        c.set_slab_cols(C)
        parts = [c.solve_block(dXR[:, a * pR:min(m, a + block) * pR], p_R=pR)
                 for a in range(0, m, block)]
        assert all(np.all(i.cpu().numpy() == 0) for _, i in parts)
        outs[C] = torch.cat([b for b, _ in parts]).cpu().numpy()
    c.free()
    ref = orc.gls_sequence(M, XL, XR, Y, pR)
    err = orc.relative_error(outs[128], ref)
    say("max rel err", err.max())
    assert err.max() < TOL_B
    assert np.array_equal(outs[128], outs[64])


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("n,pad,offset", [(1000, 5, 0), (1000, 16, 3), (203, 13, 1)])
def test_genotypes_with_a_padded_leading_dimension(G, prec, n, pad, offset):
    """X_R inside a larger column-major array (ldxr = n + pad, the block
    starting `offset` rows down): the same bits as the packed array.  Covers
    the aligned and the unaligned loads of the centering pre-pass."""
    say("padded ld", prec, n, pad, offset)
    from paper_1210_7325_amd import gls
    w, M, XL, Y, XR = small_problem(n, m=150)
    c = gls.Cohort(to_dev(M), precision=prec).whiten_fixed(to_dev(XL), to_dev(Y), intercept_col=0)
    ref, _ = c.solve_block(to_dev(XR))
    big = np.full((n + pad, XR.shape[1]), 7, dtype=np.int8)
    big[offset:offset + n] = XR
    dbig = to_dev(big)
    view = dbig[offset:offset + n]                 # stride(1) = n + pad
    assert view.stride(0) == 1 and view.stride(1) == n + pad
    B, info = c.solve_block(view)
    assert np.array_equal(B.cpu().numpy(), ref.cpu().numpy())
    assert np.all(info.cpu().numpy() == 0)
    c.free()


@pytest.mark.parametrize("prec,slab", [("fp64", 0), ("fp64", 128), ("fp32_refine", 128)])
def test_multi_cohort_launch_equals_single(G, prec, slab):
    """One launch over cohorts of different n (K = 3, 6 and 2 row blocks:
    with 128-column slabs the paired-block solve meets a lone last block,
    three pairs, and a last block left to the last-block kernel in the same
    launch) gives each cohort the bits of its own launch."""
    say("multi", prec, slab)
    from paper_1210_7325_amd import gls
    probs = [small_problem(n, pL=pL, pR=pR, m=m, t=t, seed=i)
             for i, (n, pL, pR, t, m) in enumerate([(300, 3, 1, 1, 100), (700, 5, 2, 2, 64),
                                                      (129, 2, 1, 1, 30)])]
    alone, items, cohorts = [], [], []
    for (w, M, XL, Y, XR), pR in zip(probs, (1, 2, 1)):
        c = gls.Cohort(to_dev(M), precision=prec).whiten_fixed(to_dev(XL), to_dev(Y), intercept_col=0)
        c.set_slab_cols(slab)
        dXR = to_dev(XR)
        B, _ = c.solve_block(dXR, p_R=pR)
        alone.append(B.cpu().numpy())
        B2 = torch.empty_like(B)
        info2 = torch.empty(B.shape[0], dtype=torch.int32, device="cuda")
        items.append((c, dXR, pR, B2, info2))
        cohorts.append(c)
    gls.solve_multi(items)
    torch.cuda.synchronize()
    for (c, dXR, pR, B2, info2), a in zip(items, alone):
        assert np.array_equal(B2.cpu().numpy(), a)
        assert int(info2.abs().sum()) == 0
    for c in cohorts:
        c.free()


def test_forked_streams_equal(G):
    say("fork")
    from paper_1210_7325_amd import gls
    w, M, XL, Y, XR = small_problem(600, m=512)
    c = gls.Cohort(to_dev(M)).whiten_fixed(to_dev(XL), to_dev(Y))
    dXR = to_dev(XR)
    Bref, _ = c.solve_block(dXR)
    torch.cuda.synchronize()
    forks = [c.fork() for _ in range(3)]
    outs = []
    for i, f in enumerate(forks):
        with torch.cuda.stream(f.stream):
            outs.append(f.solve_block(dXR[:, 128 * i:128 * (i + 1)])[0])
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert np.array_equal(o.cpu().numpy(), Bref[128 * i:128 * (i + 1)].cpu().numpy())
    for f in forks:
        f.free()
    c.free()


def test_full_scale_sampled_in_bench_configuration(G):
    """n = 10,000, p = 4, m = 1,000,000 in blocks of 4096, eight blocks per
    launch in slabs of the automatic width (128 columns) exactly as bench.py
    times it; 300 problems sampled across the whole sequence (first, last
    partial block, and a stride) checked one by one against the oracle."""
    import bench
    w = dg.SCALE
    say("full scale", w.name)
    M = dg.make_M(w)
    XL, Y = dg.make_XL(w), dg.make_Y(w)
    dM = torch.from_numpy(M).cuda()
    dXL, dY = to_dev(XL), to_dev(Y)
    dXR = bench.upload_genotypes(torch, w, w.m)
    Bout = torch.empty((w.m, w.t, w.p), dtype=torch.float64, device="cuda")
    info = torch.full((w.m,), -7, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    bench.run_step(G, torch, dM, dXL, dY, dXR, w, w.m, w.block, [stream], 0, Bout, info, batch=8)
    torch.cuda.synchronize()
    assert int((info != 0).sum()) == 0
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([np.arange(4), np.arange(w.m - 4, w.m),
                                    rng.choice(w.m, 292, replace=False)]))
    B = Bout[torch.from_numpy(idx).cuda()].cpu().numpy()
    XRs = np.concatenate([dg.make_XR(w, int(i), 1) for i in idx], axis=1)
    ref = orc.gls_sequence(M, XL, XRs, Y, w.p_R)
    err = orc.relative_error(B, ref)
    say("full scale sampled max rel err", err.max())
    assert err.max() < TOL_B
    del dXR


def test_layout_copies_are_ordered_on_the_handle_stream(G):
    """Row-major inputs are copied to column-major on the handle's own stream
    before the library's kernels read them (the copy used to run on the
    current stream and could race a factorization on a side stream)."""
    say("row-major inputs on a side stream")
    w, M, XL, Y, XR = small_problem(3000, pL=4, m=200, seed=31)
    side = torch.cuda.Stream()
    Lref = orc.cholesky_lower(M)
    ref = orc.gls_sequence(M, XL, XR, Y, 1)
    for rep in range(3):
        Mr = torch.from_numpy(np.ascontiguousarray(M)).cuda()        # row-major
        XLr = torch.from_numpy(np.ascontiguousarray(XL)).cuda()
        Yr = torch.from_numpy(np.ascontiguousarray(Y)).cuda()
        XRr = torch.from_numpy(np.ascontiguousarray(XR)).cuda()
        torch.cuda.synchronize()
        c = G.Cohort(Mr, stream=side).whiten_fixed(XLr, Yr)
        B, info = c.solve_block(XRr)
        side.synchronize()
        assert maxrel(c.copy_factor().cpu().numpy(), Lref) < TOL_MID
        assert orc.relative_error(B.cpu().numpy(), ref).max() < TOL_B
        c.free()


def test_workspace_regrowth_after_launch_on_another_stream(G):
    """A block solved through gls_solve_multi on a stream other than the
    handle's, then a larger block on the handle's own stream (the workspace
    grows while the first launch may still read it): both results match the
    oracle."""
    say("workspace regrowth across streams")
    w, M, XL, Y, XR = small_problem(900, m=3000, seed=5)
    c = G.Cohort(to_dev(M)).whiten_fixed(to_dev(XL), to_dev(Y))
    dXR = to_dev(XR)
    other = torch.cuda.Stream()
    Ba = torch.empty((200, 1, 4), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    G.solve_multi([(c, dXR[:, :200], 1, Ba, None)], stream=other)
    Bb, _ = c.solve_block(dXR, p_R=1)          # 3000 columns: the workspace grows
    torch.cuda.synchronize()
    ref = orc.gls_sequence(M, XL, XR, Y, 1)
    assert orc.relative_error(Ba.cpu().numpy(), ref[:200]).max() < 1e-10
    assert orc.relative_error(Bb.cpu().numpy(), ref).max() < 1e-10
    c.free()


@pytest.mark.parametrize("prec,pR,t", [("fp64", 1, 1), ("fp64", 3, 2), ("fp32_refine", 1, 2)])
def test_rounds_split_items_bitwise(G, prec, pR, t):
    """One cohort's work beyond one round of work-groups (more 64-column
    slabs than compute units) goes out as a launch that fills the round and
    one for the rest at its own width, splitting an item between the two:
    the same bits as the same items at one fixed width (one launch), and
    within the oracle's bound on a sample of problems, the split item's
    included."""
    from paper_1210_7325_amd import gls
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n = 300
    per_item = (cus * 64 * 11 // 10) // 3 // pR   # problems per item: 1.1 rounds of 64-column slabs in all
    m = 3 * per_item
    say("rounds", prec, pR, t, "cus", cus, "problems", m)
    w, M, XL, Y, XR = small_problem(n, pR=pR, m=m, t=t, seed=17 + pR)
    dXR = to_dev(XR)
    outs = {}
    for C in (0, 64):
        c = gls.Cohort(to_dev(M), precision=prec).whiten_fixed(to_dev(XL), to_dev(Y), intercept_col=0)
        hs = [c] + [c.fork(torch.cuda.current_stream()) for _ in range(2)]
        for h in hs:
            h.set_slab_cols(C)
        p = 3 + pR
        B = torch.full((m, t, p), float("nan"), dtype=torch.float64, device="cuda")
        info = torch.full((m,), -7, dtype=torch.int32, device="cuda")
        items = [(hs[j], dXR[:, j * per_item * pR:(j + 1) * per_item * pR], pR,
                  B[j * per_item:(j + 1) * per_item], info[j * per_item:(j + 1) * per_item]) for j in range(3)]
        gls.solve_multi(items, stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        outs[C] = (B.cpu().numpy(), info.cpu().numpy())
        for h in hs[1:]:
            h.free()
        c.free()
    assert np.all(outs[0][1] == 0) and np.all(outs[64][1] == 0)
    assert np.array_equal(outs[0][0], outs[64][0])
    # the third item is split between the two launches: sample around its split
    split = 2 * per_item + (cus - 2 * ((per_item * pR + 63) // 64)) * 64 // pR
    idx = np.unique(np.clip(np.array([0, per_item - 1, per_item, 2 * per_item, split - 2, split - 1, split,
                                      split + 1, m - 1]), 0, m - 1))
    XRs = np.concatenate([XR[:, i * pR:(i + 1) * pR] for i in idx], axis=1)
    ref = orc.gls_sequence(M, XL, XRs, Y, pR)
    err = orc.relative_error(outs[0][0][idx], ref)
    say("max rel err", err.max())
    assert err.max() < (1e-10 if prec == "fp64" else 1e-8)


@pytest.mark.parametrize("prec", ["fp64", "fp32_refine"])
def test_kernel_launch_record(G, prec):
    """The per-launch timing record (gls_kernel_launches): one entry per
    launch of the triangular solve, in launch order, whose columns add up to
    the call's right-hand sides, whose durations add up to gls_kernel_time's
    sum, and whose slab widths show the rounds: a first launch of at most
    one slab per compute unit, then the rest at a width of its own."""
    from paper_1210_7325_amd import gls
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    m = cus * 64 * 11 // 10
    say("launch record", prec, "cus", cus, "problems", m)
    w, M, XL, Y, XR = small_problem(300, m=m, seed=23)
    c = gls.Cohort(to_dev(M), precision=prec).whiten_fixed(to_dev(XL), to_dev(Y), intercept_col=0)
    c.set_kernel_timing(True)
    B, info = c.solve_block(to_dev(XR), p_R=1)
    torch.cuda.synchronize()
    rec = c.kernel_launches(0)
    ms, cnt = c.kernel_time(0)
    asm = c.kernel_launches(1)
    c.free()
    say("record", rec)
    assert np.all(info.cpu().numpy() == 0)
    assert len(rec) == cnt >= 2
    assert sum(r[1] for r in rec) == m
    assert abs(sum(r[0] for r in rec) - ms) <= 1e-6 * ms
    assert all(r[0] > 0 and r[2] in (16, 32, 64, 128) for r in rec)
    assert rec[0][1] <= cus * rec[0][2]
    # kind 1: each launch of the solve is followed by one of the assembly,
    # preceded in the FP32_REFINE form by the centering pre-pass
    per = 2 if prec == "fp32_refine" else 1
    assert len(asm) == per * len(rec)
    assert [r[1] for r in asm[per - 1::per]] == [r[1] for r in rec]
    assert [r[1] for r in asm[::per]] == [r[1] for r in rec]
