"""Throughput of the GLS-sequence hot path on one MI355X.

One step = one whole pass of the in-core algorithm (Sec. 2, Alg. 5) over
the throughput workload: factor M (n = 10,000), whiten X_L and y, then solve
m = 1,000,000 single-SNP problems (p = 4) in blocks of 4096 SNPs, every
input resident in HBM before the clock starts.  Blocks are handed `--batch`
at a time to one launch (gls_solve_multi over handles that share the factor
through gls_fork, each with its own workspace), so a single launch fills the
chip.

The same steps are then timed in the FP32_REFINE form, and both forms are
checked against the CPU oracle on a sample of problems.  `--workload mixed`
runs the p = 20 (p_L = 16, p_R = 4) mixed-precision workload instead.

Prints ONE JSON line; progress goes to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload scale|mixed]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1210_7325_amd import datagen as dg  # noqa: E402

METRIC = "GLS solves/sec (b_i/s) at n=1e4,p=4; TRSM % of FP64/FP32 MFMA peak"
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# the paper's in-core/out-of-core time for n=10^4, p=4, m=10^6 on 12 Xeon
# cores (Table 3): 816 s, i.e. 1,225 solves/s
PAPER_BI_PER_S = 1_000_000 / 816.0
WORKLOADS = {"scale": dg.SCALE, "mixed": dg.MIXED, "stream": dg.STREAM, "serve": dg.SERVE_BASE,
             "ablation": dg.SCALE, "phenotypes": dg.PHENO}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="scale")
    ap.add_argument("--m", type=int, default=None, help="problems per step (default: workload m)")
    ap.add_argument("--block", type=int, default=None, help="SNPs per solve call (default 4096)")
    ap.add_argument("--streams", type=int, default=1)
    ap.add_argument("--batch", type=int, default=None,
                    help="blocks whitened per launch (default: enough columns for one slab of "
                         "the widest width, 128, per CU)")
    ap.add_argument("--slab-cols", type=int, default=0,
                    help="columns per work-group of the solve: 16 (FP64 only), 32, 64, 128, "
                         "or 0 to let the library choose per launch")
    ap.add_argument("--forms", default="fp64,fp32_refine",
                    help="precisions to time, the first is the headline")
    ap.add_argument("--parity-sample", type=int, default=1000,
                    help="problems checked against the oracle per form (0 skips)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget of the oracle's CPU sample (0 skips it)")
    ap.add_argument("--serve-jobs", type=int, default=16, help="jobs in the serving mix")
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="offered load of the Poisson arrivals, relative to 50 TFLOP/s")
    ap.add_argument("--serve-m-max", type=float, default=2e6,
                    help="upper end of the log-uniform m range (the full mix uses 1e7)")
    ap.add_argument("--serve-streams", type=int, default=2,
                    help="serving: compute streams the rounds alternate over")
    ap.add_argument("--serve-target-cols", type=int, default=32768,
                    help="genotype columns a serving round aims at (items grow together up to it)")
    ap.add_argument("--serve-inflight", type=int, default=4,
                    help="serving: rounds queued on the device at once")
    ap.add_argument("--serve-ingest", choices=("host", "device"), default="host",
                    help="serving: job genotypes produced on the host and copied through pinned "
                         "staging (host), or generated in device memory (device)")
    ap.add_argument("--stream-source", choices=("generator", "file"), default="generator",
                    help="stream workload: genotypes from the host generator or from a file "
                         "read by the library's reader (written first, removed after)")
    ap.add_argument("--stream-sink", choices=("memory", "file"), default="memory",
                    help="stream workload: results to host memory, or to a file written by the "
                         "library's asynchronous writer (removed after the run)")
    ap.add_argument("--stream-file", default=None,
                    help="genotype file for --stream-source file (default: under $TMPDIR)")
    ap.add_argument("--stream-direct", type=int, default=1,
                    help="read the genotype file with O_DIRECT (page cache bypassed) when possible")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (for scaling HBM counters)")
    return ap.parse_args()


def measured_traffic(batch, slab_cols, precision):
    """HBM bytes per launch of the FP64 triangular-solve kernel from the
    committed rocprofv3 counter summary, or None if the kernel source has
    changed since the counters were taken (or the launch shape differs)."""
    from paper_1210_7325_amd.build import trsm_source_digest
    if precision != "fp64":
        return None
    path = os.path.join(ROOT, "profiles", "trsm_fp64_n10000_traffic.md")
    try:
        kv = dict(l.split(": ", 1) for l in open(path).read().splitlines() if ": " in l)
        if kv.get("kernel_source_sha256") != trsm_source_digest() \
                or int(kv["blocks_per_launch"]) != batch \
                or slab_cols not in (0, int(kv["slab_cols"])):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration():
    """A plain copy of a known size (1 GiB read + 1 GiB written), run under
    rocprofv3 --pmc to scale FETCH_SIZE / WRITE_SIZE readings."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": src.numel() * 8, "dispatches": 3}))


def upload_genotypes(torch, w, m):
    """X_R for problems 0..m-1 as an int8 (n, m*p_R) column-major device tensor,
    generated on the host in chunks and copied through pinned memory."""
    ncols = m * w.p_R
    dev = torch.empty((ncols, w.n), dtype=torch.int8, device="cuda")
    chunk = max(w.p_R, (256 << 20) // w.n // w.p_R * w.p_R)
    pinned = [torch.empty((chunk, w.n), dtype=torch.int8).pin_memory() for _ in range(2)]
    done = [None, None]
    t0 = time.time()
    for i, a in enumerate(range(0, m, chunk // w.p_R)):
        b = min(m, a + chunk // w.p_R)
        k = i % 2
        if done[k] is not None:
            done[k].synchronize()
        buf = pinned[k]
        dg.make_XR(w, a, b - a, out=buf.numpy())
        dev[a * w.p_R:b * w.p_R].copy_(buf[:(b - a) * w.p_R], non_blocking=True)
        ev = torch.cuda.Event()
        ev.record()
        done[k] = ev
    torch.cuda.synchronize()
    log(f"genotypes: {ncols} columns x {w.n} in {time.time() - t0:.1f}s")
    return dev.t()


def run_step(gls, torch, dM, dXL, dY, dXR, w, m, block, streams, slab_cols, Bout, info,
             timing=False, batch=4, precision="fp64", phases=None):
    """One full pass: factor, whiten, all blocks.  `batch` blocks of `block`
    SNPs are whitened by one launch (gls_solve_multi over forked handles,
    each with its own workspace); launch groups rotate over `streams`.
    Returns the kernel times recorded by each group's first handle.  With
    `phases` (a list), four events on the first stream are appended: start,
    after the factorization, after the fixed part, after the last block."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if phases is not None else None
    if ev:
        ev[0].record(streams[0])
    c = gls.Cohort(dM, precision=precision, stream=streams[0])
    if ev:
        ev[1].record(streams[0])
    c.set_slab_cols(slab_cols)
    c.whiten_fixed(dXL, dY, intercept_col=0)
    if ev:
        ev[2].record(streams[0])
    groups = []
    for si, s in enumerate(streams):
        hs = [c if si == 0 and j == 0 else c.fork(s) for j in range(batch)]
        for h in hs:
            h.reserve(block * w.p_R)
        if timing:
            hs[0].set_kernel_timing(True)
        groups.append((s, hs))
    nblk = (m + block - 1) // block
    for gi, g0 in enumerate(range(0, nblk, batch)):
        s, hs = groups[gi % len(groups)]
        items = []
        for j, b in enumerate(range(g0, min(nblk, g0 + batch))):
            a, e = b * block, min(m, (b + 1) * block)
            items.append((hs[j], dXR[:, a * w.p_R:e * w.p_R], w.p_R, Bout[a:e], info[a:e]))
        gls.solve_multi(items, stream=s)
    times = None
    if timing:
        times = [(hs[0].kernel_time(0), hs[0].kernel_time(1), hs[0].kernel_launches(0))
                 for _, hs in groups]
    if ev:
        for s in streams[1:]:
            streams[0].wait_stream(s)
        ev[3].record(streams[0])
        phases.extend(ev)
    for s in streams:
        s.synchronize()
    for _, hs in groups:
        for h in hs:
            if h is not c:
                h.free()
    c.free()
    return times


def time_form(gls, torch, args, w, m, block, batch, dM, dXL, dY, dXR, Bout, info, precision):
    streams = [torch.cuda.Stream() for _ in range(args.streams)]
    for i in range(args.warmup):
        run_step(gls, torch, dM, dXL, dY, dXR, w, m, block, streams, args.slab_cols, Bout, info,
                 batch=batch, precision=precision)
        log(f"[{precision}] warmup step {i} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kt = []
    ph = []
    for i in range(args.steps):
        kt.append(run_step(gls, torch, dM, dXL, dY, dXR, w, m, block, streams, args.slab_cols,
                           Bout, info, timing=True, batch=batch, precision=precision,
                           phases=ph if i == args.steps - 1 else None))
        log(f"[{precision}] step {i} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # the last step split into factorization (a0), fixed part (a1) and the
    # sequence of blocks (a2-a4), from events on the first stream
    factor_ms, fixed_ms, solve_ms = (ph[j].elapsed_time(ph[j + 1]) for j in range(3))
    trsm_ms = sum(t[0][0] for step in kt for t in step)
    trsm_n = sum(t[0][1] for step in kt for t in step)
    asm_ms = sum(t[1][0] for step in kt for t in step)
    asm_n = sum(t[1][1] for step in kt for t in step)
    # algorithmic work of the triangular solve: n^2 flops per right-hand side.
    # The roofline is taken over the full launches (the widest slab and the
    # most columns: the dominant kernel's launches); the tail rounds of
    # narrower slabs are reported beside it, and the rate over all launches.
    per = [l for step in kt for t in step for l in t[2]]
    full = max((slab, cols) for _, cols, slab in per)
    full_l = [ms for ms, cols, slab in per if (slab, cols) == full]
    full_avg = sum(full_l) / len(full_l)
    flops_per_launch = float(w.n) ** 2 * full[1]
    achieved = flops_per_launch / (full_avg * 1e-3) / 1e12
    all_tflops = float(w.n) ** 2 * m * w.p_R * args.steps / (trsm_ms * 1e-3) / 1e12
    tail = [(ms, cols, slab) for ms, cols, slab in per[:len(per) // args.steps]
            if (slab, cols) != full]
    peak = PEAK_FP64_TFLOPS if precision == "fp64" else PEAK_FP32_TFLOPS
    step_tflops = float(w.n) ** 2 * m * w.p_R * args.steps / dt / 1e12
    r = {
        "value": m * args.steps / dt, "ms_per_step": dt / args.steps * 1e3,
        "trsm_launches": len(full_l), "trsm_avg_ms": full_avg, "full_cols": full[1],
        "full_slab": full[0], "tail_launches": [
            {"ms": round(ms, 3), "cols": cols, "slab": slab} for ms, cols, slab in tail],
        "all_launches": trsm_n, "all_avg_ms": trsm_ms / trsm_n, "all_tflops": all_tflops,
        "flops_per_launch": flops_per_launch, "trsm_tflops": achieved, "peak": peak,
        "step_tflops": step_tflops, "assemble_avg_ms": asm_ms / max(asm_n, 1),
        "rank_deficient": int((info != 0).sum()),
        "factor_ms": factor_ms, "fixed_ms": fixed_ms, "solve_ms": solve_ms,
    }
    log(f"[{precision}] {r['value']:.0f} b_i/s, {r['ms_per_step']:.1f} ms/step, TRSM "
        f"{achieved:.1f} TFLOP/s ({achieved / peak * 100:.1f}% of {peak}), step {step_tflops:.1f}")
    return r


def parity_sample(w, m, M, XL, Y, lu, outs, sample):
    """Max / p99.99 relative error of each form against the oracle on a
    sample of problems spread over the whole sequence."""
    from oracle import gls_oracle as orc
    rng = np.random.default_rng(12107325)
    idx = np.unique(np.concatenate([[0, m - 1], rng.choice(m, min(sample, m) - 2, replace=False)]))
    XRs = np.concatenate([dg.make_XR(w, int(i), 1) for i in idx], axis=1)
    ref = orc.gls_sequence(M, XL, XRs, Y, w.p_R, lu=lu)
    res = {}
    for name, B in outs.items():
        err = orc.relative_error(B[idx], ref)
        res[name] = {"max_rel_err": float(err.max()), "p9999_rel_err": float(np.quantile(err, 0.9999)),
                     "sample": int(len(idx))}
        log(f"[{name}] parity on {len(idx)} problems: max rel err {err.max():.3e}")
    return res


def host_alg5(M, XL, XR, Y, p_R=1, block=4096, L=None):
    """The paper's fast algorithm (Sec. 2, Alg. 5 "hp-gwas") with numpy/scipy
    BLAS on the host cores: a context figure beside the oracle, which
    computes the definition of Eq. (1) instead.  Not part of the oracle and
    not the product path.

    Steps in the paper's order: the Cholesky factor of M (potrf); W_L =
    L^{-1} X_L and ytil = L^{-1} y (trsm, trsv); S_TL = W_L^T W_L and
    C_T = W_L^T ytil (syrk, gemv); then per block of SNPs one triangular
    solve W_R = L^{-1} X_R of the whole block (the grouped trsm), and per
    problem S_BL = W_R_i^T W_L, S_BR = W_R_i^T W_R_i, C_B = W_R_i^T ytil,
    assembled with S_TL, C_T as in Fig. 1 and solved.  Output (m, t, p) like
    the library's b."""
    import scipy.linalg as sla
    Y = np.asarray(Y, dtype=np.float64)
    if Y.ndim == 1:
        Y = Y[:, None]
    if L is None:
        L = np.linalg.cholesky(np.asarray(M, dtype=np.float64))
    WL = sla.solve_triangular(L, np.asarray(XL, dtype=np.float64), lower=True)
    yt = sla.solve_triangular(L, Y, lower=True)
    STL, CT = WL.T @ WL, WL.T @ yt
    n, p_L = WL.shape
    t = yt.shape[1]
    m = XR.shape[1] // p_R
    p = p_L + p_R
    out = np.empty((m, t, p), dtype=np.float64)
    for a in range(0, m, block):
        b = min(m, a + block)
        k = b - a
        WR = sla.solve_triangular(L, np.asarray(XR[:, a * p_R:b * p_R], dtype=np.float64),
                                  lower=True)
        Wk = WR.T.reshape(k, p_R, n)                  # W_R_i^T, (k, p_R, n)
        S = np.empty((k, p, p))
        S[:, :p_L, :p_L] = STL
        SBL = Wk @ WL                                 # (k, p_R, p_L)
        S[:, p_L:, :p_L] = SBL
        S[:, :p_L, p_L:] = SBL.transpose(0, 2, 1)
        S[:, p_L:, p_L:] = Wk @ Wk.transpose(0, 2, 1)
        c = np.empty((k, p, t))
        c[:, :p_L] = CT
        c[:, p_L:] = Wk @ yt
        out[a:b] = np.linalg.solve(S, c).transpose(0, 2, 1)
    return out


def cpu_baseline(w, M, XL, Y, budget_s, lu=None, t_factor=None):
    """The oracle, as it stands, on the host cores: LU factorization of M plus
    per-problem solves on a bounded sample, extrapolated linearly in m."""
    from oracle import gls_oracle as orc
    import scipy.linalg as sla
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [os.cpu_count()])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    if lu is None:
        t0 = time.time()
        lu = sla.lu_factor(M)
        t_factor = time.time() - t0
    pilot = 512  # large enough that the per-problem estimate holds for the whole sample
    XR = dg.make_XR(w, 0, pilot)
    t0 = time.time()
    orc.gls_sequence(M, XL, XR, Y, w.p_R, lu=lu)
    t_pilot = time.time() - t0
    per = t_pilot / pilot
    sample = int(max(pilot, min(200_000, (budget_s - t_factor - t_pilot) / max(per, 1e-9))))
    XR = dg.make_XR(w, pilot, sample)
    t0 = time.time()
    orc.gls_sequence(M, XL, XR, Y, w.p_R, lu=lu)
    t_sample = time.time() - t0
    per = t_sample / sample
    total = t_factor + per * w.m
    out = {
        "value": w.m / total, "unit": "b_i/s", "cores": int(cores), "kind": "oracle",
        "sample": (f"LU of M (n={w.n}) {t_factor:.1f}s + {sample} problems in {t_sample:.1f}s, "
                   f"extrapolated to m={w.m}"),
        "host": host_info(),
    }
    # context: the paper's own algorithm (Alg. 5) on the same cores, one
    # block of SNPs timed after the factorization and the fixed part
    t0 = time.time()
    L = np.linalg.cholesky(M)
    host_alg5(M, XL, dg.make_XR(w, 0, 1), Y, w.p_R, L=L)  # the fixed part
    t_pre = time.time() - t0
    nb = min(w.block, 2048)
    XR = dg.make_XR(w, 0, nb)
    t0 = time.time()
    host_alg5(M, XL, XR, Y, w.p_R, block=nb, L=L)
    t_blk = time.time() - t0
    out["context_alg5"] = {
        "value": w.m / (t_pre + t_blk / nb * w.m), "unit": "b_i/s", "kind": "context",
        "sample": (f"paper's Alg. 5 (hp-gwas) with numpy/scipy BLAS on the host: Cholesky + fixed "
                   f"part {t_pre:.1f}s, one block of {nb} problems {t_blk:.1f}s, extrapolated to m={w.m}"),
    }
    return out


def host_info():
    """The machine's host CPU: model name and logical cores."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"cpu": model, "nproc": os.cpu_count()}


def stream_bench(args):
    """The streamed form (Sec. 4, Alg. 8) for the n = 20,000, p = 6, t = 8
    workload in blocks of 8192 problems: genotypes produced on the host (the
    C generator, or the library's file reader with --stream-source file)
    into pinned double buffers while the device solves; results handed to a
    Python sink in host memory, or written to a file by the library's
    asynchronous writer (--stream-sink file).  Reports the streamed rate,
    the device time inside the same run (overlap = device time / wall
    time), the paper's condition time(compute) against time(load) +
    time(store), and the in-core rate of the first problems (at most 2^19)
    with the genotypes resident, whose results must be the same bits."""
    import scipy.linalg as sla
    import torch
    from oracle import gls_oracle as orc
    from paper_1210_7325_amd import gls, stream
    w = dg.STREAM
    m = args.m or 64 * w.block
    block = args.block or w.block
    m_in = min(m, 1 << 19)  # the in-core comparison's problems
    forms = args.forms.split(",")
    torch.cuda.set_device(0)
    t0 = time.time()
    M = dg.make_M(w)
    XL, Y = dg.make_XL(w), dg.make_Y(w)
    log(f"M built (n={w.n}, q={w.q}) in {time.time() - t0:.1f}s")
    dM = torch.from_numpy(M).cuda()
    dXL = torch.from_numpy(np.asfortranarray(XL)).cuda()
    dY = torch.from_numpy(np.asfortranarray(Y)).cuda()
    import tempfile
    tmpdir = args.stream_file and os.path.dirname(args.stream_file) or tempfile.gettempdir()
    src = None
    if args.stream_source == "file":
        path = args.stream_file or os.path.join(tmpdir, f"gls_genotypes_n{w.n}_m{m}.bin")
        t0 = time.time()
        nbytes = stream.write_genotype_file(path, w, m)
        log(f"genotype file {path}: {nbytes / 1e9:.2f} GB written in {time.time() - t0:.1f}s")
        src = stream.FileSource(path, w.n, w.p_R, direct=bool(args.stream_direct), threads=8)
        fill, ctx = src.fill, src.ctx
    else:
        fill, ctx = stream.workload_fill(w)
    dXR = upload_genotypes(torch, w, m_in)
    res, outs = {}, {}
    for prec in forms:
        t0 = time.perf_counter()
        c = gls.Cohort(dM, precision=prec)
        c.set_slab_cols(args.slab_cols)
        c.whiten_fixed(dXL, dY, intercept_col=0)
        torch.cuda.synchronize()
        setup_ms = (time.perf_counter() - t0) * 1e3
        stream.solve_stream(c, 0, min(m, 2 * block), block, w.p_R, fill, ctx)  # warm-up
        c.set_kernel_timing(True)
        read0 = src.stats() if src else (0, 0.0)
        wst = None
        if args.stream_sink == "file":
            bpath = os.path.join(tmpdir, f"gls_b_{prec}_m{m}.bin")
            wr = stream.FileWriter(bpath, None, w.t, w.p, snp_base=0, depth=4)
            try:
                st = stream.solve_stream_to(c, 0, m, block, w.p_R, fill, ctx, wr.sink, wr.ctx)
            finally:
                wst = wr.close()
            B = np.memmap(bpath, dtype=np.float64, mode="r", shape=(m, w.t, w.p))
        else:
            B, info, st = stream.solve_stream(c, 0, m, block, w.p_R, fill, ctx)
        read1 = src.stats() if src else (0, 0.0)
        dev_ms = c.kernel_time(0)[0] + c.kernel_time(1)[0]
        c.set_kernel_timing(False)
        # in-core: the first m_in problems with the genotypes resident, 4 blocks per launch
        Bin = torch.empty((m_in, w.t, w.p), dtype=torch.float64, device="cuda")
        inf = torch.empty((m_in,), dtype=torch.int32, device="cuda")
        hs = [c] + [c.fork(torch.cuda.current_stream()) for _ in range(3)]
        for h in hs:
            h.reserve(block * w.p_R)

        def in_core():
            nblk = (m_in + block - 1) // block
            for g0 in range(0, nblk, 4):
                items = []
                for j, b in enumerate(range(g0, min(nblk, g0 + 4))):
                    a, e = b * block, min(m_in, (b + 1) * block)
                    items.append((hs[j], dXR[:, a * w.p_R:e * w.p_R], w.p_R, Bin[a:e], inf[a:e]))
                gls.solve_multi(items)
            torch.cuda.synchronize()
        in_core()
        t1 = time.perf_counter()
        in_core()
        in_core_s = time.perf_counter() - t1
        same = bool(np.array_equal(Bin.cpu().numpy(), np.asarray(B[:m_in])))
        for h in hs[1:]:
            h.free()
        c.free()
        del Bin
        wall_s = st["wall_ms"] * 1e-3
        nblocks = st["blocks"]
        store_ms = st["sink_ms"] + (wst["write_ms"] + wst["close_ms"] if wst else 0.0)
        res[prec] = {
            "value": round(m / wall_s, 1), "unit": "b_i/s", "wall_ms": round(st["wall_ms"], 1),
            "device_ms": round(dev_ms, 1), "overlap": round(dev_ms / st["wall_ms"], 4),
            "fill_ms": round(st["fill_ms"], 1), "sink_ms": round(st["sink_ms"], 1),
            "host_wait_ms": round(st["wait_ms"], 1),
            "h2d_gbps": round(st["bytes_h2d"] / wall_s / 1e9, 2),
            "in_core_value": round(m_in / in_core_s, 1), "in_core_problems": m_in,
            "streamed_vs_in_core": round((m_in / in_core_s) / (m / wall_s), 4),
            "bitwise_equal_to_in_core": same,
            "per_block_device_ms": round(dev_ms / nblocks, 2),
            "per_block_fill_ms": round(st["fill_ms"] / nblocks, 2),
            "per_block_store_ms": round(store_ms / nblocks, 2),
            # Sec. 4: the I/O hides behind the computation when
            # time(compute) > time(load) + time(store)
            "compute_over_io": round(dev_ms / max(st["fill_ms"] + store_ms, 1e-9), 3),
            "factor_and_whiten_ms": round(setup_ms, 1),
        }
        if wst:
            res[prec].update({"b_file_bytes": wst["bytes"], "write_ms": round(wst["write_ms"], 1),
                              "writer_wait_ms": round(wst["wait_ms"], 1),
                              "close_ms": round(wst["close_ms"], 1),
                              "write_gbps": round(wst["bytes"] / max(wst["write_ms"], 1e-9) / 1e6, 2)})
        if src:
            rb, rms = read1[0] - read0[0], read1[1] - read0[1]
            res[prec]["file_read_gbps"] = round(rb / max(rms, 1e-9) / 1e6, 2)
        outs[prec] = B
        log(f"[{prec}] streamed {m / wall_s:.0f} b_i/s (device {dev_ms:.0f} of {st['wall_ms']:.0f} ms, "
            f"fill {st['fill_ms']:.0f} ms, store {store_ms:.0f} ms), in-core {m_in / in_core_s:.0f} "
            f"b_i/s, bitwise equal {same}")
    del dXR
    if src:
        src.close()
        os.remove(path)
    parity = {}
    if args.parity_sample > 0:
        lu = sla.lu_factor(M)
        parity = parity_sample(w, m, M, XL, Y, lu, outs, min(args.parity_sample, 300))
    if args.stream_sink == "file":
        for prec in forms:
            fname = outs[prec].filename
            del outs[prec]
            os.remove(fname)
    head = res[forms[0]]
    out = {
        "metric": "GLS solves/sec with streamed genotypes (n=2e4, p=6, t=8 phenotypes)",
        "value": head["value"], "unit": "b_i/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": head["wall_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if forms[0] == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "p": w.p, "p_L": w.p_L, "p_R": w.p_R, "t": w.t,
                   "m": m, "block": block,
                   "source": ("file read by gls_file_fill (written before the run, "
                              + ("O_DIRECT" if args.stream_direct else "buffered") + ")")
                   if src else "host C generator into pinned double buffers",
                   "sink": ("file written by gls_writer_sink (asynchronous, depth 4, fdatasync at "
                            "close)") if args.stream_sink == "file" else "host memory (Python sink)",
                   "parallelism": "1 GPU"},
        "forms": {k: {**v, **parity.get(k, {})} for k, v in res.items()},
    }
    print(json.dumps(out), flush=True)


def ablation_bench(args):
    """The grouping ablation of the paper's Fig. 2 on the GPU (n = 10^4, p = 4):
    the same whitening and per-problem solves with the genotype columns
    grouped into launches of 64 .. 32,768 right-hand sides, with 64-column
    slabs (1 .. 512 of them for 256 compute units) and with the library's
    per-launch choice of slab width (16 .. 128 columns).  The paper groups many trsv into one
    trsm for BLAS-3 efficiency on a CPU; on the GPU the grouping is what
    fills the chip, and a launch of one slab leaves 255 compute units idle.
    Each setting times four launches after a warm-up; the rate is problems
    per second of wall time (factorization and fixed part excluded)."""
    import torch
    from paper_1210_7325_amd import gls
    w = dg.SCALE
    torch.cuda.set_device(0)
    M = dg.make_M(w)
    dM = torch.from_numpy(M).cuda()
    dXL = torch.from_numpy(np.asfortranarray(dg.make_XL(w))).cuda()
    dY = torch.from_numpy(np.asfortranarray(dg.make_Y(w))).cuda()
    c = gls.Cohort(dM).whiten_fixed(dXL, dY, intercept_col=0)
    rows = []
    mmax = 4 * 16384
    dXR = upload_genotypes(torch, w, mmax)
    B = torch.empty((mmax, w.t, w.p), dtype=torch.float64, device="cuda")
    info = torch.empty((mmax,), dtype=torch.int32, device="cuda")
    for slab, cols in [(sc, cl) for sc in (64, 0) for cl in (64, 256, 1024, 4096, 16384, 32768)]:
        c.set_slab_cols(slab)
        batch = max(1, cols // 4096)
        block = cols // batch
        hs = [c] + [c.fork(torch.cuda.current_stream()) for _ in range(batch - 1)]
        for h in hs:
            h.reserve(block)
        launches = max(2, min(mmax // cols, 4))

        def run():
            for L in range(launches):
                items = []
                for j in range(batch):
                    a = (L * batch + j) * block
                    items.append((hs[j], dXR[:, a:a + block], 1, B[a:a + block], info[a:a + block]))
                gls.solve_multi(items)
            torch.cuda.synchronize()
        run()
        t0 = time.perf_counter()
        run()
        dt = time.perf_counter() - t0
        rate = launches * cols / dt
        rows.append({"rhs_per_launch": cols, "slab_cols": slab or "auto",
                     "ms_per_launch": round(dt / launches * 1e3, 3), "value": round(rate, 1),
                     "tflops": round(float(w.n) ** 2 * rate / 1e12, 2)})
        log(f"[ablation] slabs {slab or 'auto'}: {cols:6d} RHS per launch: {rate:10.0f} b_i/s, "
            f"{dt / launches * 1e3:.2f} ms/launch")
        for h in hs[1:]:
            h.free()
    c.set_slab_cols(0)
    algs = algorithm_ablation(torch, gls, w, M, dM, dXL, dY, dXR, B, c)
    c.free()
    head = rows[-1]
    fixed = [r for r in rows if r["slab_cols"] == 64]
    out = {
        "metric": "GLS solves/sec vs right-hand sides grouped per launch (n=1e4, p=4)",
        "value": head["value"], "unit": "b_i/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": head["ms_per_launch"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "ablation_grouping_n10000_p4", "n": w.n, "p": w.p,
                   "parallelism": "1 GPU"},
        "grouping": rows,
        "grouping_gain_64_col_slabs": round(fixed[-1]["value"] / fixed[0]["value"], 1),
        "grouping_gain_auto_slabs": round(rows[-1]["value"] / rows[len(fixed)]["value"], 1),
        "algorithms": algs,
    }
    print(json.dumps(out), flush=True)


def algorithm_ablation(torch, gls, w, M, dM, dXL, dY, dXR, Bhp, c):
    """The paper's algorithms of Fig. 2 on the GPU, n = 10^4, p = 4, on the
    library's own triangular-solve kernels (FP64 right-hand sides through
    gls_whiten_block_f64 where the algorithm whitens whole X_i):

      Alg. 3 (black-box): per problem, factor M, whiten X_i (p columns) and
        y, then S_i = X_i^T X_i, b_i = X_i^T y, b_i = S_i^-1 b_i;
      Alg. 4 (seq-gls): factor M and whiten y once; per problem whiten X_i
        (p columns: few right-hand sides per launch), then as above;
      Alg. 4 grouped: the same, with the p columns of 8,192 problems whitened
        by one launch (32,768 right-hand sides, as a full launch of Alg. 5);
      Alg. 5 (hp-gwas): the library's solve (fixed part once, only the
        genotype column of each problem whitened), 32,768 problems per launch
        (the last row of the grouping sweep).

    The small products and p x p solves of Alg. 3 and Alg. 4 are batched
    torch FP64 operations (bmm, linalg.solve): they are not the part being
    compared.  Each variant's b_i are checked against Alg. 5's on the
    problems it solved."""
    p, n = w.p, w.n
    yt = c.whiten_block(dY)                                   # L^{-1} y (trsv)
    XR64 = dXR.double()

    def design(i0, g):
        """[X_L | x_i] for problems i0..i0+g-1, n x (p g) column-major FP64."""
        X = torch.empty((g, p, n), dtype=torch.float64, device="cuda")
        X[:, :w.p_L, :] = dXL.t().unsqueeze(0)
        X[:, w.p_L:, :] = XR64[:, i0:i0 + g].t().unsqueeze(1)
        return X.reshape(g * p, n).t()

    def finish(W, g, ytil):
        Wb = W.t().reshape(g, p, n)                            # W_i^T, (g, p, n)
        S = torch.bmm(Wb, Wb.transpose(1, 2).contiguous())     # X_i^T M^-1 X_i
        r = torch.matmul(Wb, ytil)                             # X_i^T M^-1 y
        return torch.linalg.solve(S, r)[:, :, 0]

    res = {}
    # Alg. 4, one problem per launch
    k4 = 32
    out4 = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(k4):
        out4.append(finish(c.whiten_block(design(i, 1)), 1, yt))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res["alg4_seq_gls_per_problem"] = {"problems": k4, "ms_per_problem": round(dt / k4 * 1e3, 3),
                                       "value": round(k4 / dt, 1)}
    # Alg. 4 grouped: 8,192 problems (32,768 FP64 columns) per launch
    g = 8192
    Wg = torch.empty((g * p, n), dtype=torch.float64, device="cuda").t()
    outg = finish(c.whiten_block(design(0, g), Wg), g, yt)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for rep in range(2):
        outg = finish(c.whiten_block(design(rep * g, g), Wg), g, yt)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res["alg4_seq_gls_grouped"] = {"problems_per_launch": g, "rhs_per_launch": g * p,
                                   "ms_per_launch": round(dt / 2 * 1e3, 3),
                                   "value": round(2 * g / dt, 1)}
    del Wg
    # Alg. 3, black-box: the factorization inside the loop
    k3 = 6
    out3 = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(k3):
        ci = gls.Cohort(dM)
        yti = ci.whiten_block(dY)
        out3.append(finish(ci.whiten_block(design(i, 1)), 1, yti))
        ci.free()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res["alg3_black_box"] = {"problems": k3, "ms_per_problem": round(dt / k3 * 1e3, 3),
                             "value": round(k3 / dt, 1)}
    # Alg. 5 at the same grouping (32,768 right-hand sides per launch)
    hb = Bhp[:, 0, :].double()
    ref = hb[:g]                      # Alg. 5's b of the first problems (from the grouping sweep)
    errs = {
        "alg4_seq_gls_per_problem": float(((torch.cat(out4) - ref[:k4]).abs().amax(1)
                                           / ref[:k4].abs().amax(1)).max()),
        "alg4_seq_gls_grouped": float(((outg - hb[g:2 * g]).abs().amax(1)
                                       / hb[g:2 * g].abs().amax(1)).max()),
        "alg3_black_box": float(((torch.cat(out3) - ref[:k3]).abs().amax(1)
                                 / ref[:k3].abs().amax(1)).max()),
    }
    for k, e in errs.items():
        res[k]["max_rel_err_vs_alg5"] = e
    for k, v in res.items():
        log(f"[ablation] {k}: {v['value']:.1f} b_i/s ({v}), max rel err vs Alg. 5 {errs[k]:.2e}")
    return res


def phenotypes_bench(args):
    """Phenotypes with distinct covariance matrices (the phenotype index of
    Eq. (1) with its own M_j): t = 4 phenotypes, M_j = h_j Phi + (1 - h_j) I
    + 1e-3 I (h_j = 0.2, 0.4, 0.6, 0.8), n = 10^4, p = 4, m = 131,072 SNPs
    shared by all phenotypes.  One handle per M_j (factor and fixed part
    resident); each launch solves `batch` blocks of 4096 SNPs for every
    phenotype (gls_solve_multi items sharing the X_R block).  One step =
    the t factorizations, fixed parts and all t*m problems.  Rate: b_ij/s."""
    import scipy.linalg as sla
    import torch
    from oracle import gls_oracle as orc
    from paper_1210_7325_amd import gls
    w = dg.PHENO
    hs = dg.PHENO_H
    m = args.m or w.m
    block = args.block or w.block
    torch.cuda.set_device(0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    t0 = time.time()
    phi = dg.make_phi(w)
    Ms = [dg.make_M(w, phi, h=h) for h in hs]
    XL, Y = dg.make_XL(w), dg.make_Y(w)
    log(f"M_1..M_{len(hs)} built (n={w.n}, q={w.q}) in {time.time() - t0:.1f}s")
    dMs = [torch.from_numpy(M).cuda() for M in Ms]
    dXL = torch.from_numpy(np.asfortranarray(XL)).cuda()
    dYs = [torch.from_numpy(np.asfortranarray(Y[:, j:j + 1])).cuda() for j in range(len(hs))]
    dXR = upload_genotypes(torch, w, m)
    # blocks per launch: one 128-column slab per CU over all phenotypes
    batch = args.batch or max(1, min(gls_max_items() // len(hs), cus * 128 // (block * w.p_R * len(hs))))
    res, outs = {}, {}
    for prec in args.forms.split(","):
        Bs = [torch.empty((m, 1, w.p), dtype=torch.float64, device="cuda") for _ in hs]
        infos = [torch.empty((m,), dtype=torch.int32, device="cuda") for _ in hs]

        def step(timing=False):
            cs = [gls.Cohort(dM, precision=prec).whiten_fixed(dXL, dY, intercept_col=0)
                  for dM, dY in zip(dMs, dYs)]
            hs_all = [[c] + [c.fork(torch.cuda.current_stream()) for _ in range(batch - 1)]
                      for c in cs]
            for hh in hs_all:
                for h in hh:
                    h.reserve(block * w.p_R)
            if timing:
                hs_all[0][0].set_kernel_timing(True)
            nblk = (m + block - 1) // block
            for g0 in range(0, nblk, batch):
                items = []
                for j in range(len(hs)):
                    for k, b in enumerate(range(g0, min(nblk, g0 + batch))):
                        a, e = b * block, min(m, (b + 1) * block)
                        items.append((hs_all[j][k], dXR[:, a * w.p_R:e * w.p_R], w.p_R, Bs[j][a:e],
                                      infos[j][a:e]))
                gls.solve_multi(items)
            kt = hs_all[0][0].kernel_time(0) if timing else None
            torch.cuda.synchronize()
            for hh in hs_all:
                for h in hh[1:]:
                    h.free()
            for c in cs:
                c.free()
            return kt
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kts = [step(timing=True) for _ in range(args.steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        trsm_ms = sum(k[0] for k in kts)
        trsm_n = sum(k[1] for k in kts)
        flops = float(w.n) ** 2 * m * w.p_R * len(hs) * args.steps
        peak = PEAK_FP64_TFLOPS if prec == "fp64" else PEAK_FP32_TFLOPS
        res[prec] = {"value": round(len(hs) * m * args.steps / dt, 1), "unit": "b_ij/s",
                     "ms_per_step": round(dt / args.steps * 1e3, 2),
                     "trsm_tflops": round(flops / (trsm_ms * 1e-3) / 1e12, 3), "trsm_peak": peak,
                     "trsm_launches": trsm_n, "blocks_per_launch_per_phenotype": batch,
                     "rank_deficient": int(sum(int((inf != 0).sum()) for inf in infos))}
        outs[prec] = [B.cpu().numpy() for B in Bs]
        log(f"[{prec}] {res[prec]['value']:.0f} b_ij/s, {res[prec]['ms_per_step']:.1f} ms/step, "
            f"TRSM {res[prec]['trsm_tflops']:.1f} TFLOP/s")
    del dXR
    if args.parity_sample > 0:
        rng = np.random.default_rng(12107325)
        idx = np.unique(np.concatenate([[0, m - 1], rng.choice(m, min(args.parity_sample, m) - 2,
                                                              replace=False)]))
        XRs = np.concatenate([dg.make_XR(w, int(i), 1) for i in idx], axis=1)
        for j, M in enumerate(Ms):
            ref = orc.gls_sequence(M, XL, XRs, Y[:, j:j + 1], w.p_R, lu=sla.lu_factor(M))
            for prec in outs:
                err = orc.relative_error(outs[prec][j][idx], ref)
                key = "max_rel_err_by_phenotype"
                res[prec].setdefault(key, []).append(float(err.max()))
                log(f"[{prec}] phenotype {j} (h = {hs[j]}): max rel err {err.max():.3e} "
                    f"on {len(idx)} problems")
        for prec in outs:
            res[prec]["parity_sample"] = int(len(idx))
    forms = args.forms.split(",")
    head = res[forms[0]]
    out = {
        "metric": "GLS solves/sec for t phenotypes with distinct M_j (n=1e4, p=4)",
        "value": head["value"], "unit": "b_ij/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if forms[0] == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "p": w.p, "p_L": w.p_L, "p_R": w.p_R,
                   "phenotypes": len(hs), "h": list(hs), "m": m, "block": block,
                   "M_j": f"h_j*ZZ^T/q+(1-h_j)I+1e-3I, q={w.q}", "parallelism": "1 GPU"},
        "forms": res,
    }
    print(json.dumps(out), flush=True)


def gls_max_items():
    """Work items the library puts in one launch of gls_solve_multi (more are
    split over several launches)."""
    return 16


def serve_bench(args):
    """The serving mix: Poisson arrivals of GWAS jobs (n in {1500, 4000,
    10000, 20000}, p uniform in 4..20, m log-uniform in [1e5, m_max], each
    with its own M = h Phi + (1-h) I + 1e-3 I, h ~ U[0.2, 0.8]) through the
    continuous-batching scheduler, once per precision on the same mix."""
    import torch
    from paper_1210_7325_amd import serve
    torch.cuda.set_device(0)
    proto = serve.make_jobs(args.serve_jobs, rate=1.0, m_range=(1e5, args.serve_m_max))
    work = sum(float(j.n) ** 2 * j.m for j in proto)
    # arrival rate for the requested offered load at 50 TFLOP/s of whitening
    rate = args.serve_load * 50e12 / (work / len(proto))
    t0 = time.time()
    phi = {}
    for n in sorted({j.n for j in proto}):
        phi[n] = torch.from_numpy(dg.make_phi(dg.SERVE_BASE.replace(n=n, q=2 * n))).cuda()
    log(f"Phi for n in {sorted(phi)} built in {time.time() - t0:.1f}s; rate {rate:.3f} jobs/s, "
        f"{work / 1e15:.2f} PFLOP of whitening")
    res = {}
    for prec in args.forms.split(","):
        jobs = serve.make_jobs(args.serve_jobs, rate=rate, m_range=(1e5, args.serve_m_max))
        ex = serve.GpuExecutor(precision=prec, phi=phi, ingest=args.serve_ingest,
                               streams=args.serve_streams, slots=args.serve_inflight + 1)
        stats = serve.Scheduler(ex, budget_bytes=(200 << 30) - ex.staging_bytes(),
                                inflight=args.serve_inflight, target_cols=args.serve_target_cols,
                                log=lambda msg, prec=prec: log(f"[{prec}] {msg}")).run(jobs)
        stats["timeline"] = ex.timeline_summary()
        log(f"[{prec}] timeline: {stats['timeline']}")
        stats["jobs_detail"] = [(j.id, j.n, j.p, j.m, round(j.arrival, 3), round(j.finished - j.arrival, 3)
                                 if j.finished is not None else None, j.state, j.error) for j in jobs]
        res[prec] = stats
        log(f"[{prec}] {stats['solves_per_s']:.0f} b_i/s, {stats['whitening_tflops']:.1f} TFLOP/s, "
            f"latency p50 {stats['latency_p50_s']:.2f}s p99 {stats['latency_p99_s']:.2f}s, "
            f"{stats['items_per_round']:.1f} items/round, done {stats['done']}/{stats['jobs']}")
    head = res[args.forms.split(",")[0]]
    out = {
        "metric": "GWAS serving mix: solves/s with p50/p99 job latency",
        "value": round(head["solves_per_s"], 1), "unit": "b_i/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": round(head["makespan_s"] * 1e3, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "serving_mix", "jobs": args.serve_jobs, "arrival_rate": rate,
                   "offered_load_at_50TF": args.serve_load, "n": [1500, 4000, 10000, 20000],
                   "p": [4, 20], "m": [1e5, args.serve_m_max], "h": [0.2, 0.8],
                   "hbm_budget_bytes": 200 << 30, "ingest": args.serve_ingest,
                   "compute_streams": args.serve_streams, "rounds_inflight": args.serve_inflight,
                   "round_target_cols": args.serve_target_cols, "parallelism": "1 GPU"},
        "forms": res,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "stream" and args.gpus == 1:
        stream_bench(args)
        return
    if args.workload == "serve" and args.gpus == 1:
        serve_bench(args)
        return
    if args.workload == "ablation" and args.gpus == 1:
        ablation_bench(args)
        return
    if args.workload == "phenotypes" and args.gpus == 1:
        phenotypes_bench(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        log("bench.py: only --gpus 1 is supported (one GPU per box)")
        sys.exit(2)
    import scipy.linalg as sla
    import torch
    from paper_1210_7325_amd import gls

    gls.lib()
    w = WORKLOADS[args.workload]
    m = args.m or w.m
    block = args.block or w.block
    forms = args.forms.split(",")
    torch.cuda.set_device(0)
    cus = torch.cuda.get_device_properties(0).multi_processor_count

    def batch_for(prec):
        # blocks per launch: one slab of the widest width per CU
        if args.batch:
            return args.batch
        widest = args.slab_cols or 128
        return max(1, cus * widest // (block * w.p_R))
    batch = batch_for(forms[0])

    t0 = time.time()
    M = dg.make_M(w)
    XL, Y = dg.make_XL(w), dg.make_Y(w)
    log(f"M built (n={w.n}, q={w.q}) in {time.time() - t0:.1f}s")
    dM = torch.from_numpy(M).cuda()
    dXL = torch.from_numpy(np.asfortranarray(XL)).cuda()
    dY = torch.from_numpy(np.asfortranarray(Y)).cuda()
    dXR = upload_genotypes(torch, w, m)
    info = torch.empty((m,), dtype=torch.int32, device="cuda")

    results, outs = {}, {}
    for prec in forms:
        Bout = torch.empty((m, w.t, w.p), dtype=torch.float64, device="cuda")
        results[prec] = time_form(gls, torch, args, w, m, block, batch_for(prec), dM, dXL, dY, dXR,
                                  Bout, info, prec)
        outs[prec] = Bout.cpu().numpy()
        del Bout
    del dXR

    lu, t_factor = None, None
    parity = {}
    if args.parity_sample > 0 or args.cpu_seconds > 0:
        t0 = time.time()
        lu = sla.lu_factor(M)
        t_factor = time.time() - t0
    if args.parity_sample > 0:
        parity = parity_sample(w, m, M, XL, Y, lu, outs, args.parity_sample)
    cpu = None
    if args.cpu_seconds > 0:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(w, M, XL, Y, args.cpu_seconds, lu=lu, t_factor=t_factor)
        log(f"cpu: {cpu['value']:.1f} b_i/s ({cpu['sample']}); context Alg. 5: "
            f"{cpu['context_alg5']['value']:.1f} b_i/s ({cpu['context_alg5']['sample']})")

    head = results[forms[0]]
    roofline = {
        "bound": "mfma", "achieved": round(head["trsm_tflops"], 3), "peak": head["peak"],
        "unit": "TFLOP/s", "frac": round(head["trsm_tflops"] / head["peak"], 4),
        "traffic": measured_traffic(batch, args.slab_cols, forms[0]),
        "kernel": ("k_trsm_pair (blocked lower solve, row blocks in pairs, FP64 MFMA)" if forms[0] == "fp64"
                   else "k_trsm_mixed (blocked lower solve, FP32 MFMA products + FP64 diagonal)"),
        # the full launches (32,768 right-hand sides in 128-column slabs at
        # the default sizes), each bracketing the main kernel and its
        # last-block kernel; the tail rounds and the rate over every launch
        # of the step follow
        "launches": head["trsm_launches"], "avg_launch_ms": round(head["trsm_avg_ms"], 4),
        "cols_per_launch": head["full_cols"], "slab_cols": head["full_slab"],
        "flops_per_launch": head["flops_per_launch"], "blocks_per_launch": batch,
        "tail_launches_per_step": head["tail_launches"],
        "all_launches_tflops": round(head["all_tflops"], 3),
        "all_launches_avg_ms": round(head["all_avg_ms"], 4),
        "step_tflops": round(head["step_tflops"], 3),
        "step_frac": round(head["step_tflops"] / head["peak"], 4),
        "assemble_avg_launch_ms": round(head["assemble_avg_ms"], 4),
        # the diagonal steps W_k = inv(L_kk) R_k: about NB / n of the MFMA work
        "diag_flop_share": round(128.0 / w.n, 4),
        # the assembly's stream of whitened genotypes: 8 n_pad bytes per column
        "assemble_gbps": round(8.0 * (-(-w.n // 128) * 128) * m * w.p_R / head["all_launches"]
                               * args.steps / (head["assemble_avg_ms"] * 1e-3) / 1e9, 1),
    }
    phases = {
        "factor_ms": round(head["factor_ms"], 2), "fixed_ms": round(head["fixed_ms"], 2),
        "solve_ms": round(head["solve_ms"], 2),
        "solve_only_value": round(m / (head["solve_ms"] * 1e-3), 1),
        # int8 genotypes consumed per second of the step (tiny: the path is MFMA-bound)
        "genotype_gbps": round(float(w.n) * m * w.p_R / (head["ms_per_step"] * 1e-3) / 1e9, 2),
    }
    form_out = {}
    for prec in forms[1:]:
        r = results[prec]
        # every problem of the step against the headline form's b (the FP64
        # path, itself within ~3e-14 of the oracle on the sample above)
        ref = outs[forms[0]]
        num = np.max(np.abs(outs[prec] - ref), axis=-1)
        err_all = num / np.max(np.abs(ref), axis=-1)
        full = {"full_m_max_rel_err": float(err_all.max()),
                "full_m_p9999_rel_err": float(np.quantile(err_all, 0.9999)),
                "full_m_problems": int(err_all.shape[0]),
                "full_m_reference": f"the {forms[0]} GPU path on all problems"}
        log(f"[{prec}] all {err_all.shape[0]} problems against {forms[0]}: max rel err "
            f"{err_all.max():.3e}, p99.99 {full['full_m_p9999_rel_err']:.3e}")
        form_out[prec] = {
            "value": round(r["value"], 1), "unit": "b_i/s", "ms_per_step": round(r["ms_per_step"], 2),
            "speedup_vs_" + forms[0]: round(r["value"] / head["value"], 3),
            "trsm_tflops": round(r["trsm_tflops"], 3), "trsm_peak": r["peak"],
            "trsm_frac": round(r["trsm_tflops"] / r["peak"], 4),
            "trsm_avg_launch_ms": round(r["trsm_avg_ms"], 4), "blocks_per_launch": batch_for(prec),
            **parity.get(prec, {}), **full,
        }
    out = {
        "metric": METRIC, "value": round(head["value"], 1), "unit": "b_i/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms_per_step"], 2),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": round(head["value"] / PAPER_BI_PER_S, 2) if w is dg.SCALE else None,
        "dtype": "f64" if forms[0] == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "p": w.p, "p_L": w.p_L, "p_R": w.p_R, "t": w.t,
                   "m": m, "block": block, "blocks_per_launch": batch, "streams": args.streams,
                   "slab_cols": args.slab_cols or "auto",
                   "M": f"h*ZZ^T/q+(1-h)I+1e-3I, q={w.q}, h={w.h}", "parallelism": "1 GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "phases": phases,
        "parity": parity.get(forms[0]), "forms": form_out,
        "baseline_note": "vs_baseline divides by the paper's 12-core CPU rate for the same "
                         "workload (816 s for m=10^6, Table 3): context, other hardware",
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
