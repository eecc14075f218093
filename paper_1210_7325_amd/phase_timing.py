"""Where the paired-block FP64 solve spends its cycles (a measurement, not
part of the library).

Runs one launch of k_trsm_pair (128-column slabs, 256 work-groups, one per
compute unit) through libgls_phase.so, the library built with phase
timestamps (csrc/trsm_phase_timing.hip; same kernels, same results), and
prints, from the stamps of thread 0 of every work-group:

* the shader clock over the walk (shader-clock cycles / constant-clock time),
* the off-diagonal GEMM's MFMA rate as a fraction of what the clock allows
  (128 FP64 flops per cycle and compute unit: four SIMDs, one
  16x16x4 MFMA of 2,048 flops per 64 cycles each), per range of pairs,
* the share of the walk's cycles in the phases that are not the GEMM
  (right-hand sides, the diagonal steps, the L_{k+1,k} W_k update, stores,
  barriers and the terms of a split last block's sum).

    python -m paper_1210_7325_amd.phase_timing [--n 10000] [--cols 32768]
"""
from __future__ import annotations

import argparse
import ctypes
import os
import sys

import numpy as np

POINTS = ("loop top", "GEMM done", "W_k done", "update done", "W_k+1 done", "barrier")


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=10_000)
    ap.add_argument("--cols", type=int, default=32_768, help="right-hand sides (one launch: <= 128 x CUs)")
    ap.add_argument("--runs", type=int, default=3, help="launches; the last one's stamps are read")
    ap.add_argument("--lib", default=None, help="another build of libgls_phase.so (for comparisons)")
    args = ap.parse_args()

    import torch
    from paper_1210_7325_amd import datagen as dg
    from paper_1210_7325_amd import gls
    path = args.lib or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgls_phase.so")
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run python -m paper_1210_7325_amd.build")
    gls.LIB_PATH = path
    L = gls.lib()
    L.gls_phase_times.restype = ctypes.c_int
    L.gls_phase_times.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]

    w = dg.SCALE.replace(n=args.n)
    M = torch.from_numpy(dg.make_M(w)).cuda()
    X = torch.from_numpy(np.asfortranarray(dg.make_XR(w, 0, args.cols))).cuda()
    c = gls.Cohort(M)
    c.whiten_fixed(torch.from_numpy(np.asfortranarray(dg.make_XL(w))).cuda(),
                   torch.from_numpy(np.asfortranarray(dg.make_Y(w))).cuda(), intercept_col=0)
    c.set_slab_cols(128)
    c.set_kernel_timing(True)
    for _ in range(args.runs):
        B, info = c.solve_block(X, p_R=1)
    torch.cuda.synchronize()
    launches = c.kernel_launches(0)
    assert int((info != 0).sum()) == 0

    dims = (ctypes.c_int * 3)()
    size = 256 * 64 * 6
    rt = np.zeros(size, dtype=np.uint64)
    cyc = np.zeros(size, dtype=np.uint64)
    if L.gls_phase_times(rt.ctypes.data, cyc.ctypes.data, dims) != 0:
        raise RuntimeError("gls_phase_times failed")
    wgs, pairs_max, npt = dims[0], dims[1], dims[2]
    K = -(-args.n // 128)
    nslab = -(-args.cols // 128)
    last_split = (args.n - (K - 1) * 128) <= 32     # the last block goes to k_trsm_last
    kmain = K - 1 if last_split else K
    npair = (kmain + 1) // 2
    full = kmain % 2 == 0                             # every pair has two blocks
    nw = min(wgs, nslab)
    T = rt.reshape(wgs, pairs_max, npt)[:nw, :npair].astype(np.int64)
    C = cyc.reshape(wgs, pairs_max, npt)[:nw, :npair].astype(np.int64)
    walk_s = (T[:, -1, 5] - T[:, 0, 0]) / 1e8
    walk_cyc = C[:, -1, 5] - C[:, 0, 0]
    clock = walk_cyc / walk_s
    ph = np.diff(C, axis=2)                          # 5 phases per pair (cycles)
    k = 2 * np.arange(npair)
    gemm_ideal = 2 * 128 * (128 * k) * 128 * 2.0 / 128  # cycles at 128 flop / cycle / CU
    gemm_cyc = ph[:, :, 0].mean(0)

    def frac(sl):
        return gemm_ideal[sl].sum() / gemm_cyc[sl].sum()

    print(f"# Phase cycles of k_trsm_pair (n = {args.n}, {args.cols} right-hand sides, {nslab} work-groups; "
          f"the last of {args.runs} launches)\n")
    print("Command (`$REPO` = repository root): `python -m paper_1210_7325_amd.phase_timing "
          f"--n {args.n} --cols {args.cols} --runs {args.runs}` (run from `$REPO`; needs "
          "`libgls_phase.so` from `python -m paper_1210_7325_amd.build`)\n")
    print(f"Launch durations (HIP events, ms): {', '.join(f'{l[0]:.2f}' for l in launches)}\n")
    print("| quantity | value |\n|---|---|")
    print(f"| walk of a work-group (ms, mean / min / max) | {walk_s.mean()*1e3:.2f} / {walk_s.min()*1e3:.2f} / "
          f"{walk_s.max()*1e3:.2f} |")
    print(f"| shader clock over the walk (GHz, mean) | {clock.mean()/1e9:.3f} |")
    print(f"| GEMM: MFMA rate / clock-limited peak, all pairs | {frac(slice(1, npair)):.4f} |")
    for a, b in ((1, npair // 4), (npair // 4, npair // 2), (npair // 2, npair)):
        print(f"| GEMM: the same, pairs {a}-{b - 1} | {frac(slice(a, b)):.4f} |")
    tot = walk_cyc.mean()
    for i, name in enumerate(("GEMM", "right-hand side k, W_k and its store", "right-hand side k+1 and "
                              "L_{k+1,k} W_k", "W_{k+1} and its store",
                              "closing barrier and the last block's sum")):
        print(f"| cycles in {name} (share of the walk) | {ph[:, :, i].sum(1).mean()/tot:.4f} |")
    other = ph[:, :, 1:].sum(2).mean(0)
    # the non-GEMM phases' MFMA work: two diagonal steps (18 k-step pairs of
    # 8 MFMAs per wave, 8 waves), the update (16 k-step pairs x 16 MFMAs per
    # wave) and, with a split last block, its sum (two blocks of 16 k-step
    # pairs x 2 MFMAs per 16-row tile and wave)
    last_tiles = (1 if args.n - (K - 1) * 128 <= 16 else 2) if last_split else 0
    nong_ideal = (2 * 18 * 8 * 8 + 16 * 16 * 8 + 2 * 16 * 2 * last_tiles * 8) * 2048 / 128.0
    print(f"| non-GEMM phases per pair (cycles, mean) / their MFMA work at the clock-limited rate | "
          f"{other.mean():.0f} / {nong_ideal:.0f} |")
    flops = float(args.n) ** 2 * min(args.cols, nslab * 128)
    print(f"| whole walk: algorithmic flops / (128 x walk cycles) | {flops / nslab / (128 * tot):.4f} |")
    if not full:
        print("\n(The last pair holds one block.)")


if __name__ == "__main__":
    sys.exit(main())
