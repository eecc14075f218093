// Per-problem assembly and p x p solve (a3/a4) and the centering pre-pass of the FP32_REFINE form.
#include "gls_device.h"

namespace gls {

// ---------------------------------------------------------------------------
// a3/a4: per-problem assembly and solve (Alg. 5 loop body: S_BL_i, S_BR_i,
// b_B_i by gemv/dot, then posv of the p x p system; Fig. 1 partition).
//
// One work-group per group of problems laid out in 4 tiles of 16 columns,
// PT = floor(16 / p_R) problems per tile (a problem never straddles two
// tiles).  The per-column dot products are small products on FP64 MFMA:
// per tile and 4-row k-step, A = W^T (16 columns x 4 rows) is exactly what a
// lane holds in the slab layout (lane l: W[4s + l/16][16ct + l%16]), and
//   D_F  += A  F[4s .. 4s+3][16 et .. 16 et + 15]       (W^T [W_L | ytil])
//   D_G  += A  W[4s .. 4s+3][tile]                       (W^T W of the tile)
// where the Gram's B operand is the same register as A.  Wave w takes the
// row octets w, w + 8, ... (one 16-byte pair per tile per octet, i.e. two
// k-steps; as_depth<ET>() octets in flight).  The per-wave products are reduced
// in LDS in a fixed order; then each problem is solved by one wavefront:
// Cholesky, forward and backward substitution with lane j holding column j
// of S_i and row j of c_i, and wave-wide broadcasts (v_readlane) between
// the steps.  Every sum runs over the rows in an order fixed by the row
// index alone, so a column's result does not depend on which group, launch
// or slab width it is solved in.
constexpr int AS_WAVES = 8;
constexpr int AS_COLS = AS_GROUP_COLS;     // columns per work-group (4 tiles of 16)
// row octets in flight per wave (fewer with two F tiles: registers)
template <int ET> constexpr int as_depth() { return 2; }
// columns reduced per pass (two passes: the reduction buffer is half the
// group, so that two work-groups fit one compute unit)
constexpr int AS_RED_COLS = AS_COLS / 2;
constexpr int AS_DOTS = 2 * 16 + 16;       // per column: up to 32 F dots + 16 Gram entries

// Cholesky of a p x p SPD matrix held by one wavefront, lane j holding
// column j (col[a] = S[a][j]).  On return lane j holds column j of the
// lower factor G (rows >= j).  fail = order of the first leading minor
// that is not positive (0 if none).
__device__ __forceinline__ void wave_cholesky(double (&col)[MAXP], int p, int lane, int& fail) {
  fail = 0;
  for (int k = 0; k < p; k++) {
    double d = 0.0;
#pragma unroll
    for (int a = 0; a < MAXP; a++)
      if (a == k) d = bcast_lane(col[a], k);
    if (!(d > 0.0) || !(d < INFINITY)) { fail = k + 1; return; }
    const double gdiag = sqrt(d);
    if (lane == k) {
#pragma unroll
      for (int a = 0; a < MAXP; a++) {
        if (a > k) col[a] = col[a] / gdiag;
        else if (a == k) col[a] = gdiag;
      }
    }
    double gk[MAXP];
    double gmine = 0.0;
#pragma unroll
    for (int a = 0; a < MAXP; a++) {
      gk[a] = (a > k && a < p) ? bcast_lane(col[a], k) : 0.0;
      if (a == lane) gmine = gk[a];
    }
    if (lane > k && lane < p) {
#pragma unroll
      for (int a = 0; a < MAXP; a++)
        if (a >= lane) col[a] -= gk[a] * gmine;
    }
  }
}

// Solve G G^T x = r in place (r: lane j holds row j, t columns), G from
// wave_cholesky: forward substitution G z = r, then backward G^T x = z.
__device__ __forceinline__ void wave_cholsolve(const double (&col)[MAXP], double (&r)[MAXT], int p,
                                               int t, int lane) {
  for (int k = 0; k < p; k++) {
    double gkk = 0.0, gmine = 0.0;
#pragma unroll
    for (int a = 0; a < MAXP; a++) {
      if (a == k) gkk = bcast_lane(col[a], k);
      const double g = (a > k && a < p) ? bcast_lane(col[a], k) : 0.0;
      if (a == lane) gmine = g;
    }
#pragma unroll
    for (int j = 0; j < MAXT; j++) {
      if (j < t) {
        const double zk = bcast_lane(r[j], k) / gkk;
        if (lane == k) r[j] = zk;
        else if (lane > k && lane < p) r[j] -= gmine * zk;
      }
    }
  }
  for (int k = p - 1; k >= 0; k--) {
    double gkk = 0.0, gki = 0.0;
#pragma unroll
    for (int a = 0; a < MAXP; a++)
      if (a == k) { gkk = bcast_lane(col[a], k); gki = col[a]; }
#pragma unroll
    for (int j = 0; j < MAXT; j++) {
      if (j < t) {
        const double bk = bcast_lane(r[j], k) / gkk;
        if (lane == k) r[j] = bk;
        else if (lane < k) r[j] -= gki * bk;
      }
    }
  }
}

// Products of the 64 columns of a group with the rows of F (ET tiles of 16
// columns of F, zero past ldf) and, if GRAM, the Gram matrix of each column
// tile, accumulated per wave on FP64 MFMA.  loadA(ct, o) gives the lane's
// A-operand pair of tile ct for row octet o: rows 8o + l/16 (.x) and
// 8o + 4 + l/16 (.y) of column l%16.  F: row-major, ld = ldf, at least
// 8 noct rows.  acc[ct][et] (et < ET) and acc[ct][ET] (Gram) use the MFMA
// output layout: lane l, element i = row l/16 + 4i (a column of the tile),
// column l%16.
template <int ET, bool GRAM, class LoadA>
__device__ __forceinline__ void mfma_dots(LoadA loadA, const double* __restrict__ F, int ldf,
                                          int64_t noct, int wave, int lane,
                                          d4 (&acc)[4][ET + 1]) {
  const int r = lane / 16, cl = lane % 16;
#pragma unroll
  for (int ct = 0; ct < 4; ct++)
#pragma unroll
    for (int et = 0; et <= ET; et++) acc[ct][et] = d4{0.0, 0.0, 0.0, 0.0};
  constexpr int DEPTH = as_depth<ET>();
  d2 av[DEPTH][4];
  double f0[DEPTH][ET], f1[DEPTH][ET];
  auto fetch = [&](int64_t o, d2 (&a)[4], double (&g0)[ET], double (&g1)[ET])
      __attribute__((always_inline)) {
#pragma unroll
    for (int ct = 0; ct < 4; ct++) a[ct] = loadA(ct, o);
    const double* __restrict__ p0 = F + (8 * o + r) * ldf;
    const double* __restrict__ p1 = p0 + 4 * ldf;
#pragma unroll
    for (int et = 0; et < ET; et++) {
      const int e = 16 * et + cl;
      g0[et] = e < ldf ? p0[e] : 0.0;
      g1[et] = e < ldf ? p1[e] : 0.0;
    }
  };
  // every fetch is issued on every path (octets past the end clamped to the
  // last one and never used), so that the waits the compiler places for a
  // stage's operands do not also cover the fetches of the stages after it
  auto clamp = [&](int64_t o) { return o < noct ? o : noct - 1; };
#pragma unroll
  for (int st = 0; st < DEPTH; st++) fetch(clamp(wave + 8 * st), av[st], f0[st], f1[st]);
  for (int64_t o0 = wave; o0 < noct; o0 += 8 * DEPTH) {
#pragma unroll
    for (int st = 0; st < DEPTH; st++) {
      const int64_t o = o0 + 8 * st;
      if (o < noct) {
#pragma unroll
        for (int ct = 0; ct < 4; ct++) {
#pragma unroll
          for (int et = 0; et < ET; et++) {
            acc[ct][et] = MFMA64(av[st][ct].x, f0[st][et], acc[ct][et]);
            acc[ct][et] = MFMA64(av[st][ct].y, f1[st][et], acc[ct][et]);
          }
          if (GRAM) {
            acc[ct][ET] = MFMA64(av[st][ct].x, av[st][ct].x, acc[ct][ET]);
            acc[ct][ET] = MFMA64(av[st][ct].y, av[st][ct].y, acc[ct][ET]);
          }
        }
      }
      fetch(clamp(o + 8 * DEPTH), av[st], f0[st], f1[st]);
    }
  }
}

// The same products for p_R = 1 and ldf <= VD_LDF on FP64 FMAs, straight
// into dots: lane (r, cl) of tile ct keeps its column's sums over its rows
// (rows 8o + r and 8o + 4 + r of the wave's octets o) with the ldf columns
// of F and with itself (the 1 x 1 Gram), then the four lanes of a column
// add theirs (lanes r = 0..3, pairs first) and the waves theirs, in wave
// order.  An MFMA here would compute a 16 x 16 tile of which 4 columns (and,
// for the Gram, the diagonal) are used: on the FMAs the products take a
// sixth of the cycles, and the kernel is left to the memory stream.  Every
// sum runs over the rows in an order fixed by the row index alone.
constexpr int VD_LDF = 4;

template <class LoadA>
__device__ __forceinline__ void valu_dots(LoadA loadA, const double* __restrict__ F, int ldf, int64_t noct,
                                          int wave, int lane, double* __restrict__ red,
                                          double (*dots)[AS_DOTS]) {
  constexpr int E = VD_LDF + 1;  // F columns, then the squared norm
  const int r = lane / 16, cl = lane % 16;
  double part[4][E];
#pragma unroll
  for (int ct = 0; ct < 4; ct++)
#pragma unroll
    for (int e = 0; e < E; e++) part[ct][e] = 0.0;
  constexpr int DEPTH = 2;
  d2 av[DEPTH][4];
  double f0[DEPTH][VD_LDF], f1[DEPTH][VD_LDF];
  // (F's columns past ldf are read at column ldf - 1: those sums are never used)
  auto fetch = [&](int64_t o, d2 (&a)[4], double (&g0)[VD_LDF], double (&g1)[VD_LDF])
      __attribute__((always_inline)) {
#pragma unroll
    for (int ct = 0; ct < 4; ct++) a[ct] = loadA(ct, o);
    const double* __restrict__ p0 = F + (8 * o + r) * ldf;
    const double* __restrict__ p1 = p0 + 4 * ldf;
#pragma unroll
    for (int e = 0; e < VD_LDF; e++) {
      g0[e] = p0[e < ldf ? e : ldf - 1];
      g1[e] = p1[e < ldf ? e : ldf - 1];
    }
  };
  auto clamp = [&](int64_t o) { return o < noct ? o : noct - 1; };
  auto products = [&](int st) __attribute__((always_inline)) {
#pragma unroll
    for (int ct = 0; ct < 4; ct++) {
#pragma unroll
      for (int e = 0; e < VD_LDF; e++) {
        part[ct][e] = fma(av[st][ct].x, f0[st][e], part[ct][e]);
        part[ct][e] = fma(av[st][ct].y, f1[st][e], part[ct][e]);
      }
      part[ct][VD_LDF] = fma(av[st][ct].x, av[st][ct].x, part[ct][VD_LDF]);
      part[ct][VD_LDF] = fma(av[st][ct].y, av[st][ct].y, part[ct][VD_LDF]);
    }
  };
#pragma unroll
  for (int st = 0; st < DEPTH; st++) fetch(clamp(wave + 8 * st), av[st], f0[st], f1[st]);
  // whole rounds of DEPTH octets without a branch (so that each wait is for
  // the stage it feeds, not for every load in flight), then the last round
  int64_t o0 = wave;
  for (; o0 + 8 * (DEPTH - 1) < noct; o0 += 8 * DEPTH) {
#pragma unroll
    for (int st = 0; st < DEPTH; st++) {
      products(st);
      __builtin_amdgcn_sched_barrier(0);
      fetch(clamp(o0 + 8 * (st + DEPTH)), av[st], f0[st], f1[st]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int st = 0; st < DEPTH; st++)
    if (o0 + 8 * st < noct) products(st);
  // the four lanes of each column: (r0 + r1) + (r2 + r3) on every lane
  // (a + b is b + a to the bit); lane r = 0 then holds the wave's sum
#pragma unroll
  for (int ct = 0; ct < 4; ct++)
#pragma unroll
    for (int e = 0; e < E; e++) {
      double v = part[ct][e];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (r == 0) red[(wave * AS_COLS + 16 * ct + cl) * E + e] = v;
    }
  __syncthreads();
  for (int idx = threadIdx.x; idx < AS_COLS * E; idx += 64 * AS_WAVES) {
    const int c = idx / E, e = idx % E;
    double v = 0.0;
    for (int w = 0; w < AS_WAVES; w++) v += red[(w * AS_COLS + c) * E + e];
    if (e < ldf) dots[c][e] = v;
    if (e == VD_LDF) dots[c][ldf] = v;
  }
  __syncthreads();
}

// Fixed-order sum over the waves of one 16-wide slice of the products:
// slice et of every tile lands in red, then dots[c][16 et + e] (e < elim)
// or, for the Gram slice (gram_pR > 0), dots[c][base + q] = G[c][c0 + q]
// for q < gram_pR, c0 the first column of c's problem in its tile.
template <int ET>
__device__ __forceinline__ void reduce_slice(const d4 (&acc)[4][ET + 1], int et, int wave, int lane,
                                             double (*red)[AS_RED_COLS][17],
                                             double (*dots)[AS_DOTS], int elim, int base,
                                             int gram_pR) {
  const int r = lane / 16, cl = lane % 16;
#pragma unroll
  for (int h = 0; h < AS_COLS / AS_RED_COLS; h++) {
    constexpr int TPH = AS_RED_COLS / 16;  // column tiles per pass
#pragma unroll
    for (int ct = h * TPH; ct < (h + 1) * TPH; ct++)
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int k = 0; k <= ET; k++)
          if (k == et) red[wave][16 * (ct - h * TPH) + r + 4 * i][cl] = acc[ct][k][i];
    __syncthreads();
    for (int idx = threadIdx.x; idx < AS_RED_COLS * 16; idx += 64 * AS_WAVES) {
      const int cr = idx / 16, e = idx % 16, c = h * AS_RED_COLS + cr;
      if (gram_pR == 0) {
        if (16 * et + e < elim) {
          double v = 0.0;
          for (int w = 0; w < AS_WAVES; w++) v += red[w][cr][e];
          dots[c][16 * et + e] = v;
        }
      } else if (e < gram_pR && c % 16 < 16 / gram_pR * gram_pR) {   // columns of a problem
        const int c0 = (c % 16) - (c % 16) % gram_pR;   // problem's first column in the tile
        double v = 0.0;
        for (int w = 0; w < AS_WAVES; w++) v += red[w][cr][c0 + e];
        dots[c][base + e] = v;
      }
    }
    __syncthreads();
  }
}

// REFINE = false: the FP64 path.  REFINE = true: the FP32_REFINE form; the
// whitened columns are those of the centered genotypes x' = x - s, S^(0) and
// c^(0) come from them, and one FP64 refinement step on the normal
// equations uses S' = [S_TL, E^T; E, S^(0)_BR], c' = [C_T; e_y] with
// E = x'^T Z_L and e_y = x'^T Z_y exact to FP64 rounding (Z = M^{-1}[X_L|Y]):
//   r = c' - S' b0,  d = (G G^T)^{-1} r,  b' = b0 + d,
// then b_L[icol] -= s^T b'_R undoes the centering.
template <bool REFINE, int ET>
__global__ __launch_bounds__(64 * AS_WAVES, ET <= 1 ? 4 : 2) void k_assemble_solve(const AsmTable tab) {
  __shared__ double red[AS_WAVES][AS_RED_COLS][17];
  __shared__ double dots[AS_COLS][AS_DOTS];

  int jb = 0;
  while (jb + 1 < tab.njobs && (int64_t)blockIdx.x >= tab.j[jb + 1].grp0) jb++;
  const AsmDesc& J = tab.j[jb];
  const int pL = J.pL, pR = J.pR, t = J.t, p = pL + pR;
  const int ldf = pL + t;
  const int PT = 16 / pR;                   // problems per tile
  const int G = 4 * PT;                     // problems per group
  const int64_t snp0 = ((int64_t)blockIdx.x - J.grp0) * G;
  const int ng = (int)((J.nsnp - snp0) < G ? (J.nsnp - snp0) : G);
  const int64_t col0 = snp0 * pR;           // first genotype column of the group
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;
  const int r = lane / 16, cl = lane % 16;

  // lane (r, cl) of tile ct reads column col0 + (ct PT) pR + cl when that is
  // a column of the group, else column col0 (its products are not used)
  size_t base[4];
#pragma unroll
  for (int ct = 0; ct < 4; ct++) {
    const int gp = ct * PT + cl / pR;       // problem of the lane's column
    const bool valid = cl < PT * pR && gp < ng;
    base[ct] = slab_index(r, col0 + (valid ? (int64_t)ct * PT * pR + cl : 0), J.C, J.n_pad);
  }
  const size_t ostride = (size_t)(J.C / 16) * 128;  // one row octet of a slab
  const double* __restrict__ W = J.W;
  auto loadA = [&](int ct, int64_t o) __attribute__((always_inline)) -> d2 {
    return *reinterpret_cast<const d2*>(W + base[ct] + (size_t)o * ostride);
  };
  if constexpr (ET == 0) {
    // (every job of this launch has p_R = 1 and ldf <= VD_LDF)
    static_assert(AS_WAVES * AS_COLS * (VD_LDF + 1) <= AS_WAVES * AS_RED_COLS * 17, "red holds the sums");
    valu_dots(loadA, J.F, ldf, (J.n + 7) / 8, wave, lane, &red[0][0][0], dots);
  } else {
    d4 acc[4][ET + 1];
    mfma_dots<ET, true>(loadA, J.F, ldf, (J.n + 7) / 8, wave, lane, acc);
#pragma unroll
    for (int et = 0; et < ET; et++) reduce_slice<ET>(acc, et, wave, lane, red, dots, ldf, 0, 0);
    reduce_slice<ET>(acc, ET, wave, lane, red, dots, 0, ldf, pR);
  }

  // one wavefront per problem
  for (int g = wave; g < ng; g += AS_WAVES) {
    const int c0 = 16 * (g / PT) + (g % PT) * pR;   // the problem's first column in dots
    // S^(0)[a][b] of Fig. 1 from S_TL and the reduced dot products
    auto S0 = [&](int a, int b) -> double {
      if (a < pL && b < pL) return J.STL[a + b * pL];
      if (a >= pL && b >= pL) return dots[c0 + a - pL][ldf + b - pL];
      if (a >= pL) return dots[c0 + a - pL][b];
      return dots[c0 + b - pL][a];
    };
    double col[MAXP], crow[MAXT];
#pragma unroll
    for (int a = 0; a < MAXP; a++) col[a] = (lane < p && a < p) ? S0(a, lane) : 0.0;
#pragma unroll
    for (int j = 0; j < MAXT; j++) {
      crow[j] = 0.0;
      if (lane < p && j < t) crow[j] = lane < pL ? J.CT[lane + j * pL] : dots[c0 + lane - pL][pL + j];
    }
    int fail = 0;
    wave_cholesky(col, p, lane, fail);
    if (!fail) {
      wave_cholsolve(col, crow, p, t, lane);
      if (REFINE) {
        // residual of the normal equations with the FP64-exact blocks
        const int64_t cbase = col0 + (int64_t)g * pR;  // first genotype column of the problem
        double rr[MAXT];
#pragma unroll
        for (int j = 0; j < MAXT; j++) {
          rr[j] = 0.0;
          if (j < t) {
            double v = 0.0;
            if (lane < pL) v = J.CT[lane + j * pL];
            else if (lane < p) v = J.XZ[(cbase + lane - pL) * ldf + pL + j];
            for (int b = 0; b < p; b++) {
              const double bb = bcast_lane(crow[j], b);
              double sab = 0.0;
              if (lane < pL && b < pL) sab = J.STL[lane + b * pL];
              else if (lane < pL && b < p) sab = J.XZ[(cbase + b - pL) * ldf + lane];
              else if (lane < p && b < pL) sab = J.XZ[(cbase + lane - pL) * ldf + b];
              else if (lane < p && b < p) sab = dots[c0 + lane - pL][ldf + b - pL];
              v -= sab * bb;
            }
            rr[j] = lane < p ? v : 0.0;
          }
        }
        wave_cholsolve(col, rr, p, t, lane);
#pragma unroll
        for (int j = 0; j < MAXT; j++) crow[j] += rr[j];
        // undo the centering: b_L[icol] -= sum_q s_q b'_R[q]
#pragma unroll
        for (int j = 0; j < MAXT; j++) {
          if (j < t) {
            double corr = 0.0;
            for (int qq = 0; qq < pR; qq++) corr += J.shift[cbase + qq] * bcast_lane(crow[j], pL + qq);
            if (lane == J.icol) crow[j] -= corr;
          }
        }
      }
    }
    const int64_t i = snp0 + g;
    if (lane < p) {
#pragma unroll
      for (int j = 0; j < MAXT; j++)
        if (j < t) J.B[(i * t + j) * J.ldb + lane] = fail ? NAN : crow[j];
    }
    if (lane == 0 && J.info) J.info[i] = fail;
  }
}

// ---------------------------------------------------------------------------
// a5: FP32_REFINE form

// Centering pre-pass: per genotype column the exact dyadic shift
// s = round(256 * mean(x)) / 256 (x - s is exact in FP32: at most 10
// significant bits) and (x - s)^T Z with Z = M^{-1}[X_L | Y], in one read of
// the genotypes: x^T Z and the integer column sum are accumulated together,
// and (x - s)^T Z = x^T Z - s (1^T Z) with 1^T Z summed once per cohort.
// One work-group per 64 columns, one column per lane; its XZ_WAVES waves
// take contiguous segments of rows (multiples of 16), each lane reading 16
// genotypes of its column per step (one 16-byte load when the column start
// and the leading dimension allow it, byte loads otherwise and at the end of
// a segment) and updating its ldf products with FP64 FMAs, the row of Z
// being the same for the whole wave (scalar loads).  The segments' partial
// products meet in LDS and are summed in wave order, so a column's result
// depends on its column alone.  FMAs rather than matrix cores: there are
// only ldf = p_L + t products per genotype, fewer than the 16-wide tile of
// an FP64 MFMA.
constexpr int XZ_WAVES = 8;

template <int LDFMAX>
__global__ __launch_bounds__(64 * XZ_WAVES) void k_xz_shift(const XzTable tab) {
  __shared__ double part[XZ_WAVES][4][64];
  __shared__ int isum[XZ_WAVES][64];
  int jb = 0;
  while (jb + 1 < tab.njobs && (int64_t)blockIdx.x >= tab.j[jb + 1].grp0) jb++;
  const XzDesc& J = tab.j[jb];
  const int64_t col0 = ((int64_t)blockIdx.x - J.grp0) * 64;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;
  const int64_t n = J.n;
  const int ldf = J.ldf;
  const int64_t col = col0 + lane < J.ncols ? col0 + lane : col0;
  const int8_t* __restrict__ x = J.X + col * J.ldx;
  const double* __restrict__ Z = J.Z;
  const bool vec = ((reinterpret_cast<uintptr_t>(J.X) | (uintptr_t)J.ldx) & 15) == 0;
  const int64_t seg = (n + 16 * XZ_WAVES - 1) / (16 * XZ_WAVES) * 16;
  const int64_t r0 = (int64_t)wave * seg, r1 = r0 + seg < n ? r0 + seg : n;
  double acc[LDFMAX];
#pragma unroll
  for (int e = 0; e < LDFMAX; e++) acc[e] = 0.0;
  int s = 0;
  // 16 genotypes of the lane's column times 16 rows of Z (every one of the
  // LDFMAX entries of a row is read: Z carries LDFMAX doubles of padding past
  // its last row, and the products past ldf are never used).  The rows of Z
  // go to scalar registers RG at a time, so that no more than about 80 of
  // them hold rows in flight.
  constexpr int RG = LDFMAX <= 4 ? 16 : LDFMAX <= 8 ? 4 : LDFMAX <= 20 ? 2 : 1;
  auto step = [&](int64_t row, const int (&g)[16]) __attribute__((always_inline)) {
#pragma unroll
    for (int i = 0; i < 16; i++) {
      s += g[i];
      const double xi = (double)g[i];
      const double* __restrict__ zr = Z + (row + i) * ldf;
#pragma unroll
      for (int e = 0; e < LDFMAX; e++) acc[e] = fma(xi, zr[e], acc[e]);
      if ((i + 1) % RG == 0) __builtin_amdgcn_sched_barrier(0);
    }
  };
  auto unpack = [](const uint4& v, int (&g)[16]) __attribute__((always_inline)) {
    const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 16; i++) g[i] = (int)(int8_t)(w4[i / 4] >> (8 * (i % 4)));
  };
  int64_t row = r0;
  if (vec && row + 16 <= r1) {
    // the next 16 genotypes are loaded while the current ones are used
    uint4 nxt = *reinterpret_cast<const uint4*>(x + row);
    for (; row + 16 <= r1; row += 16) {
      const uint4 cur = nxt;
      if (row + 32 <= r1) nxt = *reinterpret_cast<const uint4*>(x + row + 16);
      int g[16];
      unpack(cur, g);
      step(row, g);
    }
  }
  for (; row < r1; row += 16) {
    // unaligned genotypes, or the rows past the last full 16 (0 past r1,
    // with Z rows that exist: r1 <= n rounded up to 16 <= n_pad)
    int g[16];
#pragma unroll
    for (int i = 0; i < 16; i++) g[i] = row + i < r1 ? (int)x[row + i] : 0;
    step(row, g);
  }
  isum[wave][lane] = s;
  // the segments' partial products, four entries at a time, summed in wave
  // order by the wave that owns the entry
#pragma unroll
  for (int e0 = 0; e0 < LDFMAX; e0 += 4) {
#pragma unroll
    for (int q = 0; q < 4; q++) part[wave][q][lane] = e0 + q < LDFMAX ? acc[e0 + q] : 0.0;
    __syncthreads();
    if (wave < 4 && e0 + wave < ldf) {
      int tot = 0;
      for (int w = 0; w < XZ_WAVES; w++) tot += isum[w][lane];
      const double shift = rint(256.0 * (double)tot / (double)n) / 256.0;
      double v = 0.0;
      for (int w = 0; w < XZ_WAVES; w++) v += part[w][wave][lane];
      if (col0 + lane < J.ncols) {
        J.XZ[(col0 + lane) * ldf + e0 + wave] = v - shift * J.z1[e0 + wave];
        if (e0 == 0 && wave == 0) J.shift[col0 + lane] = shift;
      }
    }
    __syncthreads();
  }
}

// z1 = 1^T Z (column sums of Z over its n rows): one work-group per column,
// fixed-order reduction.
__global__ __launch_bounds__(256) void k_colsum(const double* __restrict__ Z, int64_t n, int ld,
                                                double* __restrict__ z1) {
  const int e = blockIdx.x;
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) s += Z[r * ld + e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) z1[e] = red[0];
}


hipError_t launch_assemble_solve(const AsmTable& tab_in, int64_t ngroups, bool refine, hipStream_t st) {
  // The jobs with one genotype column per problem and ldf <= VD_LDF go to
  // the FMA form (ET = 0), the others to the MFMA form, each in a launch of
  // its own: a job takes the same form whatever the other jobs of the call,
  // so its results do not depend on them.
  AsmTable fma_tab, tab;
  fma_tab.njobs = tab.njobs = 0;
  int64_t fma_groups = 0, groups = 0;
  for (int i = 0; i < tab_in.njobs; i++) {
    AsmDesc d = tab_in.j[i];
    const int64_t per_group = (AS_GROUP_COLS / 16) * (16 / d.pR);
    const int64_t ng = (d.nsnp + per_group - 1) / per_group;
    if (d.pR == 1 && d.pL + d.t <= VD_LDF) {
      d.grp0 = fma_groups;
      fma_tab.j[fma_tab.njobs++] = d;
      fma_groups += ng;
    } else {
      d.grp0 = groups;
      tab.j[tab.njobs++] = d;
      groups += ng;
    }
  }
  if (fma_groups + groups != ngroups) return hipErrorInvalidValue;
  const unsigned nt = 64 * AS_WAVES;
  if (fma_groups > 0) {
    if (refine) k_assemble_solve<true, 0><<<(unsigned)fma_groups, nt, 0, st>>>(fma_tab);
    else k_assemble_solve<false, 0><<<(unsigned)fma_groups, nt, 0, st>>>(fma_tab);
  }
  if (groups == 0) return hipGetLastError();
  int w = 1;  // widest F = [W_L | ytil] of the table: one or two 16-column tiles
  for (int i = 0; i < tab.njobs; i++) w = std::max(w, tab.j[i].pL + tab.j[i].t);
  const unsigned g = (unsigned)groups;
  if (w <= 16) {
    if (refine) k_assemble_solve<true, 1><<<g, nt, 0, st>>>(tab);
    else k_assemble_solve<false, 1><<<g, nt, 0, st>>>(tab);
  } else {
    if (refine) k_assemble_solve<true, 2><<<g, nt, 0, st>>>(tab);
    else k_assemble_solve<false, 2><<<g, nt, 0, st>>>(tab);
  }
  return hipGetLastError();
}

hipError_t launch_xz_shift(const XzTable& tab, int64_t ngroups, hipStream_t st) {
  int w = 1;  // widest Z = M^{-1}[X_L | Y] of the table
  for (int i = 0; i < tab.njobs; i++) w = std::max(w, tab.j[i].ldf);
  const unsigned g = (unsigned)ngroups, nt = 64 * XZ_WAVES;
  if (w <= 4) k_xz_shift<4><<<g, nt, 0, st>>>(tab);
  else if (w <= 8) k_xz_shift<8><<<g, nt, 0, st>>>(tab);
  else if (w <= 16) k_xz_shift<16><<<g, nt, 0, st>>>(tab);
  else if (w <= 20) k_xz_shift<20><<<g, nt, 0, st>>>(tab);
  else if (w <= MAXP + MAXT) k_xz_shift<MAXP + MAXT><<<g, nt, 0, st>>>(tab);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_colsum(const double* Z, int64_t n, int ld, double* z1, hipStream_t st) {
  k_colsum<<<(unsigned)ld, 256, 0, st>>>(Z, n, ld, z1);
  return hipGetLastError();
}

}  // namespace gls
