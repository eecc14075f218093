// Factorization of M and unpacking of the factor (a0).
#include "gls_device.h"

#include <utility>

namespace gls {

// ---------------------------------------------------------------------------
// a0: factorization  M = L L^T  (potrf; Alg. 3-5, first line)

// A := lower(M) padded to n_pad with the identity; strict upper part zero.
__global__ void k_copy_pad(const double* __restrict__ M, int64_t ldm, int64_t n,
                           double* __restrict__ A, int64_t n_pad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t j = blockIdx.y;
  for (; j < n_pad; j += gridDim.y) {
    if (i >= n_pad) return;
    double v;
    if (i < n && j < n) v = (i >= j) ? M[i + j * ldm] : 0.0;
    else v = (i == j) ? 1.0 : 0.0;
    A[i + j * n_pad] = v;
  }
}

// Cholesky of the diagonal block k and its inverse, blocked by 16 columns
// with the block in LDS (column-major, leading dimension SLD).
//   factor, panel p (columns c0 = 16p ..): wave 0 factors the panel (rows
//     c0 .. NB-1, 16 columns) in registers, lane l holding rows c0 + l and
//     c0 + l + 64: per column the pivot and the column of L come from
//     v_readlane broadcasts (no barrier), L[i][j] = A[i][j] * (1 / sqrt(A[j][j]))
//     (reciprocal multiply, as LAPACK's unblocked potf2), then the rank-1
//     update of the panel's later columns; then all four waves subtract
//     L21 L21^T from the trailing lower tiles on FP64 MFMA (16 x 16 tiles,
//     four k-steps each).  Two barriers per panel instead of one per column.
//   inverse X = inv(L), in packed lower storage: the diagonal 16 x 16 blocks
//     by forward substitution (one lane per column, X_pp e_j), then block
//     column j of X (two block columns per wave, j and 7 - j, so that every
//     wave has 7 blocks): X_ij = -X_ii sum_{m=j}^{i-1} L_im X_mj for
//     i = j+1 .., both products on FP64 MFMA.
// Writes L_kk into A and into Ldiag[k], inv(L_kk) into Linv[k] (NB x NB
// column-major, lower, zeros above).  A non-positive or non-finite pivot of a
// real row sets *info (order of the failing leading minor) and stops the
// process: every later kernel sees *info != 0 and returns at once.
constexpr int SLD = NB + 1;                   // padded leading dimension of the block in LDS
__device__ __forceinline__ int pk(int r, int c) { return c * NB - c * (c - 1) / 2 + (r - c); }  // packed lower
constexpr int PK = NB * (NB + 1) / 2;         // packed lower triangle

// wave 0: factor the panel of columns c0 .. c0+15 (rows c0 .. NB-1) of S in
// place; returns the failing pivot's code (0 if none)
__device__ __forceinline__ int panel_factor(double* __restrict__ S, int c0, int lane, int64_t o, int64_t n) {
  double v[2][16];
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int row = c0 + lane + 64 * h;
#pragma unroll
    for (int q = 0; q < 16; q++) v[h][q] = row < NB ? S[(c0 + q) * SLD + row] : 0.0;
  }
#pragma unroll
  for (int jj = 0; jj < 16; jj++) {
    const double d = bcast_lane(v[0][jj], jj);   // pivot A[c0+jj][c0+jj]: lane jj, first row set
    if (!(d > 0.0) || !(d < INFINITY)) return (o + c0 + jj < n) ? (int)(o + c0 + jj + 1) : (int)(o + 1);
    const double g = sqrt(d), rg = 1.0 / g;
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const int row = c0 + lane + 64 * h;
      v[h][jj] = row > c0 + jj ? v[h][jj] * rg : (row == c0 + jj ? g : 0.0);
    }
    // L[c0+jj'][jj] of the panel's later columns (lanes jj', first row set);
    // the entries above the diagonal this touches are never read
#pragma unroll
    for (int q = jj + 1; q < 16; q++) {
      const double lq = bcast_lane(v[0][jj], q);
#pragma unroll
      for (int h = 0; h < 2; h++) v[h][q] = fma(-v[h][jj], lq, v[h][q]);
    }
  }
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int row = c0 + lane + 64 * h;
    if (row < NB) {
#pragma unroll
      for (int q = 0; q < 16; q++) S[(c0 + q) * SLD + row] = row >= c0 + q ? v[h][q] : 0.0;
    }
  }
  return 0;
}

// all waves: S[r][c] -= sum_{q<16} L[r][c0+q] L[c][c0+q] over the lower
// 16 x 16 tiles (ti >= tj) of rows and columns >= c0 + 16
__device__ __forceinline__ void trailing_update(double* __restrict__ S, int c0, int wave, int lane) {
  const int T = (NB - c0) / 16 - 1;
  const int ntiles = T * (T + 1) / 2;
  const int i16 = lane % 16, k4 = lane / 16;
  for (int idx = wave; idx < ntiles; idx += 4) {
    // idx -> (ti, tj), tj <= ti, rows of tiles in order
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= idx) ti++;
    const int tj = idx - ti * (ti + 1) / 2;
    const int r0 = c0 + 16 + 16 * ti, q0 = c0 + 16 + 16 * tj;
    d4 acc;
#pragma unroll
    for (int e = 0; e < 4; e++) acc[e] = S[(q0 + i16) * SLD + r0 + k4 + 4 * e];
#pragma unroll
    for (int s = 0; s < 4; s++) {
      const double a = -S[(c0 + 4 * s + k4) * SLD + r0 + i16];   // A[i][k] = -L[r0 + i][c0 + 4s + k]
      const double b = S[(c0 + 4 * s + k4) * SLD + q0 + i16];    // B[k][j] = L[q0 + j][c0 + 4s + k]
      acc = MFMA64(a, b, acc);
    }
#pragma unroll
    for (int e = 0; e < 4; e++) S[(q0 + i16) * SLD + r0 + k4 + 4 * e] = acc[e];
  }
}

__global__ __launch_bounds__(256) void k_potf2_inv(double* __restrict__ A, int64_t lda,
                                                    int k, int64_t n,
                                                    double* __restrict__ Ldiag,
                                                    double* __restrict__ Linv,
                                                    int* __restrict__ info) {
  static_assert(NB == 128, "8 panels of 16 columns; two row sets of 64 lanes");
  // the block (factor phase), then the packed L and X (inverse phase) and
  // one 16 x 16 scratch tile per wave
  constexpr int S_DOUBLES = 2 * PK + 4 * 256 > NB * SLD ? 2 * PK + 4 * 256 : NB * SLD;
  __shared__ double S[S_DOUBLES];
  __shared__ int fail_s;
  if (*info != 0) return;
  const int t = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(t / 64), lane = t % 64;
  const int64_t o = (int64_t)k * NB;
  // (unconditional loads, 16 in flight: the block's strict upper part is
  // memory of the matrix too)
#pragma unroll 16
  for (int m = 0; m < NB * NB / 256; m++) {
    const int idx = t + 256 * m, r = idx % NB, c = idx / NB;
    const double v = A[(o + r) + (o + c) * lda];
    S[c * SLD + r] = r >= c ? v : 0.0;
  }
  if (t == 0) fail_s = 0;
  __syncthreads();
  for (int p = 0; p < NB / 16; p++) {
    const int c0 = 16 * p;
    if (wave == 0) {
      const int f = panel_factor(S, c0, lane, o, n);
      if (f && lane == 0) fail_s = f;
    }
    __syncthreads();
    if (fail_s) break;
    if (c0 + 16 < NB) trailing_update(S, c0, wave, lane);
    __syncthreads();
  }
  if (fail_s) {
    if (t == 0) *info = fail_s;
    return;
  }
  // L out; the lower triangle into registers for the packing
  double lreg[(PK + 255) / 256];
#pragma unroll
  for (int m = 0; m < (PK + 255) / 256; m++) lreg[m] = 0.0;
#pragma unroll 16
  for (int m = 0; m < NB * NB / 256; m++) {
    const int idx = t + 256 * m, r = idx % NB, c = idx / NB;
    const double sv = S[c * SLD + r];
    const double v = r >= c ? sv : 0.0;
    A[(o + r) + (o + c) * lda] = v;
    Ldiag[(size_t)k * NB * NB + r + (size_t)c * NB] = v;
  }
  // packed position pi = t + 256 m  ->  (r, c): c from the column ends
  // (pi grows with m, so c only moves forward)
  {
    int c = 0;
#pragma unroll
    for (int m = 0; m < (PK + 255) / 256; m++) {
      const int pi = t + 256 * m;
      if (pi < PK) {
        while (pk(NB - 1, c) < pi) c++;
        lreg[m] = S[c * SLD + c + (pi - pk(c, c))];
      }
    }
  }
  __syncthreads();
  double* __restrict__ Lp = S;               // packed L
  double* __restrict__ Xp = S + PK;          // packed X = inv(L)
  double* __restrict__ Tw = S + 2 * PK + 256 * wave;  // this wave's 16 x 16 scratch (row-major)
#pragma unroll
  for (int m = 0; m < (PK + 255) / 256; m++) {
    const int pi = t + 256 * m;
    if (pi < PK) Lp[pi] = lreg[m];
  }
  __syncthreads();
  // diagonal blocks: wave w takes blocks w and w + 4, lane j < 16 column j
  const int i16 = lane % 16, k4 = lane / 16;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int b0 = 16 * (wave + 4 * h);
    double x[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
      double sacc = i == lane ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < i; m++) sacc = fma(-Lp[pk(b0 + i, b0 + m)], x[m], sacc);
      x[i] = sacc * (1.0 / Lp[pk(b0 + i, b0 + i)]);
    }
    if (lane < 16) {
#pragma unroll
      for (int i = 0; i < 16; i++)
        if (i >= lane) Xp[pk(b0 + i, b0 + lane)] = x[i];
    }
  }
  __syncthreads();
  // off-diagonal blocks, block columns j = wave and 7 - wave
  auto xload = [&](int r, int c) -> double { return r >= c ? Xp[pk(r, c)] : 0.0; };
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int jb = h == 0 ? wave : NB / 16 - 1 - wave;
    for (int ib = jb + 1; ib < NB / 16; ib++) {
      // T = sum_{m=jb}^{ib-1} L_{ib,m} X_{m,jb}
      d4 acc = (d4){0, 0, 0, 0};
      for (int mb = jb; mb < ib; mb++) {
#pragma unroll
        for (int s = 0; s < 4; s++) {
          const int kk = 16 * mb + 4 * s + k4;
          const double a = Lp[pk(16 * ib + i16, kk)];   // A[i][k] = L[16 ib + i][kk]
          const double b = xload(kk, 16 * jb + i16);    // B[k][j] = X[kk][16 jb + j]
          acc = MFMA64(a, b, acc);
        }
      }
      // T to the scratch tile (row-major), then X_ij = -X_ii T
#pragma unroll
      for (int e = 0; e < 4; e++) Tw[(k4 + 4 * e) * 16 + i16] = acc[e];
      d4 acc2 = (d4){0, 0, 0, 0};
#pragma unroll
      for (int s = 0; s < 4; s++) {
        const double a = -xload(16 * ib + i16, 16 * ib + 4 * s + k4);   // A[i][k] = -X_ii[i][4s + k]
        const double b = Tw[(4 * s + k4) * 16 + i16];                    // B[k][j] = T[4s + k][j]
        acc2 = MFMA64(a, b, acc2);
      }
#pragma unroll
      for (int e = 0; e < 4; e++) Xp[pk(16 * ib + k4 + 4 * e, 16 * jb + i16)] = acc2[e];
    }
  }
  __syncthreads();
  // (pk(r, c) lies inside the packed X also for r < c: the reads are
  // unconditional)
#pragma unroll 16
  for (int m = 0; m < NB * NB / 256; m++) {
    const int idx = t + 256 * m, r = idx % NB, c = idx / NB;
    const double xv = Xp[pk(r, c)];
    Linv[(size_t)k * NB * NB + r + (size_t)c * NB] = r >= c ? xv : 0.0;
  }
}

// Tile product on MFMA: a 128 x 128 tile computed by 4 waves (64 x 64 each)
// from column-major operands: acc = sum_l A[i][l] * Bt[j][l] over 4 kd_end
// columns (A and Bt are NB-row panels with leading dimension lda / ldb;
// kd_end a multiple of 4).  The operands of k-step kk + 4 are loaded while
// k-step kk's MFMAs run: a ring of four k-steps, unrolled so that every slot
// is a fixed set of registers (indexes past the end are clamped to the last
// k-step; those loads are never used).
__device__ __forceinline__ void tile_abt(const double* __restrict__ Ap, int64_t lda,
                                         const double* __restrict__ Bp, int64_t ldb,
                                         int kd_end, d4 (&acc)[4][4], int wr, int wc, int lane) {
  constexpr int RING = 4;
  const int r16 = lane % 16, k4 = lane / 16;
  auto load = [&](int kk, double (&a)[4], double (&b)[4]) {
    kk = kk < kd_end ? kk : kd_end - 1;
    const int64_t col = 4 * kk + k4;
#pragma unroll
    for (int t = 0; t < 4; t++) {
      a[t] = Ap[(wr * 64 + t * 16 + r16) + col * lda];
      b[t] = Bp[(wc * 64 + t * 16 + r16) + col * ldb];
    }
  };
  double a[RING][4], b[RING][4];
#pragma unroll
  for (int s = 0; s < RING; s++) load(s, a[s], b[s]);
  for (int kk0 = 0; kk0 < kd_end; kk0 += RING) {
#pragma unroll
    for (int s = 0; s < RING; s++) {
#pragma unroll
      for (int rt = 0; rt < 4; rt++)
#pragma unroll
        for (int ct = 0; ct < 4; ct++) acc[rt][ct] = MFMA64(a[s][rt], b[s][ct], acc[rt][ct]);
      load(kk0 + s + RING, a[s], b[s]);
      // keep the refill where it is issued, RING k-steps ahead of its use
      asm volatile("" ::: "memory");
    }
  }
}

// Panel: A[r, k] := A[r, k] * inv(L_kk)^T for every row block r > k.
__global__ __launch_bounds__(256) void k_panel(double* __restrict__ A, int64_t lda, int k,
                                               const double* __restrict__ Linv,
                                               const int* __restrict__ info) {
  if (*info != 0) return;
  const int r = k + 1 + blockIdx.x;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wr = wave / 2, wc = wave % 2;
  double* Ap = A + (int64_t)r * NB + (int64_t)k * NB * lda;
  const double* Li = Linv + (size_t)k * NB * NB;
  d4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) acc[a][b] = (d4){0, 0, 0, 0};
  // inv(L_kk)[j][l] = 0 for l > j: columns of this wave end at wc*64+63
  tile_abt(Ap, lda, Li, NB, (wc * 64 + 64) / 4, acc, wr, wc, lane);
  __syncthreads();
#pragma unroll
  for (int rt = 0; rt < 4; rt++)
#pragma unroll
    for (int ct = 0; ct < 4; ct++)
#pragma unroll
      for (int i = 0; i < 4; i++)
        Ap[(wr * 64 + rt * 16 + lane / 16 + 4 * i) + (int64_t)(wc * 64 + ct * 16 + lane % 16) * lda] =
            acc[rt][ct][i];
}

// Trailing update: A[r, s] -= A[r, k] A[s, k]^T for s0 <= s <= r < K (one
// work-group per tile): the whole lower triangle of column blocks s >= s0,
// or (col_only) column block s0 alone.
__global__ __launch_bounds__(256) void k_syrk(double* __restrict__ A, int64_t lda, int k, int K,
                                              int s0, int col_only, const int* __restrict__ info) {
  if (*info != 0) return;
  const int64_t t = blockIdx.x;
  int r, s;
  if (col_only) {
    r = s0 + (int)t;
    s = s0;
  } else {
    int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((int64_t)(i + 1) * (i + 2) / 2 <= t) i++;
    while ((int64_t)i * (i + 1) / 2 > t) i--;
    const int j = (int)(t - (int64_t)i * (i + 1) / 2);
    r = s0 + i;
    s = s0 + j;
  }
  if (r >= K) return;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wr = wave / 2, wc = wave % 2;
  double* C = A + (int64_t)r * NB + (int64_t)s * NB * lda;
  // -(-C + A_rk A_sk^T): the same bits as C - A_rk A_sk^T (round to nearest
  // is symmetric under negation), with unnegated operands in the MFMAs
  d4 acc[4][4];
#pragma unroll
  for (int rt = 0; rt < 4; rt++)
#pragma unroll
    for (int ct = 0; ct < 4; ct++)
#pragma unroll
      for (int e = 0; e < 4; e++)
        acc[rt][ct][e] = -C[(wr * 64 + rt * 16 + lane / 16 + 4 * e) + (int64_t)(wc * 64 + ct * 16 + lane % 16) * lda];
  tile_abt(A + (int64_t)r * NB + (int64_t)k * NB * lda, lda,
           A + (int64_t)s * NB + (int64_t)k * NB * lda, lda, NB / 4, acc, wr, wc, lane);
#pragma unroll
  for (int rt = 0; rt < 4; rt++)
#pragma unroll
    for (int ct = 0; ct < 4; ct++)
#pragma unroll
      for (int e = 0; e < 4; e++)
        C[(wr * 64 + rt * 16 + lane / 16 + 4 * e) + (int64_t)(wc * 64 + ct * 16 + lane % 16) * lda] = -acc[rt][ct][e];
}

// Pack L's off-diagonal strips and the inverted diagonal blocks into the
// fragment layout.  Block (k, j) of the grid: j < k packs L[k, j] into
// strip k; j == k packs inv(L_kk).  FP32 copies are written when Lstrips32
// is not null (FP32_REFINE form).
__global__ __launch_bounds__(256) void k_pack(const double* __restrict__ A, int64_t lda,
                                              const double* __restrict__ Linv,
                                              double* __restrict__ Lstrips,
                                              double* __restrict__ LinvP,
                                              float* __restrict__ Lstrips32, int K) {
  const int64_t t = blockIdx.x;  // enumerates (k, j), 0 <= j <= k < K
  int k = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(k + 1) * (k + 2) / 2 <= t) k++;
  while ((int64_t)k * (k + 1) / 2 > t) k--;
  const int j = (int)(t - (int64_t)k * (k + 1) / 2);
  for (int d = threadIdx.x; d < NB * NB; d += 256) {
    // d = ((kp * (NB/16) + rt) * 64 + lane) * 2 + kk, with kp local to block j
    const int kk = d & 1, lane = (d >> 1) & 63, rt = (d >> 7) % (NB / 16), kp = (d >> 7) / (NB / 16);
    const int row = rt * 16 + lane % 16;       // within the block
    const int colb = (2 * kp + kk) * 4 + lane / 16;
    if (j < k) {
      const double v = A[((int64_t)k * NB + row) + ((int64_t)j * NB + colb) * lda];
      const size_t dst = strip_offset(k) + (size_t)j * NB * NB + d;
      Lstrips[dst] = v;
      if (Lstrips32) {
        // FP32 copy in the quad layout: ((kq * (NB/16) + rt) * 64 + lane) * 4 + k-step % 4
        const int ks = colb / 4, lane32 = (colb % 4) * 16 + row % 16;
        const size_t dst32 = strip_offset(k) + (size_t)j * NB * NB +
                             ((size_t)((ks / 4) * (NB / 16) + row / 16) * 64 + lane32) * 4 + ks % 4;
        Lstrips32[dst32] = (float)v;
      }
    } else {
      LinvP[(size_t)k * NB * NB + d] = Linv[(size_t)k * NB * NB + row + (size_t)colb * NB];
    }
  }
}

// Unpack the factor (strips + diagonal blocks) to a caller's column-major
// n x n array; the strict upper triangle is zeroed.
__global__ void k_unpack_factor(const double* __restrict__ Lstrips,
                                const double* __restrict__ Ldiag, int64_t n,
                                double* __restrict__ L, int64_t ldl) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
    if (i >= n) return;
    double v = 0.0;
    if (i >= j) {
      const int kb = (int)(i / NB), jb = (int)(j / NB);
      const int row = (int)(i % NB), colb = (int)(j % NB);
      if (kb == jb) {
        v = Ldiag[(size_t)kb * NB * NB + row + (size_t)colb * NB];
      } else {
        const int col = (int)j;
        const int ks = col / 4, kp_ = ks / 2, kk = ks % 2;
        const int lane = (col % 4) * 16 + row % 16, rt = row / 16;
        v = Lstrips[strip_offset(kb) + ((size_t)kp_ * (NB / 16) + rt) * 128 + lane * 2 + kk];
      }
    }
    L[i + j * ldl] = v;
  }
}


hipError_t launch_factor(const double* M, int64_t ldm, int64_t n, int64_t n_pad, int K,
                         double* A, double* Ldiag, double* Linv, double* Lstrips, double* LinvP,
                         float* Lstrips32, int* dinfo, hipStream_t st) {
  {
    dim3 grid((unsigned)((n_pad + 255) / 256), (unsigned)(n_pad < 65535 ? n_pad : 65535));
    k_copy_pad<<<grid, 256, 0, st>>>(M, ldm, n, A, n_pad);
  }
  // Right-looking with a lookahead of one block column: step k updates the
  // next column block k+1 first, on st, then the rest of the trailing matrix
  // on a second stream, so that the diagonal step and the panel of k+1 (a
  // sequential chain of small launches) run beside the large update of k.
  // Before it updates column block k+1, step k waits for the rest-update of
  // step k-1 (which also wrote that column); the last one is waited for
  // before the packing.
  hipStream_t s2 = nullptr;
  hipEvent_t ev_panel = nullptr, ev_rest = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_panel, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ev_rest, hipEventDisableTiming);
  bool rest_pending = false;
  for (int k = 0; k < K && e == hipSuccess; k++) {
    k_potf2_inv<<<1, 256, 0, st>>>(A, n_pad, k, n, Ldiag, Linv, dinfo);
    if (k + 1 >= K) break;
    k_panel<<<K - 1 - k, 256, 0, st>>>(A, n_pad, k, Linv, dinfo);
    if (rest_pending) e = hipStreamWaitEvent(st, ev_rest, 0);
    if (e != hipSuccess) break;
    const int64_t d = K - 1 - k;
    k_syrk<<<(unsigned)d, 256, 0, st>>>(A, n_pad, k, K, k + 1, 1, dinfo);
    rest_pending = false;
    if (d > 1) {
      const int64_t d2 = d - 1;
      e = hipEventRecord(ev_panel, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(s2, ev_panel, 0);
      if (e != hipSuccess) break;
      k_syrk<<<(unsigned)(d2 * (d2 + 1) / 2), 256, 0, s2>>>(A, n_pad, k, K, k + 2, 0, dinfo);
      e = hipEventRecord(ev_rest, s2);
      rest_pending = true;
    }
  }
  if (e == hipSuccess && rest_pending) e = hipStreamWaitEvent(st, ev_rest, 0);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) {
    const int64_t nblk = (int64_t)K * (K + 1) / 2;
    k_pack<<<(unsigned)nblk, 256, 0, st>>>(A, n_pad, Linv, Lstrips, LinvP, Lstrips32, K);
    e = hipGetLastError();
  }
  // the second stream's work is ordered before st's packing; its handles go
  // once that work is done
  if (s2) {
    (void)hipStreamSynchronize(s2);
    (void)hipStreamDestroy(s2);
  }
  if (ev_panel) (void)hipEventDestroy(ev_panel);
  if (ev_rest) (void)hipEventDestroy(ev_rest);
  return e;
}

hipError_t launch_unpack_factor(const double* Lstrips, const double* Ldiag, int64_t n, double* L,
                                int64_t ldl, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)(n < 65535 ? n : 65535));
  k_unpack_factor<<<grid, 256, 0, st>>>(Lstrips, Ldiag, n, L, ldl);
  return hipGetLastError();
}

}  // namespace gls
