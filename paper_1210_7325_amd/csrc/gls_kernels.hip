// Device kernels of the GLS-sequence solver (gfx950 / CDNA4).
//
// Paper: Fabregat-Traver, Aulchenko, Bientinesi, "Solving Sequences of
// Generalized Least-Squares Problems on Multi-threaded Architectures".
// The kernels implement the steps of the in-core algorithm "hp-gwas"
// (Sec. 2, Alg. 5): potrf of M, trsm of X_L / y / the genotype block,
// syrk/gemv for S_TL and C_T, and per problem the gemv/dot assembly of
// S_i, c_i (Fig. 1) followed by posv.
//
// Layouts (all FP64 unless noted):
//  * A: the factorization's work matrix, n_pad x n_pad column-major
//    (n_pad = K*NB), identity on the padded diagonal.
//  * Packed factor for the triangular solve ("fragment layout"): the strip
//    of row block k, L[kNB:(k+1)NB, 0:kNB], is stored as a sequence of
//    k-step pairs; one pair holds, for each 16-row tile, 64 lanes x 2
//    doubles, lane l of k-step s holding L[row0 + l%16][4s + l/16] (the A
//    operand of v_mfma_f64_16x16x4f64).  Strip k starts at k(k-1)/2 NB^2.
//    The inverted diagonal blocks use the same layout with NB columns.
//  * Whitened genotypes ("slab layout"): columns are grouped in slabs of C;
//    a slab holds n_pad x C values as k-step pairs of 16-column tiles, lane
//    l of k-step s holding W[4s + l/16][16ct + l%16] (the B operand).
//  * FP64 MFMA output: lane l, element i holds D[l/16 + 4i][l%16], which is
//    exactly the B-operand position of k-step (tile_row0/4 + i) at lane l,
//    so results go to the slab layout without any lane exchange.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include <algorithm>

#include "gls_internal.h"

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

#define MFMA64(a, b, c) __builtin_amdgcn_mfma_f64_16x16x4f64((a), (b), (c), 0, 0, 0)
#define MFMA32(a, b, c) __builtin_amdgcn_mfma_f32_16x16x4f32((a), (b), (c), 0, 0, 0)

namespace gls {

// ---------------------------------------------------------------------------
// small helpers
__device__ __forceinline__ double bcast_lane(double v, int src) {
  // v of lane `src` to every lane (src is wave-uniform)
  int2 x = *reinterpret_cast<int2*>(&v);
  x.x = __builtin_amdgcn_readlane(x.x, src);
  x.y = __builtin_amdgcn_readlane(x.y, src);
  return *reinterpret_cast<double*>(&x);
}

__device__ __forceinline__ size_t strip_offset(int k) {
  return (size_t)k * (size_t)(k - 1) / 2 * (size_t)(NB * NB);
}

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

// Unblocked Cholesky of the diagonal block k in LDS, then its inverse.
// Writes L_kk into A and into Ldiag[k], inv(L_kk) into Linv[k] (NB x NB
// column-major, lower).  A non-positive or non-finite pivot of a real row
// sets *info (order of the failing leading minor) and stops the process:
// every later kernel sees *info != 0 and returns at once.
__global__ __launch_bounds__(256) void k_potf2_inv(double* __restrict__ A, int64_t lda,
                                                    int k, int64_t n,
                                                    double* __restrict__ Ldiag,
                                                    double* __restrict__ Linv,
                                                    int* __restrict__ info) {
  __shared__ double T[NB][NB + 1];
  __shared__ int fail;
  if (*info != 0) return;
  const int tid = threadIdx.x;
  const int64_t o = (int64_t)k * NB;
  for (int idx = tid; idx < NB * NB; idx += 256) {
    int i = idx % NB, j = idx / NB;
    T[i][j] = (i >= j) ? A[(o + i) + (o + j) * lda] : 0.0;
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int j = 0; j < NB; j++) {
    double d = T[j][j];
    if (!(d > 0.0) || !(d < INFINITY)) {
      if (tid == 0) fail = (o + j < n) ? (int)(o + j + 1) : -1;
      break;
    }
    double g = sqrt(d);
    __syncthreads();
    for (int i = j + 1 + tid; i < NB; i += 256) T[i][j] /= g;
    if (tid == 0) T[j][j] = g;
    __syncthreads();
    const int m = NB - j - 1;
    for (int idx = tid; idx < m * m; idx += 256) {
      int i = j + 1 + idx / m, l = j + 1 + idx % m;
      if (l <= i) T[i][l] -= T[i][j] * T[l][j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (fail != 0) {
    if (tid == 0) *info = fail > 0 ? fail : (int)(o + 1);
    return;
  }
  for (int idx = tid; idx < NB * NB; idx += 256) {
    int i = idx % NB, j = idx / NB;
    double v = (i >= j) ? T[i][j] : 0.0;
    A[(o + i) + (o + j) * lda] = v;
    Ldiag[(size_t)k * NB * NB + idx] = v;
  }
  __syncthreads();
  // in-place inverse, last column first: column j of inv(L) below the
  // diagonal is -inv(L)[j+1:, j+1:] L[j+1:, j] / L[j][j]
  __shared__ double s[NB];
  for (int j = NB - 1; j >= 0; j--) {
    double djj = 1.0 / T[j][j];
    for (int i = j + 1 + tid; i < NB; i += 256) {
      double acc = 0.0;
      for (int l = j + 1; l <= i; l++) acc += T[i][l] * T[l][j];
      s[i] = acc;
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < NB; i += 256) T[i][j] = -djj * s[i];
    if (tid == 0) T[j][j] = djj;
    __syncthreads();
  }
  for (int idx = tid; idx < NB * NB; idx += 256) {
    int i = idx % NB, j = idx / NB;
    Linv[(size_t)k * NB * NB + idx] = (i >= j) ? T[i][j] : 0.0;
  }
}

// Tile product on MFMA: a 128 x 128 tile computed by 4 waves (64 x 64 each)
// from column-major operands: acc = sum_l A[i][l] * Bt[j][l] over KD
// columns (A and Bt are NB-row panels with leading dimension lda / ldb).
__device__ __forceinline__ void tile_abt(const double* __restrict__ Ap, int64_t lda,
                                         const double* __restrict__ Bp, int64_t ldb,
                                         int kd_end, d4 (&acc)[4][4], int wr, int wc,
                                         int lane, double sign) {
  const int r16 = lane % 16, k4 = lane / 16;
  for (int kk = 0; kk < kd_end; kk++) {
    double a[4], b[4];
    const int64_t col = 4 * kk + k4;
#pragma unroll
    for (int t = 0; t < 4; t++) {
      a[t] = sign * Ap[(wr * 64 + t * 16 + r16) + col * lda];
      b[t] = Bp[(wc * 64 + t * 16 + r16) + col * ldb];
    }
#pragma unroll
    for (int rt = 0; rt < 4; rt++)
#pragma unroll
      for (int ct = 0; ct < 4; ct++) acc[rt][ct] = MFMA64(a[rt], b[ct], acc[rt][ct]);
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
  tile_abt(Ap, lda, Li, NB, (wc * 64 + 64) / 4, acc, wr, wc, lane, 1.0);
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

// Trailing update: A[r, s] -= A[r, k] A[s, k]^T for k < s <= r < K.
__global__ __launch_bounds__(256) void k_syrk(double* __restrict__ A, int64_t lda, int k, int K,
                                              const int* __restrict__ info) {
  if (*info != 0) return;
  const int64_t t = blockIdx.x;
  int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((int64_t)(i + 1) * (i + 2) / 2 <= t) i++;
  while ((int64_t)i * (i + 1) / 2 > t) i--;
  const int j = (int)(t - (int64_t)i * (i + 1) / 2);
  const int r = k + 1 + i, s = k + 1 + j;
  if (r >= K) return;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wr = wave / 2, wc = wave % 2;
  double* C = A + (int64_t)r * NB + (int64_t)s * NB * lda;
  d4 acc[4][4];
#pragma unroll
  for (int rt = 0; rt < 4; rt++)
#pragma unroll
    for (int ct = 0; ct < 4; ct++)
#pragma unroll
      for (int e = 0; e < 4; e++)
        acc[rt][ct][e] = C[(wr * 64 + rt * 16 + lane / 16 + 4 * e) + (int64_t)(wc * 64 + ct * 16 + lane % 16) * lda];
  tile_abt(A + (int64_t)r * NB + (int64_t)k * NB * lda, lda,
           A + (int64_t)s * NB + (int64_t)k * NB * lda, lda, NB / 4, acc, wr, wc, lane, -1.0);
#pragma unroll
  for (int rt = 0; rt < 4; rt++)
#pragma unroll
    for (int ct = 0; ct < 4; ct++)
#pragma unroll
      for (int e = 0; e < 4; e++)
        C[(wr * 64 + rt * 16 + lane / 16 + 4 * e) + (int64_t)(wc * 64 + ct * 16 + lane % 16) * lda] = acc[rt][ct][e];
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

// ---------------------------------------------------------------------------
// a1/a2: blocked lower triangular solve  W = L^{-1} X  (the trsm of Alg. 5,
// grouped over many right-hand sides as the paper prescribes)
//
// One work-group owns a slab of C columns and walks the row blocks
// k = 0..K-1 (left-looking):
//   R_k = X_k - sum_{j<k} L_kj W_j     FP64 MFMA, operands streamed from the
//                                      packed strip and the slab's own W
//   W_k = inv(L_kk) R_k                FP64 MFMA, R_k staged in LDS
// The waves split the NB rows of a block (WR ways) and the C columns (WC
// ways).  X is int8 genotypes (exact in FP64) or FP64 (fixed part).
template <typename TIn>
__device__ __forceinline__ double load_x(const TIn* __restrict__ X, int64_t ldx, int64_t row,
                                         int64_t col, int64_t n, int64_t ncols) {
  return (row < n && col < ncols) ? (double)X[col * ldx + row] : 0.0;
}

template <int C, int WR, int WC, int D, typename TIn>
__global__ __launch_bounds__(64 * WR * WC) void k_trsm(const JobTable tab) {
  constexpr int RW = NB / WR, RT = RW / 16;
  constexpr int CW = C / WC, CT = CW / 16;
  constexpr int CTS = C / 16;  // column tiles per slab
  constexpr int NPB = NB / 8;  // k-step pairs per row block
  static_assert(RT >= 1 && CT >= 1, "tile shape");
  static_assert(NPB % D == 0, "prefetch depth must divide the pairs of a block");
  __shared__ __attribute__((aligned(16))) double Rl[NB * C];

  // find the job of this slab
  int jb = 0;
  while (jb + 1 < tab.njobs && (int64_t)blockIdx.x >= tab.j[jb + 1].slab0) jb++;
  const JobDesc& J = tab.j[jb];
  const int64_t slab = (int64_t)blockIdx.x - J.slab0;
  const int K = J.K;
  const int64_t n = J.n, ncols = J.ncols;
  const TIn* __restrict__ X = reinterpret_cast<const TIn*>(J.X);
  const int64_t ldx = J.ldx;
  const double* __restrict__ Lstrips = J.Lstrips;
  const double* __restrict__ LinvP = J.LinvP;
  double* __restrict__ Wslab = J.W + slab * (int64_t)K * NB * C;

  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wr = wave / WC, wc = wave % WC;
  const int64_t col_base = slab * C + wc * CW;

  for (int k = 0; k < K; k++) {
    // this block's right-hand side, loaded early (consumed after the GEMM)
    double xv[RT][CT][4];
#pragma unroll
    for (int rt = 0; rt < RT; rt++)
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
#pragma unroll
        for (int i = 0; i < 4; i++)
          xv[rt][ct][i] = load_x<TIn>(X, ldx, (int64_t)k * NB + wr * RW + rt * 16 + lane / 16 + 4 * i,
                                      col_base + ct * 16 + lane % 16, n, ncols);

    d4 acc[RT][CT];
#pragma unroll
    for (int a = 0; a < RT; a++)
#pragma unroll
      for (int b = 0; b < CT; b++) acc[a][b] = (d4){0, 0, 0, 0};

    // sum_{j<k} L_kj W_j: software pipeline with D k-step pairs in flight
    const double* __restrict__ Ls = Lstrips + strip_offset(k) + (size_t)(wr * RT) * 128 + lane * 2;
    const double* __restrict__ Wb = Wslab + (size_t)(wc * CT) * 128 + lane * 2;
    const int npairs = k * NPB;
    if (npairs > 0) {
      d2 a[D][RT], b[D][CT];
#pragma unroll
      for (int s = 0; s < D; s++) {
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
          a[s][rt] = *reinterpret_cast<const d2*>(Ls + ((size_t)s * (NB / 16) + rt) * 128);
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
          b[s][ct] = *reinterpret_cast<const d2*>(Wb + ((size_t)s * CTS + ct) * 128);
      }
      for (int kp0 = 0; kp0 < npairs; kp0 += D) {
#pragma unroll
        for (int s = 0; s < D; s++) {
#pragma unroll
          for (int rt = 0; rt < RT; rt++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++) {
              acc[rt][ct] = MFMA64(a[s][rt].x, b[s][ct].x, acc[rt][ct]);
              acc[rt][ct] = MFMA64(a[s][rt].y, b[s][ct].y, acc[rt][ct]);
            }
          // refill this stage with pair kp0 + s + D (clamped to the last
          // pair; the clamped tail loads are never used)
          int nx = kp0 + s + D;
          nx = nx < npairs ? nx : npairs - 1;
#pragma unroll
          for (int rt = 0; rt < RT; rt++)
            a[s][rt] = *reinterpret_cast<const d2*>(Ls + ((size_t)nx * (NB / 16) + rt) * 128);
#pragma unroll
          for (int ct = 0; ct < CT; ct++)
            b[s][ct] = *reinterpret_cast<const d2*>(Wb + ((size_t)nx * CTS + ct) * 128);
          // keep the refill loads issued here, D stages ahead of their use
          asm volatile("" ::: "memory");
        }
      }
    }

    // R_k = X_k - acc, staged in LDS in the B-operand pair layout
#pragma unroll
    for (int rt = 0; rt < RT; rt++) {
      const int rowl = wr * RW + rt * 16;  // row of the tile within the block
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
#pragma unroll
        for (int i = 0; i < 4; i += 2) {
          const int kp = (rowl / 4 + i) / 2;
          *reinterpret_cast<d2*>(&Rl[((size_t)kp * CTS + wc * CT + ct) * 128 + lane * 2]) =
              (d2){xv[rt][ct][i] - acc[rt][ct][i], xv[rt][ct][i + 1] - acc[rt][ct][i + 1]};
        }
      }
    }
    __syncthreads();

    // W_k = inv(L_kk) R_k ; inv(L_kk) is lower triangular, so the k-steps
    // beyond this wave's last row are zero and skipped
#pragma unroll
    for (int a = 0; a < RT; a++)
#pragma unroll
      for (int b = 0; b < CT; b++) acc[a][b] = (d4){0, 0, 0, 0};
    const double* __restrict__ Li = LinvP + (size_t)k * NB * NB + (size_t)(wr * RT) * 128 + lane * 2;
    const int kp_end = (wr * RW + RW) / 8;
    for (int kp = 0; kp < kp_end; kp++) {
      d2 a[RT], b[CT];
#pragma unroll
      for (int rt = 0; rt < RT; rt++)
        a[rt] = *reinterpret_cast<const d2*>(Li + ((size_t)kp * (NB / 16) + rt) * 128);
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
        b[ct] = *reinterpret_cast<const d2*>(&Rl[((size_t)kp * CTS + wc * CT + ct) * 128 + lane * 2]);
#pragma unroll
      for (int rt = 0; rt < RT; rt++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++) {
          acc[rt][ct] = MFMA64(a[rt].x, b[ct].x, acc[rt][ct]);
          acc[rt][ct] = MFMA64(a[rt].y, b[ct].y, acc[rt][ct]);
        }
    }
    // store W_k (slab layout): element i of the FP64 output is k-step
    // (row0/4 + i) at the same lane
#pragma unroll
    for (int rt = 0; rt < RT; rt++) {
      const int64_t ks0 = (int64_t)k * (NB / 4) + (wr * RW + rt * 16) / 4;
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
#pragma unroll
        for (int i = 0; i < 4; i += 2)
          *reinterpret_cast<d2*>(Wslab + ((size_t)((ks0 + i) / 2) * CTS + wc * CT + ct) * 128 + lane * 2) =
              (d2){acc[rt][ct][i], acc[rt][ct][i + 1]};
    }
    __threadfence_block();
    __syncthreads();
  }
}

// Address of W(row, col) in the slab layout.
__device__ __forceinline__ size_t slab_index(int64_t row, int64_t col, int C, int64_t n_pad) {
  const int64_t slab = col / C, cc = col % C;
  const int64_t ks = row / 4;
  return (size_t)slab * n_pad * C + ((size_t)(ks / 2) * (C / 16) + cc / 16) * 128 +
         (size_t)(((row % 4) * 16 + cc % 16) * 2 + (ks % 2));
}

// Slab layout -> caller's column-major array (inspection).
__global__ void k_slab_to_colmajor(const double* __restrict__ W, int C, int64_t n_pad, int64_t n,
                                   int64_t col0, int64_t ncols, double* __restrict__ out, int64_t ldo) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t c = blockIdx.y; c < ncols; c += gridDim.y) {
    if (r >= n) return;
    out[r + c * ldo] = W[slab_index(r, col0 + c, C, n_pad)];
  }
}

// ---------------------------------------------------------------------------
// a1: the fixed part F = [X_L | Y] (p_L + t <= 27 columns, once per cohort),
// row-major n_pad x w.  Triangular solves on it run right-looking with one
// launch per row block: the diagonal step on block k, then the update of
// every other affected block in parallel (one work-group per block, the
// 128 x 128 block of L staged in LDS from its contiguous packed form).
//   lower (F := L^{-1} F):  F_k = inv(L_kk) F_k;  F_j -= L_jk F_k  (j > k)
//   upper (Z := L^{-T} Z):  Z_k = inv(L_kk)^T Z_k; Z_j -= L_kj^T Z_k (j < k)

// F (row-major n_pad x w, zero padding) from the two column-major inputs.
__global__ void k_pack_fixed(const double* __restrict__ XL, int64_t ldx, const double* __restrict__ Y,
                             int64_t ldy, int64_t n, int64_t n_pad, int pL, int t,
                             double* __restrict__ F) {
  const int w = pL + t;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n_pad * w) return;
  const int64_t r = idx / w;
  const int c = (int)(idx % w);
  double v = 0.0;
  if (r < n) v = (c < pL) ? XL[r + c * ldx] : Y[r + (c - pL) * ldy];
  F[idx] = v;
}

// Unpack a 128 x 128 block stored in the fragment pair layout into T[row][col].
__device__ __forceinline__ void stage_block(double (*T)[NB + 1], const double* __restrict__ blk) {
  for (int d = threadIdx.x; d < NB * NB; d += blockDim.x) {
    const int kk = d & 1, ln = (d >> 1) & 63, rt = (d >> 7) % (NB / 16), kp = (d >> 7) / (NB / 16);
    T[rt * 16 + ln % 16][(2 * kp + kk) * 4 + ln / 16] = blk[d];
  }
}

constexpr int FIX_COLS_PER_THREAD = (MAXP + MAXT + 1) / 2;

// acc[ci] = sum_b op(T)[a][b] * F[(r0 + b) * w + c] over the thread's columns
// c = half + 2 ci, with op(T) = T (lower) or T^T (upper) and b restricted to
// the nonzero triangle when `tri` is set.
template <bool UPPER>
__device__ __forceinline__ void fix_product(const double (*T)[NB + 1], const double* __restrict__ F,
                                            int64_t r0, int w, int a, int half, bool tri,
                                            double (&acc)[FIX_COLS_PER_THREAD]) {
#pragma unroll
  for (int ci = 0; ci < FIX_COLS_PER_THREAD; ci++) acc[ci] = 0.0;
  const int b0 = (tri && UPPER) ? a : 0;
  const int b1 = (tri && !UPPER) ? a + 1 : NB;
  for (int b = b0; b < b1; b++) {
    const double tv = UPPER ? T[b][a] : T[a][b];
    const double* __restrict__ f = F + (r0 + b) * w;
#pragma unroll
    for (int ci = 0; ci < FIX_COLS_PER_THREAD; ci++) {
      const int c = half + 2 * ci;
      if (c < w) acc[ci] += tv * f[c];
    }
  }
}

template <bool UPPER>
__global__ __launch_bounds__(256) void k_fix_diag(const double* __restrict__ LinvP, int k,
                                                  double* __restrict__ F, int w) {
  __shared__ double T[NB][NB + 1];
  stage_block(T, LinvP + (size_t)k * NB * NB);
  __syncthreads();
  const int a = threadIdx.x % NB, half = threadIdx.x / NB;
  double acc[FIX_COLS_PER_THREAD];
  fix_product<UPPER>(T, F, (int64_t)k * NB, w, a, half, true, acc);
  __syncthreads();  // every read of block k happens before it is overwritten
#pragma unroll
  for (int ci = 0; ci < FIX_COLS_PER_THREAD; ci++) {
    const int c = half + 2 * ci;
    if (c < w) F[((int64_t)k * NB + a) * w + c] = acc[ci];
  }
}

template <bool UPPER>
__global__ __launch_bounds__(256) void k_fix_update(const double* __restrict__ Lstrips, int k,
                                                    double* __restrict__ F, int w) {
  __shared__ double T[NB][NB + 1];
  const int j = UPPER ? (int)blockIdx.x : k + 1 + (int)blockIdx.x;
  // lower: block L_jk (strip j, block column k); upper: block L_kj (strip k, column j)
  const double* blk = UPPER ? Lstrips + strip_offset(k) + (size_t)j * NB * NB
                            : Lstrips + strip_offset(j) + (size_t)k * NB * NB;
  stage_block(T, blk);
  __syncthreads();
  const int a = threadIdx.x % NB, half = threadIdx.x / NB;
  double acc[FIX_COLS_PER_THREAD];
  fix_product<UPPER>(T, F, (int64_t)k * NB, w, a, half, false, acc);
#pragma unroll
  for (int ci = 0; ci < FIX_COLS_PER_THREAD; ci++) {
    const int c = half + 2 * ci;
    if (c < w) F[((int64_t)j * NB + a) * w + c] -= acc[ci];
  }
}

// Row-major F -> caller's column-major array (inspection).
__global__ void k_rowmajor_to_colmajor(const double* __restrict__ F, int w, int64_t n, int col0,
                                       int ncols, double* __restrict__ out, int64_t ldo) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int c = blockIdx.y;
  if (r >= n || c >= ncols) return;
  out[r + c * ldo] = F[r * w + col0 + c];
}

// S_TL = W_L^T W_L and C_T = W_L^T ytil (syrk / gemv of Alg. 5): one
// work-group per entry (a, b) of G = F^T F, fixed-order reduction.
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ F, int64_t n, int ld,
                                              int pL, int t, double* __restrict__ STL,
                                              double* __restrict__ CT) {
  const int a = blockIdx.x, b = blockIdx.y;  // a < pL, b < pL + t
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) s += F[r * ld + a] * F[r * ld + b];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (b < pL) STL[a + b * pL] = red[0];
    else CT[a + (b - pL) * pL] = red[0];
  }
}

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
template <int ET> constexpr int as_depth() { return ET == 1 ? 4 : 3; }
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
#pragma unroll
  for (int st = 0; st < DEPTH; st++)
    if (wave + 8 * st < noct) fetch(wave + 8 * st, av[st], f0[st], f1[st]);
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
        const int64_t on = o + 8 * DEPTH;
        if (on < noct) fetch(on, av[st], f0[st], f1[st]);
      }
    }
  }
}

// Fixed-order sum over the waves of one 16-wide slice of the products:
// slice et of every tile lands in red, then dots[c][16 et + e] (e < elim)
// or, for the Gram slice (gram_pR > 0), dots[c][base + q] = G[c][c0 + q]
// for q < gram_pR, c0 the first column of c's problem in its tile.
template <int ET>
__device__ __forceinline__ void reduce_slice(const d4 (&acc)[4][ET + 1], int et, int wave, int lane,
                                             double (*red)[AS_COLS][17],
                                             double (*dots)[AS_DOTS], int elim, int base,
                                             int gram_pR) {
  const int r = lane / 16, cl = lane % 16;
#pragma unroll
  for (int ct = 0; ct < 4; ct++)
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
      for (int k = 0; k <= ET; k++)
        if (k == et) red[wave][16 * ct + r + 4 * i][cl] = acc[ct][k][i];
  __syncthreads();
  for (int idx = threadIdx.x; idx < AS_COLS * 16; idx += 64 * AS_WAVES) {
    const int c = idx / 16, e = idx % 16;
    if (gram_pR == 0) {
      if (16 * et + e < elim) {
        double v = 0.0;
        for (int w = 0; w < AS_WAVES; w++) v += red[w][c][e];
        dots[c][16 * et + e] = v;
      }
    } else if (e < gram_pR && c % 16 < 16 / gram_pR * gram_pR) {   // columns of a problem
      const int c0 = (c % 16) - (c % 16) % gram_pR;   // problem's first column in the tile
      double v = 0.0;
      for (int w = 0; w < AS_WAVES; w++) v += red[w][c][c0 + e];
      dots[c][base + e] = v;
    }
  }
  __syncthreads();
}

// REFINE = false: the FP64 path.  REFINE = true: the FP32_REFINE form; the
// whitened columns are those of the centered genotypes x' = x - s, S^(0) and
// c^(0) come from them, and one FP64 refinement step on the normal
// equations uses S' = [S_TL, E^T; E, S^(0)_BR], c' = [C_T; e_y] with
// E = x'^T Z_L and e_y = x'^T Z_y exact to FP64 rounding (Z = M^{-1}[X_L|Y]):
//   r = c' - S' b0,  d = (G G^T)^{-1} r,  b' = b0 + d,
// then b_L[icol] -= s^T b'_R undoes the centering.
template <bool REFINE, int ET>
__global__ __launch_bounds__(64 * AS_WAVES) void k_assemble_solve(const AsmTable tab) {
  __shared__ double red[AS_WAVES][AS_COLS][17];
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
  d4 acc[4][ET + 1];
  mfma_dots<ET, true>(loadA, J.F, ldf, (J.n + 7) / 8, wave, lane, acc);
#pragma unroll
  for (int et = 0; et < ET; et++) reduce_slice<ET>(acc, et, wave, lane, red, dots, ldf, 0, 0);
  reduce_slice<ET>(acc, ET, wave, lane, red, dots, 0, ldf, pR);

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
// significant bits) and (x - s)^T Z with Z = M^{-1}[X_L | Y].
// One work-group per 64 columns.  First pass: lane c sums column c over the
// row octets w, w + 8, ... of its wave (one 8-byte load when the column
// start and the leading dimension allow it, byte loads otherwise and in the
// tail).  Second pass: (x - s)^T Z as the assembly's products on FP64 MFMA,
// the A operand built from two genotype bytes per lane and tile.
__device__ __forceinline__ void xz_octet(const int8_t* __restrict__ x, int64_t o, int64_t n,
                                         bool vec, int8_t (&b)[8]) {
  const int64_t r0 = 8 * o;
  if (vec && r0 + 8 <= n) {
    const int2 v = *reinterpret_cast<const int2*>(x + r0);
    __builtin_memcpy(b, &v, 8);
  } else {
#pragma unroll
    for (int i = 0; i < 8; i++) b[i] = r0 + i < n ? x[r0 + i] : (int8_t)0;
  }
}

template <int ET>
__global__ __launch_bounds__(64 * AS_WAVES) void k_xz_shift(const XzTable tab) {
  __shared__ int isum[AS_WAVES][AS_COLS];
  __shared__ double sh[AS_COLS];
  __shared__ double red[AS_WAVES][AS_COLS][17];
  __shared__ double dots[AS_COLS][AS_DOTS];
  int jb = 0;
  while (jb + 1 < tab.njobs && (int64_t)blockIdx.x >= tab.j[jb + 1].grp0) jb++;
  const XzDesc& J = tab.j[jb];
  const int64_t col0 = ((int64_t)blockIdx.x - J.grp0) * AS_COLS;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;
  const int64_t n = J.n, noct = (n + 7) / 8;
  {
    const bool valid = col0 + lane < J.ncols;
    const int8_t* __restrict__ x = J.X + (valid ? col0 + lane : col0) * J.ldx;
    const bool vec = (reinterpret_cast<uintptr_t>(J.X) % 8 == 0) && (J.ldx % 8 == 0);
    int s = 0;
    for (int64_t o0 = wave; o0 < noct; o0 += 8 * 4) {
      int8_t b[4][8];
#pragma unroll
      for (int st = 0; st < 4; st++)
        xz_octet(x, o0 + 8 * st < noct ? o0 + 8 * st : noct, n, vec, b[st]);
#pragma unroll
      for (int st = 0; st < 4; st++)
#pragma unroll
        for (int i = 0; i < 8; i++) s += b[st][i];
    }
    isum[wave][lane] = s;
  }
  __syncthreads();
  if (threadIdx.x < AS_COLS) {
    int tot = 0;
    for (int w = 0; w < AS_WAVES; w++) tot += isum[w][threadIdx.x];
    const double shift = rint(256.0 * (double)tot / (double)n) / 256.0;
    sh[threadIdx.x] = shift;
    if (col0 + threadIdx.x < J.ncols) J.shift[col0 + threadIdx.x] = shift;
  }
  __syncthreads();
  const int r = lane / 16, cl = lane % 16;
  const int8_t* xs[4];
  double sft[4];
#pragma unroll
  for (int ct = 0; ct < 4; ct++) {
    const int64_t c = col0 + 16 * ct + cl;
    xs[ct] = J.X + (c < J.ncols ? c : col0) * J.ldx;
    sft[ct] = sh[16 * ct + cl];
  }
  auto loadA = [&](int ct, int64_t o) __attribute__((always_inline)) -> d2 {
    const int64_t r0 = 8 * o + r, r1 = r0 + 4;
    const double a0 = r0 < n ? (double)xs[ct][r0] - sft[ct] : 0.0;
    const double a1 = r1 < n ? (double)xs[ct][r1] - sft[ct] : 0.0;
    return d2{a0, a1};
  };
  const int ldf = J.ldf;
  d4 acc[4][ET + 1];
  mfma_dots<ET, false>(loadA, J.Z, ldf, noct, wave, lane, acc);
#pragma unroll
  for (int et = 0; et < ET; et++) reduce_slice<ET>(acc, et, wave, lane, red, dots, ldf, 0, 0);
  for (int idx = threadIdx.x; idx < AS_COLS * ldf; idx += 64 * AS_WAVES) {
    const int c = idx / ldf, e = idx % ldf;
    if (col0 + c < J.ncols) J.XZ[(col0 + c) * ldf + e] = dots[c][e];
  }
}

// Mixed-precision blocked lower solve W = L^{-1}(X - 1 s^T): as k_trsm, but
// each off-diagonal product L_kj W_j uses FP32-rounded operands on FP32 MFMA
// (v_mfma_f32_16x16x4f32) with FP32 accumulation over one chunk of CHQ
// k-step quads (4 k-steps each; CHQ = NB/16 is one whole diagonal block),
// and the chunk is added into an FP64 running accumulator.  The diagonal
// step inv(L_kk) R_k stays FP64.  Both W (FP64, for the assembly) and an
// FP32 copy (quad layout, for later trailing products) are stored.
// The FP32 output layout is lane l, element i -> row 4(l/16) + i.
template <int C, int WR, int WC, int D, int CHQ>
__global__ __launch_bounds__(64 * WR * WC) void k_trsm_mixed(const JobTable tab) {
  constexpr int RW = NB / WR, RT = RW / 16;
  constexpr int CW = C / WC, CT = CW / 16;
  constexpr int CTS = C / 16;
  constexpr int NQB = NB / 16;  // k-step quads per row block
  static_assert(NQB % CHQ == 0 && (CHQ % D == 0 || D % CHQ == 0), "chunking");
  __shared__ __attribute__((aligned(16))) double Rl[NB * C];

  int jb = 0;
  while (jb + 1 < tab.njobs && (int64_t)blockIdx.x >= tab.j[jb + 1].slab0) jb++;
  const JobDesc& J = tab.j[jb];
  const int64_t slab = (int64_t)blockIdx.x - J.slab0;
  const int K = J.K;
  const int64_t n = J.n, ncols = J.ncols;
  const int8_t* __restrict__ X = reinterpret_cast<const int8_t*>(J.X);
  const int64_t ldx = J.ldx;
  const double* __restrict__ shift = J.shift;
  const float* __restrict__ L32 = J.Lstrips32;
  const double* __restrict__ LinvP = J.LinvP;
  double* __restrict__ Wslab = J.W + slab * (int64_t)K * NB * C;
  float* __restrict__ W32slab = J.W32 + slab * (int64_t)K * NB * C;

  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int wr = wave / WC, wc = wave % WC;
  const int64_t col_base = slab * C + wc * CW;

  for (int k = 0; k < K; k++) {
    double xv[RT][CT][4];
#pragma unroll
    for (int rt = 0; rt < RT; rt++)
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
        const int64_t col = col_base + ct * 16 + lane % 16;
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int64_t row = (int64_t)k * NB + wr * RW + rt * 16 + 4 * (lane / 16) + i;
          xv[rt][ct][i] = (row < n && col < ncols) ? (double)X[col * ldx + row] - shift[col] : 0.0;
        }
      }

    d4 acc[RT][CT];
    f4 c32[RT][CT];
#pragma unroll
    for (int a = 0; a < RT; a++)
#pragma unroll
      for (int b = 0; b < CT; b++) {
        acc[a][b] = (d4){0, 0, 0, 0};
        c32[a][b] = (f4){0, 0, 0, 0};
      }

    const float* __restrict__ Ls = L32 + strip_offset(k) + (size_t)(wr * RT) * 256 + lane * 4;
    const float* __restrict__ Wb = W32slab + (size_t)(wc * CT) * 256 + lane * 4;
    const int nq = k * NQB;
    if (nq > 0) {
      f4 a[D][RT], b[D][CT];
#pragma unroll
      for (int s = 0; s < D; s++) {
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
          a[s][rt] = *reinterpret_cast<const f4*>(Ls + ((size_t)s * (NB / 16) + rt) * 256);
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
          b[s][ct] = *reinterpret_cast<const f4*>(Wb + ((size_t)s * CTS + ct) * 256);
      }
      for (int q0 = 0; q0 < nq; q0 += D) {
#pragma unroll
        for (int s = 0; s < D; s++) {
#pragma unroll
          for (int rt = 0; rt < RT; rt++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++) {
              c32[rt][ct] = MFMA32(a[s][rt].x, b[s][ct].x, c32[rt][ct]);
              c32[rt][ct] = MFMA32(a[s][rt].y, b[s][ct].y, c32[rt][ct]);
              c32[rt][ct] = MFMA32(a[s][rt].z, b[s][ct].z, c32[rt][ct]);
              c32[rt][ct] = MFMA32(a[s][rt].w, b[s][ct].w, c32[rt][ct]);
            }
          int nx = q0 + s + D;
          nx = nx < nq ? nx : nq - 1;
#pragma unroll
          for (int rt = 0; rt < RT; rt++)
            a[s][rt] = *reinterpret_cast<const f4*>(Ls + ((size_t)nx * (NB / 16) + rt) * 256);
#pragma unroll
          for (int ct = 0; ct < CT; ct++)
            b[s][ct] = *reinterpret_cast<const f4*>(Wb + ((size_t)nx * CTS + ct) * 256);
          asm volatile("" ::: "memory");
          if (CHQ <= D && (s + 1) % CHQ == 0) {
            // end of an FP32 chunk: fold into the FP64 running sum
#pragma unroll
            for (int rt = 0; rt < RT; rt++)
#pragma unroll
              for (int ct = 0; ct < CT; ct++) {
#pragma unroll
                for (int i = 0; i < 4; i++) acc[rt][ct][i] += (double)c32[rt][ct][i];
                c32[rt][ct] = (f4){0, 0, 0, 0};
              }
          }
        }
        if (CHQ > D && (q0 + D) % CHQ == 0) {
#pragma unroll
          for (int rt = 0; rt < RT; rt++)
#pragma unroll
            for (int ct = 0; ct < CT; ct++) {
#pragma unroll
              for (int i = 0; i < 4; i++) acc[rt][ct][i] += (double)c32[rt][ct][i];
              c32[rt][ct] = (f4){0, 0, 0, 0};
            }
        }
      }
    }

    // R_k = (x - s) - acc, to LDS in the FP64 B-operand pair layout: element
    // (row 4g + i) of the FP32 output goes to k-step (row0/4 + g), lane 16i + l%16
#pragma unroll
    for (int rt = 0; rt < RT; rt++) {
      const int rowl = wr * RW + rt * 16;
      const int ks = rowl / 4 + lane / 16;
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
#pragma unroll
        for (int i = 0; i < 4; i++)
          Rl[((size_t)(ks / 2) * CTS + wc * CT + ct) * 128 + (i * 16 + lane % 16) * 2 + (ks % 2)] =
              xv[rt][ct][i] - acc[rt][ct][i];
    }
    __syncthreads();

    d4 w64[RT][CT];
#pragma unroll
    for (int a = 0; a < RT; a++)
#pragma unroll
      for (int b = 0; b < CT; b++) w64[a][b] = (d4){0, 0, 0, 0};
    const double* __restrict__ Li = LinvP + (size_t)k * NB * NB + (size_t)(wr * RT) * 128 + lane * 2;
    const int kp_end = (wr * RW + RW) / 8;
    for (int kp = 0; kp < kp_end; kp++) {
      d2 a[RT], b[CT];
#pragma unroll
      for (int rt = 0; rt < RT; rt++)
        a[rt] = *reinterpret_cast<const d2*>(Li + ((size_t)kp * (NB / 16) + rt) * 128);
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
        b[ct] = *reinterpret_cast<const d2*>(&Rl[((size_t)kp * CTS + wc * CT + ct) * 128 + lane * 2]);
#pragma unroll
      for (int rt = 0; rt < RT; rt++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++) {
          w64[rt][ct] = MFMA64(a[rt].x, b[ct].x, w64[rt][ct]);
          w64[rt][ct] = MFMA64(a[rt].y, b[ct].y, w64[rt][ct]);
        }
    }
    // store W_k: FP64 pairs (identity per lane) and the FP32 quad copy
    // (element i of the FP64 output is k-step row0/4 + i, i.e. position i of
    // quad row0/16, same lane)
#pragma unroll
    for (int rt = 0; rt < RT; rt++) {
      const int64_t row0 = (int64_t)k * NB + wr * RW + rt * 16;
      const int64_t ks0 = row0 / 4;
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
#pragma unroll
        for (int i = 0; i < 4; i += 2)
          *reinterpret_cast<d2*>(Wslab + ((size_t)((ks0 + i) / 2) * CTS + wc * CT + ct) * 128 + lane * 2) =
              (d2){w64[rt][ct][i], w64[rt][ct][i + 1]};
        *reinterpret_cast<f4*>(W32slab + ((size_t)(row0 / 16) * CTS + wc * CT + ct) * 256 + lane * 4) =
            (f4){(float)w64[rt][ct][0], (float)w64[rt][ct][1], (float)w64[rt][ct][2],
                 (float)w64[rt][ct][3]};
      }
    }
    __threadfence_block();
    __syncthreads();
  }
}

}  // namespace gls

// ---------------------------------------------------------------------------
// launchers (host side, used by gls_api.cpp)
namespace gls {

hipError_t launch_factor(const double* M, int64_t ldm, int64_t n, int64_t n_pad, int K,
                         double* A, double* Ldiag, double* Linv, double* Lstrips, double* LinvP,
                         float* Lstrips32, int* dinfo, hipStream_t st) {
  {
    dim3 grid((unsigned)((n_pad + 255) / 256), (unsigned)(n_pad < 65535 ? n_pad : 65535));
    k_copy_pad<<<grid, 256, 0, st>>>(M, ldm, n, A, n_pad);
  }
  for (int k = 0; k < K; k++) {
    k_potf2_inv<<<1, 256, 0, st>>>(A, n_pad, k, n, Ldiag, Linv, dinfo);
    if (k + 1 < K) {
      k_panel<<<K - 1 - k, 256, 0, st>>>(A, n_pad, k, Linv, dinfo);
      const int64_t d = K - 1 - k;
      k_syrk<<<(unsigned)(d * (d + 1) / 2), 256, 0, st>>>(A, n_pad, k, K, dinfo);
    }
  }
  const int64_t nblk = (int64_t)K * (K + 1) / 2;
  k_pack<<<(unsigned)nblk, 256, 0, st>>>(A, n_pad, Linv, Lstrips, LinvP, Lstrips32, K);
  return hipGetLastError();
}

hipError_t launch_unpack_factor(const double* Lstrips, const double* Ldiag, int64_t n, double* L,
                                int64_t ldl, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)(n < 65535 ? n : 65535));
  k_unpack_factor<<<grid, 256, 0, st>>>(Lstrips, Ldiag, n, L, ldl);
  return hipGetLastError();
}

hipError_t launch_trsm_i8(const JobTable& tab, int64_t nslabs, int C, hipStream_t st) {
  switch (C) {
    case 16: k_trsm<16, 4, 1, TRSM_DEPTH, int8_t><<<(unsigned)nslabs, 256, 0, st>>>(tab); break;
    case 32: k_trsm<32, 4, 2, TRSM_DEPTH, int8_t><<<(unsigned)nslabs, 512, 0, st>>>(tab); break;
    case 64: k_trsm<64, 4, 2, TRSM_DEPTH, int8_t><<<(unsigned)nslabs, 512, 0, st>>>(tab); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fixed_solve(const double* XL, int64_t ldx, const double* Y, int64_t ldy,
                              int64_t n, int64_t n_pad, int K, int pL, int t, const double* Lstrips,
                              const double* LinvP, double* F, double* Z, hipStream_t st) {
  const int w = pL + t;
  const int64_t total = n_pad * w;
  k_pack_fixed<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(XL, ldx, Y, ldy, n, n_pad, pL, t, F);
  for (int k = 0; k < K; k++) {
    k_fix_diag<false><<<1, 256, 0, st>>>(LinvP, k, F, w);
    if (k + 1 < K) k_fix_update<false><<<K - 1 - k, 256, 0, st>>>(Lstrips, k, F, w);
  }
  if (Z) {
    hipError_t e = hipMemcpyAsync(Z, F, sizeof(double) * total, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    for (int k = K - 1; k >= 0; k--) {
      k_fix_diag<true><<<1, 256, 0, st>>>(LinvP, k, Z, w);
      if (k > 0) k_fix_update<true><<<k, 256, 0, st>>>(Lstrips, k, Z, w);
    }
  }
  return hipGetLastError();
}

hipError_t launch_rowmajor_to_colmajor(const double* F, int w, int64_t n, int col0, int ncols,
                                       double* out, int64_t ldo, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)ncols);
  k_rowmajor_to_colmajor<<<grid, 256, 0, st>>>(F, w, n, col0, ncols, out, ldo);
  return hipGetLastError();
}

hipError_t launch_slab_to_colmajor(const double* W, int C, int64_t n_pad, int64_t n, int64_t col0,
                                   int64_t ncols, double* out, int64_t ldo, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)(ncols < 65535 ? ncols : 65535));
  k_slab_to_colmajor<<<grid, 256, 0, st>>>(W, C, n_pad, n, col0, ncols, out, ldo);
  return hipGetLastError();
}

hipError_t launch_gram(const double* F, int64_t n, int pL, int t, double* STL, double* CT,
                       hipStream_t st) {
  dim3 grid((unsigned)pL, (unsigned)(pL + t));
  k_gram<<<grid, 256, 0, st>>>(F, n, pL + t, pL, t, STL, CT);
  return hipGetLastError();
}

hipError_t launch_assemble_solve(const AsmTable& tab, int64_t ngroups, bool refine, hipStream_t st) {
  int w = 1;  // widest F = [W_L | ytil] of the table: one or two 16-column tiles
  for (int i = 0; i < tab.njobs; i++) w = std::max(w, tab.j[i].pL + tab.j[i].t);
  const unsigned g = (unsigned)ngroups, nt = 64 * AS_WAVES;
  if (w <= 16) {
    if (refine) k_assemble_solve<true, 1><<<g, nt, 0, st>>>(tab);
    else k_assemble_solve<false, 1><<<g, nt, 0, st>>>(tab);
  } else {
    if (refine) k_assemble_solve<true, 2><<<g, nt, 0, st>>>(tab);
    else k_assemble_solve<false, 2><<<g, nt, 0, st>>>(tab);
  }
  return hipGetLastError();
}

hipError_t launch_trsm_mixed(const JobTable& tab, int64_t nslabs, int C, hipStream_t st) {
  switch (C) {
    case 32: k_trsm_mixed<32, 4, 2, 4, FP32_CHUNK_QUADS><<<(unsigned)nslabs, 512, 0, st>>>(tab); break;
    case 64: k_trsm_mixed<64, 4, 2, 4, FP32_CHUNK_QUADS><<<(unsigned)nslabs, 512, 0, st>>>(tab); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_xz_shift(const XzTable& tab, int64_t ngroups, hipStream_t st) {
  int w = 1;
  for (int i = 0; i < tab.njobs; i++) w = std::max(w, tab.j[i].ldf);
  const unsigned g = (unsigned)ngroups, nt = 64 * AS_WAVES;
  if (w <= 16) k_xz_shift<1><<<g, nt, 0, st>>>(tab);
  else k_xz_shift<2><<<g, nt, 0, st>>>(tab);
  return hipGetLastError();
}

}  // namespace gls
