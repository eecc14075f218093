// Whitening of the fixed part [X_L | Y] and its Gram blocks (a1).
#include "gls_device.h"

namespace gls {

// ---------------------------------------------------------------------------
// a1: the fixed part F = [X_L | Y] (p_L + t <= 27 columns, once per cohort),
// row-major n_pad x w.  Triangular solves on it run right-looking with one
// launch per row block: the update of every affected block with block k in
// parallel (one work-group per block), the next block's diagonal step done
// by its own work-group at the end of the same launch.
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

// Unpack a 128 x 128 block stored in the fragment pair layout into T[row][col]
// (256 threads).  Pair q of the block (16 bytes: k-steps 2 kp and 2 kp + 1 of
// lane ln of row tile rt) goes to two entries of T.  Each thread issues its
// loads in batches of 16 before storing any, so that the batch's latencies
// overlap.
__device__ __forceinline__ void stage_block(double (*T)[NB + 1], const double* __restrict__ blk) {
  constexpr int PAIRS = NB * NB / 2, PER = PAIRS / 256, BATCH = 16;
  static_assert(PER % BATCH == 0, "whole batches");
  const d2* __restrict__ src = reinterpret_cast<const d2*>(blk);
#pragma unroll
  for (int b0 = 0; b0 < PER; b0 += BATCH) {
    d2 v[BATCH];
#pragma unroll
    for (int i = 0; i < BATCH; i++) v[i] = src[threadIdx.x + 256 * (b0 + i)];
#pragma unroll
    for (int i = 0; i < BATCH; i++) {
      const int q = threadIdx.x + 256 * (b0 + i);
      const int ln = q & 63, rt = (q >> 6) % (NB / 16), kp = (q >> 6) / (NB / 16);
      T[rt * 16 + ln % 16][(2 * kp) * 4 + ln / 16] = v[i].x;
      T[rt * 16 + ln % 16][(2 * kp + 1) * 4 + ln / 16] = v[i].y;
    }
  }
}

constexpr int FIX_COLS_PER_THREAD = (MAXP + MAXT + 1) / 2;
constexpr int FIX_LD = MAXP + MAXT;  // row stride of a staged block of F

// Rows r0 .. r0 + NB - 1 of F (row-major, w columns: one contiguous run)
// into Fs[row][col].
__device__ __forceinline__ void stage_rows(double (*Fs)[FIX_LD], const double* __restrict__ F, int64_t r0,
                                           int w) {
  const double* __restrict__ src = F + r0 * w;
  for (int d = threadIdx.x; d < NB * w; d += blockDim.x) Fs[d / w][d % w] = src[d];
}

// acc[ci] = sum_b op(T)[a][b] * Fs[b][c] over the thread's columns
// c = half + 2 ci, with op(T) = T (lower) or T^T (upper) and b restricted to
// the nonzero triangle when `tri` is set.  Both operands are in LDS.
template <bool UPPER>
__device__ __forceinline__ void fix_product(const double (*T)[NB + 1], const double (*Fs)[FIX_LD], int w, int a,
                                            int half, bool tri, double (&acc)[FIX_COLS_PER_THREAD]) {
#pragma unroll
  for (int ci = 0; ci < FIX_COLS_PER_THREAD; ci++) acc[ci] = 0.0;
  const int b0 = (tri && UPPER) ? a : 0;
  const int b1 = (tri && !UPPER) ? a + 1 : NB;
  for (int b = b0; b < b1; b++) {
    const double tv = UPPER ? T[b][a] : T[a][b];
#pragma unroll
    for (int ci = 0; ci < FIX_COLS_PER_THREAD; ci++) {
      const int c = half + 2 * ci;
      if (c < w) acc[ci] += tv * Fs[b][c];
    }
  }
}

template <bool UPPER>
__global__ __launch_bounds__(256) void k_fix_diag(const double* __restrict__ LinvP, int k,
                                                  double* __restrict__ F, int w) {
  __shared__ double T[NB][NB + 1];
  __shared__ double Fs[NB][FIX_LD];
  stage_block(T, LinvP + (size_t)k * NB * NB);
  stage_rows(Fs, F, (int64_t)k * NB, w);
  __syncthreads();
  const int a = threadIdx.x % NB, half = threadIdx.x / NB;
  double acc[FIX_COLS_PER_THREAD];
  fix_product<UPPER>(T, Fs, w, a, half, true, acc);
#pragma unroll
  for (int ci = 0; ci < FIX_COLS_PER_THREAD; ci++) {
    const int c = half + 2 * ci;
    if (c < w) F[((int64_t)k * NB + a) * w + c] = acc[ci];
  }
}

// One step of the solve in a single launch: every work-group updates its
// block j with block k (lower: F_j -= L_jk F_k, j > k; upper:
// Z_j -= L_kj^T Z_k, j < k; the 128 x 128 block of L staged in LDS from its
// contiguous packed form, block k of F beside it), and the one whose block
// is the next to be finished (j = k + 1 for the lower solve, j = k - 1 for
// the upper one) then applies that block's diagonal step (as k_fix_diag),
// so that the next launch can use it.  K - 1 launches instead of 2K - 1.
template <bool UPPER>
__global__ __launch_bounds__(256) void k_fix_step(const double* __restrict__ Lstrips,
                                                  const double* __restrict__ LinvP, int k,
                                                  double* __restrict__ F, int w) {
  __shared__ double T[NB][NB + 1];
  __shared__ double Fs[NB][FIX_LD];
  const int j = UPPER ? (int)blockIdx.x : k + 1 + (int)blockIdx.x;
  const double* blk = UPPER ? Lstrips + strip_offset(k) + (size_t)j * NB * NB
                            : Lstrips + strip_offset(j) + (size_t)k * NB * NB;
  stage_block(T, blk);
  stage_rows(Fs, F, (int64_t)k * NB, w);
  __syncthreads();
  const int a = threadIdx.x % NB, half = threadIdx.x / NB;
  double acc[FIX_COLS_PER_THREAD], v[FIX_COLS_PER_THREAD];
  fix_product<UPPER>(T, Fs, w, a, half, false, acc);
#pragma unroll
  for (int ci = 0; ci < FIX_COLS_PER_THREAD; ci++) {
    const int c = half + 2 * ci;
    v[ci] = 0.0;
    if (c < w) {
      v[ci] = F[((int64_t)j * NB + a) * w + c] - acc[ci];
      F[((int64_t)j * NB + a) * w + c] = v[ci];
    }
  }
  if (j != (UPPER ? k - 1 : k + 1)) return;
  // block j is now final but for its diagonal step; once every thread is
  // done reading T and block k, they take inv(L_jj) and block j
  __syncthreads();
  stage_block(T, LinvP + (size_t)j * NB * NB);
#pragma unroll
  for (int ci = 0; ci < FIX_COLS_PER_THREAD; ci++) {
    const int c = half + 2 * ci;
    if (c < w) Fs[a][c] = v[ci];
  }
  __syncthreads();
  fix_product<UPPER>(T, Fs, w, a, half, true, acc);
#pragma unroll
  for (int ci = 0; ci < FIX_COLS_PER_THREAD; ci++) {
    const int c = half + 2 * ci;
    if (c < w) F[((int64_t)j * NB + a) * w + c] = acc[ci];
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


hipError_t launch_fixed_solve(const double* XL, int64_t ldx, const double* Y, int64_t ldy,
                              int64_t n, int64_t n_pad, int K, int pL, int t, const double* Lstrips,
                              const double* LinvP, double* F, double* Z, hipStream_t st) {
  const int w = pL + t;
  const int64_t total = n_pad * w;
  k_pack_fixed<<<(unsigned)((total + 255) / 256), 256, 0, st>>>(XL, ldx, Y, ldy, n, n_pad, pL, t, F);
  k_fix_diag<false><<<1, 256, 0, st>>>(LinvP, 0, F, w);
  for (int k = 0; k + 1 < K; k++) k_fix_step<false><<<K - 1 - k, 256, 0, st>>>(Lstrips, LinvP, k, F, w);
  if (Z) {
    hipError_t e = hipMemcpyAsync(Z, F, sizeof(double) * total, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
    k_fix_diag<true><<<1, 256, 0, st>>>(LinvP, K - 1, Z, w);
    for (int k = K - 1; k > 0; k--) k_fix_step<true><<<k, 256, 0, st>>>(Lstrips, LinvP, k, Z, w);
  }
  return hipGetLastError();
}

hipError_t launch_rowmajor_to_colmajor(const double* F, int w, int64_t n, int col0, int ncols,
                                       double* out, int64_t ldo, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)ncols);
  k_rowmajor_to_colmajor<<<grid, 256, 0, st>>>(F, w, n, col0, ncols, out, ldo);
  return hipGetLastError();
}

hipError_t launch_gram(const double* F, int64_t n, int pL, int t, double* STL, double* CT,
                       hipStream_t st) {
  dim3 grid((unsigned)pL, (unsigned)(pL + t));
  k_gram<<<grid, 256, 0, st>>>(F, n, pL + t, pL, t, STL, CT);
  return hipGetLastError();
}

}  // namespace gls
