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

// One step of the solve in a single launch: every work-group updates its
// block j with block k (lower: F_j -= L_jk F_k, j > k; upper:
// Z_j -= L_kj^T Z_k, j < k; the 128 x 128 block of L staged in LDS from its
// contiguous packed form), and the one whose block is the
// next to be finished (j = k + 1 for the lower solve, j = k - 1 for the
// upper one) then applies that block's diagonal step (as k_fix_diag), so
// that the next launch can use it.  K - 1 launches instead of 2K - 1.
template <bool UPPER>
__global__ __launch_bounds__(256) void k_fix_step(const double* __restrict__ Lstrips,
                                                  const double* __restrict__ LinvP, int k,
                                                  double* __restrict__ F, int w) {
  __shared__ double T[NB][NB + 1];
  const int j = UPPER ? (int)blockIdx.x : k + 1 + (int)blockIdx.x;
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
  if (j != (UPPER ? k - 1 : k + 1)) return;
  // block j is now final but for its diagonal step: every thread's update is
  // visible to the work-group, and T is free, after the barrier
  __syncthreads();
  stage_block(T, LinvP + (size_t)j * NB * NB);
  __syncthreads();
  fix_product<UPPER>(T, F, (int64_t)j * NB, w, a, half, true, acc);
  __syncthreads();  // every read of block j happens before it is overwritten
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
