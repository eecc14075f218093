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

// Unblocked Cholesky of the diagonal block k, then its inverse, with the
// block held in registers: thread t owns rows r + 16a and columns c + 16b
// (r = t % 16, c = t / 16, a, b < 8) of the 128 x 128 block.
//   factor, step j:  the owners of column j publish it (LDS, double
//     buffered), every thread forms L[.][j] = A[.][j] / sqrt(A[j][j]) for
//     the rows and columns it owns (reciprocal multiply, as LAPACK's
//     unblocked potf2) and applies the rank-1 update to its trailing part;
//   inverse, step j (X = inv(L) by row elimination of L X = I): the owners
//     of row j scale it by 1 / L[j][j] and publish it; every thread subtracts
//     L[i][j] X[j][.] from its rows i > j.
// The steps run in 8 groups of 16 (template parameter JB = j / 16), so each
// group touches only the register tiles it can change, with static indices.
// One barrier per step.  Writes L_kk into A and into Ldiag[k], inv(L_kk)
// into Linv[k] (NB x NB column-major, lower).  A non-positive or non-finite
// pivot of a real row sets *info (order of the failing leading minor) and
// stops the process: every later kernel sees *info != 0 and returns at once.
__device__ __forceinline__ int tri_off(int j) { return j * NB - j * (j - 1) / 2; }

struct Potf2Ctx {
  double (*buf)[NB];   // LDS, two buffers of one column or row
  double* Lp;          // LDS, L by columns, lower triangle packed
  int r, c, t;
  int64_t o, n;
  int fail;
};

template <int JB>
__device__ __forceinline__ bool potf2_group(double (&T)[8][8], Potf2Ctx& x) {
  const int r = x.r, c = x.c;
#pragma unroll 1
  for (int jj = 0; jj < 16; jj++) {
    const int j = 16 * JB + jj;
    double* col = x.buf[j & 1];
    if (c == jj) {
#pragma unroll
      for (int a = JB; a < 8; a++)
        if (a > JB || r >= jj) col[r + 16 * a] = T[a][JB];
    }
    __syncthreads();
    const double d = col[j];
    if (!(d > 0.0) || !(d < INFINITY)) {
      x.fail = (x.o + j < x.n) ? (int)(x.o + j + 1) : -1;
      return false;
    }
    const double g = sqrt(d), rg = 1.0 / g;
    double li[8], ll[8];   // L[i][j] of the owned rows, L[l][j] of the owned columns (0 if <= j)
#pragma unroll
    for (int a = JB; a < 8; a++) li[a] = (a > JB || r > jj) ? col[r + 16 * a] * rg : 0.0;
#pragma unroll
    for (int b = JB; b < 8; b++) ll[b] = (b > JB || c > jj) ? col[c + 16 * b] * rg : 0.0;
    if (x.t < NB && x.t >= j) x.Lp[tri_off(j) + x.t - j] = x.t == j ? g : col[x.t] * rg;
    if (c == jj) {
#pragma unroll
      for (int a = JB; a < 8; a++) {
        if (a == JB && r == jj) T[a][JB] = g;
        else if (a > JB || r > jj) T[a][JB] = li[a];
      }
    }
    // rank-1 update of the trailing tiles (a >= b >= JB); li, ll vanish
    // outside rows and columns > j, and the strict upper part is not used
#pragma unroll
    for (int b = JB; b < 8; b++)
#pragma unroll
      for (int a = b; a < 8; a++) T[a][b] -= li[a] * ll[b];
  }
  return true;
}

template <int JB>
__device__ __forceinline__ void trtri_group(double (&T)[8][8], Potf2Ctx& x) {
  const int r = x.r, c = x.c;
#pragma unroll 1
  for (int jj = 0; jj < 16; jj++) {
    const int j = 16 * JB + jj;
    double* row = x.buf[j & 1];
    const double djj = 1.0 / x.Lp[tri_off(j)];
    if (r == jj) {
#pragma unroll
      for (int b = 0; b <= JB; b++) {
        if (b < JB || c <= jj) {
          T[JB][b] *= djj;
          row[c + 16 * b] = T[JB][b];
        }
      }
    }
    __syncthreads();
    double li[8], xj[8];
#pragma unroll
    for (int a = JB; a < 8; a++)
      li[a] = (a > JB || r > jj) ? x.Lp[tri_off(j) + r + 16 * a - j] : 0.0;
#pragma unroll
    for (int b = 0; b <= JB; b++) xj[b] = (b < JB || c <= jj) ? row[c + 16 * b] : 0.0;
#pragma unroll
    for (int a = JB; a < 8; a++)
#pragma unroll
      for (int b = 0; b <= JB; b++) T[a][b] -= li[a] * xj[b];
  }
}

template <int... JB>
__device__ __forceinline__ bool potf2_all(double (&T)[8][8], Potf2Ctx& x,
                                          std::integer_sequence<int, JB...>) {
  return (potf2_group<JB>(T, x) && ...);
}

template <int... JB>
__device__ __forceinline__ void trtri_all(double (&T)[8][8], Potf2Ctx& x,
                                          std::integer_sequence<int, JB...>) {
  (trtri_group<JB>(T, x), ...);
}

__global__ __launch_bounds__(256) void k_potf2_inv(double* __restrict__ A, int64_t lda,
                                                    int k, int64_t n,
                                                    double* __restrict__ Ldiag,
                                                    double* __restrict__ Linv,
                                                    int* __restrict__ info) {
  static_assert(NB == 128, "8 x 8 register tiles of 16");
  __shared__ double buf[2][NB];
  __shared__ double Lp[NB * (NB + 1) / 2];
  if (*info != 0) return;
  Potf2Ctx x;
  x.buf = buf;
  x.Lp = Lp;
  x.t = threadIdx.x;
  x.r = x.t % 16;
  x.c = x.t / 16;
  x.o = (int64_t)k * NB;
  x.n = n;
  x.fail = 0;
  const int r = x.r, c = x.c;
  const int64_t o = x.o;
  double T[8][8];
#pragma unroll
  for (int b = 0; b < 8; b++)
#pragma unroll
    for (int a = 0; a < 8; a++) {
      const int i = r + 16 * a, l = c + 16 * b;
      T[a][b] = i >= l ? A[(o + i) + (o + l) * lda] : 0.0;
    }
  if (!potf2_all(T, x, std::make_integer_sequence<int, 8>{})) {
    if (x.t == 0) *info = x.fail > 0 ? x.fail : (int)(o + 1);
    return;
  }
#pragma unroll
  for (int b = 0; b < 8; b++)
#pragma unroll
    for (int a = 0; a < 8; a++) {
      const int i = r + 16 * a, l = c + 16 * b;
      const double v = i >= l ? T[a][b] : 0.0;
      A[(o + i) + (o + l) * lda] = v;
      Ldiag[(size_t)k * NB * NB + i + (size_t)l * NB] = v;
      T[a][b] = i == l ? 1.0 : 0.0;   // T becomes X, starting from the identity
    }
  __syncthreads();   // Lp complete, the buffers free
  trtri_all(T, x, std::make_integer_sequence<int, 8>{});
#pragma unroll
  for (int b = 0; b < 8; b++)
#pragma unroll
    for (int a = 0; a < 8; a++) {
      const int i = r + 16 * a, l = c + 16 * b;
      Linv[(size_t)k * NB * NB + i + (size_t)l * NB] = i >= l ? T[a][b] : 0.0;
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
