// Device-side helpers and data layouts shared by the solver's kernels
// (gfx950 / CDNA4).
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
#pragma once
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

// Address of W(row, col) in the slab layout.
__device__ __forceinline__ size_t slab_index(int64_t row, int64_t col, int C, int64_t n_pad) {
  const int64_t slab = col / C, cc = col % C;
  const int64_t ks = row / 4;
  return (size_t)slab * n_pad * C + ((size_t)(ks / 2) * (C / 16) + cc / 16) * 128 +
         (size_t)(((row % 4) * 16 + cc % 16) * 2 + (ks % 2));
}


// s_waitcnt vmcnt(N) lgkmcnt(0) (gfx9 encoding; expcnt left free)
template <int N>
__device__ __forceinline__ void wait_vm_lgkm0() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | ((N >> 4) << 14));
}

// s_waitcnt lgkmcnt(0) alone (vmcnt and expcnt left free)
__device__ __forceinline__ void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(15 | (7 << 4) | (3 << 14)); }

// Barrier without a memory fence (the caller has waited for what it needs);
// the compiler may move no memory access across it.
__device__ __forceinline__ void barrier_only() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// One 1 KB chunk (64 lanes x 16 bytes) from global memory straight into LDS
// at dst + 16 bytes * lane (global_load_lds_dwordx4; dst is wave-uniform).
// Completion is counted by vmcnt.
__device__ __forceinline__ void chunk_to_lds(const void* src, void* dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

template <typename TIn>
__device__ __forceinline__ double load_x(const TIn* __restrict__ X, int64_t ldx, int64_t row,
                                         int64_t col, int64_t n, int64_t ncols) {
  return (row < n && col < ncols) ? (double)X[col * ldx + row] : 0.0;
}

// The diagonal step W_k = inv(L_kk) R_k of the 128-row solves (four wave
// rows of two 16-row tiles), with R_k in LDS in the B-operand pair layout
// and the row tiles dealt for balance:
// 16-row tile t of inv(L_kk) R_k needs the first 2(t+1) k-step pairs (the
// rest of its row of inv(L_kk) is zero), so wave row W takes tiles W and
// NB/16 - 1 - W: NB/8 + 2 = 18 steps for every wave row (against up to
// 2 NB/8 for wave row WR - 1 when it holds the last two tiles).  Same
// products in the same order per element as diag_step.
//
// The wave row is a template parameter (the caller switches on it), so the
// 18 steps unroll with static registers: the inv(L_kk) fragments are loaded
// DIAG_PF steps ahead (the first ones by diag_prefetch, before R_k is
// staged) and the R_k fragments one step ahead, and no step waits for a
// load it has just issued (with a run-time trip count every step waited
// for its own inv(L_kk) load from L2 and its LDS reads).
constexpr int DIAG_PF = 4;

template <int W>
__device__ __forceinline__ const double* diag_a_ptr(const double* __restrict__ Li, int s) {
  constexpr int NT = NB / 16, NA = 2 * (W + 1);
  return s < NA ? Li + ((size_t)s * NT + W) * 128 : Li + ((size_t)(s - NA) * NT + (NT - 1 - W)) * 128;
}

template <int W>
__device__ __forceinline__ void diag_prefetch(const double* __restrict__ LinvP, int k, int lane, d2 (&pa)[DIAG_PF]) {
  const double* __restrict__ Li = LinvP + (size_t)k * NB * NB + lane * 2;
#pragma unroll
  for (int s = 0; s < DIAG_PF; s++) pa[s] = *reinterpret_cast<const d2*>(diag_a_ptr<W>(Li, s));
}

template <int CT, int CTS, int W>
__device__ __forceinline__ void diag_step_dealt(const double* __restrict__ LinvP, int k,
                                                const double* Rl, int wc_tile, int lane,
                                                const d2 (&pa)[DIAG_PF], d4 (&w)[2][CT]) {
  constexpr int NT = NB / 16, NA = 2 * (W + 1), NS = NA + 2 * (NT - W);
  static_assert(NS > DIAG_PF, "prefetch depth");
  const double* __restrict__ Li = LinvP + (size_t)k * NB * NB + lane * 2;
  auto read_b = [&](int s, d2 (&b)[CT]) {
    const int kp = s < NA ? s : s - NA;
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
      b[ct] = *reinterpret_cast<const d2*>(&Rl[((size_t)kp * CTS + wc_tile + ct) * 128 + lane * 2]);
  };
  d2 a[NS], b[2][CT];
#pragma unroll
  for (int s = 0; s < DIAG_PF; s++) a[s] = pa[s];
#pragma unroll
  for (int h = 0; h < 2; h++)
#pragma unroll
    for (int ct = 0; ct < CT; ct++) w[h][ct] = (d4){0, 0, 0, 0};
  read_b(0, b[0]);
#pragma unroll
  for (int s = 0; s < NS; s++) {
    if (s + DIAG_PF < NS) a[s + DIAG_PF] = *reinterpret_cast<const d2*>(diag_a_ptr<W>(Li, s + DIAG_PF));
    if (s + 1 < NS) read_b(s + 1, b[(s + 1) % 2]);
    const int h = s < NA ? 0 : 1;
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      w[h][ct] = MFMA64(a[s].x, b[s % 2][ct].x, w[h][ct]);
      w[h][ct] = MFMA64(a[s].y, b[s % 2][ct].y, w[h][ct]);
    }
    // the loads first, then the MFMAs (left alone, the scheduler sinks the
    // loads below the MFMAs to shorten their registers' lives, and every
    // step then waits for its own reads)
    if (s + DIAG_PF < NS) __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
    if (s + 1 < NS) __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, 2 * CT, 0);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Runs STMT with the constant WROW = this wave's row (wave-uniform: a
// scalar branch, no divergence).
#define DIAG_BY_ROW(STMT)                        \
  do {                                           \
    switch (wr) {                                \
      case 0: { constexpr int WROW = 0; STMT; } break; \
      case 1: { constexpr int WROW = 1; STMT; } break; \
      case 2: { constexpr int WROW = 2; STMT; } break; \
      default: { constexpr int WROW = 3; STMT; } break; \
    }                                            \
  } while (0)

}  // namespace gls
