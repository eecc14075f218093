// Mixed-precision triangular solve of the FP32_REFINE form (a5).
#include "gls_device.h"

namespace gls {

// True when the last row block's real rows (n - (K-1) NB of them) all lie in
// the first of the wave rows' tiles (RW rows); k_trsm_mixed_last then
// solves that block.
__host__ __device__ inline bool mixed_last_block_split(int64_t n, int K, int RW) {
  return K > 1 && n - (int64_t)(K - 1) * NB <= RW;
}

// The off-diagonal sum acc = sum_{j<k} L_kj W_j of the mixed solve for one
// row block, with the operands staged through LDS: a stage is two k-step
// quads, i.e. 2 (NB/16 + C/16) chunks of 1 KB (the L32 strip tiles of all
// NB rows and the W32 tiles of all C columns), copied by the work-group's
// waves straight into one of S LDS slots, S - 1 stages ahead.  Every wave
// then reads its own tiles from LDS: each operand byte crosses the L1 cache
// once per work-group, and the stages in flight cost no registers.  As in
// the FP64 solve, the barrier sits in the middle of a stage: a wave reads
// the second quad of stage st, runs the first quad, waits for its own
// copies of stage st+1 and for its LDS reads, passes the barrier (stage st+1
// visible to all, stage st read by all), refills stage st's slot with stage
// st+S, reads the first quad of stage st+1 and runs the second quad of
// stage st.  The two quads of a stage form one chunk of the FP64 running
// sum (quad_chain_fold), as two consecutive quads do in the register-ring form.
template <int C, int G>
constexpr int staged_ring_floats(int S) { return S * G * (NB / 16 + C / 16) * 256; }

// One k-step quad of FP32 MFMAs for every tile of a wave: c = sum over the
// quad's four k-steps (a fresh chain from zero).
template <int RT, int CT>
__device__ __forceinline__ void quad_chain(const f4 (&a)[RT], const f4 (&b)[CT], f4 (&c)[RT][CT]) {
#pragma unroll
  for (int rt = 0; rt < RT; rt++)
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      f4 x = MFMA32(a[rt].x, b[ct].x, ((f4){0, 0, 0, 0}));
      x = MFMA32(a[rt].y, b[ct].y, x);
      x = MFMA32(a[rt].z, b[ct].z, x);
      c[rt][ct] = MFMA32(a[rt].w, b[ct].w, x);
    }
}

// The FP64 running sum of the mixed solve takes the products in chunks of
// two k-step quads (32 k-values): c0 holds the first quad's FP32 chains
// (quad_chain), this runs the second quad's chains, adds the two in FP32 and
// adds that sum into the FP64 accumulator.  One tile row at a time, so that
// only one row of second-quad chains is live.  Every form of the solve
// (register ring, LDS staging, last-block kernel) forms the same chunks in
// the same order, so their results are the same bits.
template <int RT, int CT>
__device__ __forceinline__ void quad_chain_fold(const f4 (&a)[RT], const f4 (&b)[CT], const f4 (&c0)[RT][CT],
                                                d4 (&acc)[RT][CT]) {
#pragma unroll
  for (int rt = 0; rt < RT; rt++) {
    f4 x[CT];
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      x[ct] = MFMA32(a[rt].x, b[ct].x, ((f4){0, 0, 0, 0}));
      x[ct] = MFMA32(a[rt].y, b[ct].y, x[ct]);
      x[ct] = MFMA32(a[rt].z, b[ct].z, x[ct]);
      x[ct] = MFMA32(a[rt].w, b[ct].w, x[ct]);
    }
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int i = 0; i < 4; i++) acc[rt][ct][i] += (double)(c0[rt][ct][i] + x[ct][i]);
  }
}

template <int C, int WR, int WC, int G, int S>
__device__ __forceinline__ void gemm_staged(const float* __restrict__ Lk, const float* __restrict__ W32slab,
                                            int nq, float* __restrict__ ring_base,
                                            d4 (&acc)[NB / WR / 16][C / WC / 16]) {
  static_assert(G == 2 && S >= 2, "two quads per stage, split by the barrier");
  constexpr int RT = NB / WR / 16, CT = C / WC / 16, CTS = C / 16, NQB = NB / 16;
  constexpr int NW = WR * WC;
  constexpr int CL = G * NQB;          // chunks of L per stage
  constexpr int CPS = G * (NQB + CTS); // chunks per stage
  constexpr int LPW = CPS / NW;        // copies per wave and stage
  constexpr int NR = RT + CT;          // LDS reads per quad
  constexpr int RPS = (NR + 2) / 3;    // reads placed after each of a quad's first three k-steps
  static_assert(CPS % NW == 0 && 2 + LPW <= 4 * RT,
                "every wave copies the same number of chunks, one after each k-step of the second quad "
                "from the third on");
  float(*ring)[CPS * 256] = reinterpret_cast<float(*)[CPS * 256]>(ring_base);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  __builtin_assume(wave >= 0 && wave < NW);
  const int wr = wave / WC, wc = wave % WC;
  const int nst = nq / G;
  // copy i of this wave (chunk c = wave + i NW) of stage st (clamped to the
  // last: the tail copies are never read) into slot st % S
  auto issue_one = [&](int st, int i) {
    const int sl = st % S;
    st = st < nst ? st : nst - 1;
    const int c = wave + i * NW;
    const float* src = c < CL ? Lk + ((size_t)st * CL + c) * 256 + lane * 4
                              : W32slab + ((size_t)st * G * CTS + (c - CL)) * 256 + lane * 4;
    chunk_to_lds(src, &ring[sl][c * 256]);
  };
  // operand fragment r of quad g of stage st: r < RT rows of L, then the W
  // column tiles
  auto read_one = [&](int st, int g, int r, f4 (&a)[RT], f4 (&b)[CT]) {
    const float* __restrict__ slot = ring[st % S];
    if (r < RT)
      a[r] = *reinterpret_cast<const f4*>(slot + (g * NQB + wr * RT + r) * 256 + lane * 4);
    else
      b[r - RT] = *reinterpret_cast<const f4*>(slot + (CL + g * CTS + wc * CT + r - RT) * 256 + lane * 4);
  };
  // all S slots filled, stage 0 visible
#pragma unroll
  for (int st = 0; st < S; st++)
#pragma unroll
    for (int i = 0; i < LPW; i++) issue_one(st, i);
  wait_vm_lgkm0<(S - 1) * LPW>();
  barrier_only();
  f4 a0[RT], b0[CT], a1[RT], b1[CT];
  f4 c0[RT][CT];
#pragma unroll
  for (int r = 0; r < NR; r++) read_one(0, 0, r, a0, b0);
  // The chains of both quads run one k-step at a time (the same chains as
  // quad_chain and quad_chain_fold, the same bits), and the other
  // instructions of each half-stage sit between the steps: the second
  // quad's LDS reads in the first half; after the barrier, the next stage's
  // first reads and this wave's copies of stage st + S.  Issued as a block
  // before the MFMAs, they left the matrix pipe idle while both waves of a
  // SIMD issued them.
  for (int st = 0; st < nst; st++) {
    wait_lgkm0();
#pragma unroll
    for (int q = 0; q < 4; q++) {
#pragma unroll
      for (int rt = 0; rt < RT; rt++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
          c0[rt][ct] = MFMA32(a0[rt][q], b0[ct][q], q == 0 ? ((f4){0, 0, 0, 0}) : c0[rt][ct]);
#pragma unroll
      for (int r = q * RPS; r < (q + 1) * RPS; r++)
        if (q < 3 && r < NR) read_one(st, 1, r, a1, b1);
      __builtin_amdgcn_sched_barrier(0);
    }
    // stage st+1 is in LDS for every wave; every wave has read all of stage st
    wait_vm_lgkm0<(S - 2) * LPW>();
    barrier_only();
    // second quad and the fold into the FP64 sum, one tile row at a time
#pragma unroll
    for (int rt = 0; rt < RT; rt++) {
      f4 x[CT];
#pragma unroll
      for (int q = 0; q < 4; q++) {
#pragma unroll
        for (int ct = 0; ct < CT; ct++) x[ct] = MFMA32(a1[rt][q], b1[ct][q], q == 0 ? ((f4){0, 0, 0, 0}) : x[ct]);
        const int step = rt * 4 + q;
#pragma unroll
        for (int r = step * RPS; r < (step + 1) * RPS; r++)  // (past the last stage: reads of a clamped copy, unused)
          if (step < 3 && r < NR) read_one(st + 1, 0, r, a0, b0);
        if (step >= 2 && step < 2 + LPW) issue_one(st + S, step - 2);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
#pragma unroll
        for (int i = 0; i < 4; i++) acc[rt][ct][i] += (double)(c0[rt][ct][i] + x[ct][i]);
    }
    asm volatile("" ::: "memory");
  }
  // the ring shares its LDS with the right-hand side staged next: the tail
  // copies land and every wave is done reading before that is written
  wait_vm_lgkm0<0>();
  barrier_only();
}

// Mixed-precision blocked lower solve W = L^{-1}(X - 1 s^T): as k_trsm, but
// each off-diagonal product L_kj W_j uses FP32-rounded operands on FP32 MFMA
// (v_mfma_f32_16x16x4f32) with FP32 accumulation over one chunk of two
// k-step quads (4 k-steps each), and the chunk is added into an FP64
// running accumulator (quad_chain_fold).  The diagonal
// step inv(L_kk) R_k stays FP64.  Both W (FP64, for the assembly) and an
// FP32 copy (quad layout, for later trailing products) are stored.
// The FP32 output layout is lane l, element i -> row 4(l/16) + i.
// Operands of the off-diagonal products: S = 0, a register ring of D quads
// per wave (each wave loads its own tiles); S > 0, stages of G quads copied
// through S LDS slots (gemm_staged), which lets one work-group take 128
// columns (a 32 x 64 tile per wave) and halves the L traffic per column.
template <int C, int WR, int WC, int D, int G = 1, int S = 0>
__global__ __launch_bounds__(64 * WR * WC) void k_trsm_mixed(const JobTable tab) {
  constexpr int RW = NB / WR, RT = RW / 16;
  constexpr int CW = C / WC, CT = CW / 16;
  constexpr int CTS = C / 16;
  constexpr int NQB = NB / 16;  // k-step quads per row block
  static_assert(D % 2 == 0, "quads are folded in pairs within a ring group");
  static_assert(S == 0 || (G == 2 && NQB % G == 0 && S >= 2), "staging: a stage is a pair of quads");
  // R_k for the diagonal step; with staged operands the same LDS holds the
  // stage ring during the GEMM
  constexpr int RL_DOUBLES = NB * C > staged_ring_floats<C, G>(S) / 2 ? NB * C : staged_ring_floats<C, G>(S) / 2;
  __shared__ __attribute__((aligned(16))) double Rl[RL_DOUBLES];

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

  // the wave index is wave-uniform (kept in scalar registers)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  const int wr = wave / WC, wc = wave % WC;
  const int64_t col_base = slab * C + wc * CW;

  // the last row block is left to k_trsm_mixed_last when all of its real
  // rows lie in the first wave row's tile
  const int Kmain = mixed_last_block_split(n, K, RW) ? K - 1 : K;
  for (int k = 0; k < Kmain; k++) {
    // The block's right-hand side, loaded before the GEMM so that the GEMM
    // hides the latency: genotypes as loaded (0 outside the matrix) and the
    // shift of each column (0 past the last column); the centered value is
    // formed where it is consumed.  When the wave's tile lies inside the
    // matrix (all but the last row block and the last slab) the loads are
    // plain, so they all issue before the first wait; a guarded load is a
    // branch with a wait of its own.
    int8_t xv[RT][CT][4];
    double sc[CT];
    if ((int64_t)k * NB + wr * RW + RW <= n && col_base + CW <= ncols) {
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
        const int64_t col = col_base + ct * 16 + lane % 16;
        const int8_t* __restrict__ xc = X + col * ldx + (int64_t)k * NB + wr * RW + 4 * (lane / 16);
        sc[ct] = shift[col];
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
#pragma unroll
          for (int i = 0; i < 4; i++) xv[rt][ct][i] = xc[rt * 16 + i];
      }
    } else {
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
        const int64_t col = col_base + ct * 16 + lane % 16;
        sc[ct] = col < ncols ? shift[col] : 0.0;
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
#pragma unroll
          for (int i = 0; i < 4; i++) {
            const int64_t row = (int64_t)k * NB + wr * RW + rt * 16 + 4 * (lane / 16) + i;
            xv[rt][ct][i] = (row < n && col < ncols) ? X[col * ldx + row] : (int8_t)0;
          }
      }
    }

    d4 acc[RT][CT];
#pragma unroll
    for (int a = 0; a < RT; a++)
#pragma unroll
      for (int b = 0; b < CT; b++) acc[a][b] = (d4){0, 0, 0, 0};

    const int nq = k * NQB;
    if constexpr (S > 0) {
      if (nq > 0) gemm_staged<C, WR, WC, G, S>(L32 + strip_offset(k), W32slab, nq, reinterpret_cast<float*>(Rl), acc);
    } else if (nq > 0) {
      // register ring: D quads in flight, each wave loading its own tiles;
      // quads 2i and 2i+1 of the ring form one chunk (quad_chain_fold)
      const float* __restrict__ Ls = L32 + strip_offset(k) + (size_t)(wr * RT) * 256 + lane * 4;
      const float* __restrict__ Wb = W32slab + (size_t)(wc * CT) * 256 + lane * 4;
      f4 a[D][RT], b[D][CT];
      f4 c0[RT][CT];
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
          if (s % 2 == 0)
            quad_chain<RT, CT>(a[s], b[s], c0);
          else
            quad_chain_fold<RT, CT>(a[s], b[s], c0, acc);
          int nx = q0 + s + D;
          nx = nx < nq ? nx : nq - 1;
#pragma unroll
          for (int rt = 0; rt < RT; rt++)
            a[s][rt] = *reinterpret_cast<const f4*>(Ls + ((size_t)nx * (NB / 16) + rt) * 256);
#pragma unroll
          for (int ct = 0; ct < CT; ct++)
            b[s][ct] = *reinterpret_cast<const f4*>(Wb + ((size_t)nx * CTS + ct) * 256);
          asm volatile("" ::: "memory");
        }
      }
    }

    static_assert(WR == 4 && RT == 2, "the diagonal step deals two row tiles to each of four wave rows");
    d2 pa[DIAG_PF];
    DIAG_BY_ROW(diag_prefetch<WROW>(LinvP, k, lane, pa));

    // R_k = (x - s) - acc, to LDS in the FP64 B-operand pair layout: element
    // (row 4g + i) of the FP32 output goes to k-step (row0/4 + g), lane 16i + l%16;
    // padding rows take 0
#pragma unroll
    for (int rt = 0; rt < RT; rt++) {
      const int rowl = wr * RW + rt * 16;
      const int ks = rowl / 4 + lane / 16;
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const bool in = (int64_t)k * NB + rowl + 4 * (lane / 16) + i < n;
          Rl[((size_t)(ks / 2) * CTS + wc * CT + ct) * 128 + (i * 16 + lane % 16) * 2 + (ks % 2)] =
              (in ? (double)xv[rt][ct][i] - sc[ct] : 0.0) - acc[rt][ct][i];
        }
    }
    __syncthreads();

    // W_k = inv(L_kk) R_k with the row tiles dealt (wave row wr takes 16-row
    // tiles wr and NB/16 - 1 - wr; same products in the same order per
    // element as the last-block kernel's)
    d4 w64[2][CT];
    DIAG_BY_ROW((diag_step_dealt<CT, CTS, WROW>(LinvP, k, Rl, wc * CT, lane, pa, w64)));
    // store W_k: FP64 pairs (identity per lane) and the FP32 quad copy
    // (element i of the FP64 output is k-step row0/4 + i, i.e. position i of
    // quad row0/16, same lane); typed global stores (generic ones would be
    // flat stores, which later LDS waits would have to wait for too)
#pragma unroll
    for (int h = 0; h < 2; h++) {
      const int tile = h == 0 ? wr : NB / 16 - 1 - wr;
      const int64_t row0 = (int64_t)k * NB + 16 * tile;
      const int64_t ks0 = row0 / 4;
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
#pragma unroll
        for (int i = 0; i < 4; i += 2)
          *(__attribute__((address_space(1))) d2*)(Wslab + ((size_t)((ks0 + i) / 2) * CTS + wc * CT + ct) * 128 +
                                                   lane * 2) = (d2){w64[h][ct][i], w64[h][ct][i + 1]};
        *(__attribute__((address_space(1))) f4*)(W32slab + ((size_t)(row0 / 16) * CTS + wc * CT + ct) * 256 +
                                                 lane * 4) =
            (f4){(float)w64[h][ct][0], (float)w64[h][ct][1], (float)w64[h][ct][2], (float)w64[h][ct][3]};
      }
    }
    __threadfence_block();
    __syncthreads();
  }
}


// The last row block of every slab when mixed_last_block_split holds, after
// k_trsm_mixed has solved the others (same grid): the wave rows share the
// first tile's GEMM (FP32 chunks folded into FP64 per wave row, wave row w
// over its quarter of the quads), the FP64 partial sums meet in LDS in a
// fixed order, then the FP64 diagonal step and both stores run as in
// k_trsm_mixed (rows beyond the first tile give W = 0, as padding must).
template <int C, int WR, int WC, int D>
__global__ __launch_bounds__(64 * WR * WC) void k_trsm_mixed_last(const JobTable tab) {
  constexpr int RW = NB / WR, RT = RW / 16;
  constexpr int CW = C / WC, CT = CW / 16;
  constexpr int CTS = C / 16;
  constexpr int NQB = NB / 16;
  static_assert(D % 2 == 0, "quads are folded in pairs within a ring group");
  __shared__ __attribute__((aligned(16))) double Rl[NB * C];

  int jb = 0;
  while (jb + 1 < tab.njobs && (int64_t)blockIdx.x >= tab.j[jb + 1].slab0) jb++;
  const JobDesc& J = tab.j[jb];
  const int K = J.K;
  if (!mixed_last_block_split(J.n, K, RW)) return;
  const int k = K - 1;
  const int64_t slab = (int64_t)blockIdx.x - J.slab0;
  const int8_t* __restrict__ X = reinterpret_cast<const int8_t*>(J.X);
  const double* __restrict__ shift = J.shift;
  double* __restrict__ Wslab = J.W + slab * (int64_t)K * NB * C;
  float* __restrict__ W32slab = J.W32 + slab * (int64_t)K * NB * C;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  const int wr = wave / WC, wc = wave % WC;
  const int64_t col_base = slab * C + wc * CW;

  // the first tile's centered right-hand side, added by the first wave row
  const double xs = wr == 0 ? 1.0 : 0.0;
  double xv[RT][CT][4];
#pragma unroll
  for (int rt = 0; rt < RT; rt++)
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      const int64_t col = col_base + ct * 16 + lane % 16;
#pragma unroll
      for (int i = 0; i < 4; i++) {
        const int64_t row = (int64_t)k * NB + rt * 16 + 4 * (lane / 16) + i;
        xv[rt][ct][i] = (row < J.n && col < J.ncols) ? (double)X[col * J.ldx + row] - shift[col] : 0.0;
      }
    }
  d4 acc[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; a++)
#pragma unroll
    for (int b = 0; b < CT; b++) acc[a][b] = (d4){0, 0, 0, 0};
  const float* __restrict__ Ls = J.Lstrips32 + strip_offset(k) + lane * 4;  // row tile 0
  const float* __restrict__ Wb = W32slab + (size_t)(wc * CT) * 256 + lane * 4;
  const int ng = k * NQB / D;  // groups of D quads
  const int q0b = ng * wr / WR * D, q1b = ng * (wr + 1) / WR * D;
  if (q1b > q0b) {
    f4 a[D][RT], b[D][CT];
    f4 c0[RT][CT];
#pragma unroll
    for (int s = 0; s < D; s++) {
#pragma unroll
      for (int rt = 0; rt < RT; rt++)
        a[s][rt] = *reinterpret_cast<const f4*>(Ls + ((size_t)(q0b + s) * (NB / 16) + rt) * 256);
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
        b[s][ct] = *reinterpret_cast<const f4*>(Wb + ((size_t)(q0b + s) * CTS + ct) * 256);
      asm volatile("" ::: "memory");
    }
    for (int q0 = q0b; q0 < q1b; q0 += D) {
#pragma unroll
      for (int s = 0; s < D; s++) {
        if (s % 2 == 0)
          quad_chain<RT, CT>(a[s], b[s], c0);
        else
          quad_chain_fold<RT, CT>(a[s], b[s], c0, acc);
        int nx = q0 + s + D;
        nx = nx < q1b ? nx : q1b - 1;
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
          a[s][rt] = *reinterpret_cast<const f4*>(Ls + ((size_t)nx * (NB / 16) + rt) * 256);
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
          b[s][ct] = *reinterpret_cast<const f4*>(Wb + ((size_t)nx * CTS + ct) * 256);
        asm volatile("" ::: "memory");
      }
    }
  }
  // partial sums into this wave row's rows of Rl (the FP32 output layout:
  // element i of lane l is row 4(l/16) + i of the tile), then the first wave
  // row's rows gather them
#pragma unroll
  for (int rt = 0; rt < RT; rt++) {
    const int rowl = wr * RW + rt * 16;
    const int ks = rowl / 4 + lane / 16;
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int i = 0; i < 4; i++)
        Rl[((size_t)(ks / 2) * CTS + wc * CT + ct) * 128 + (i * 16 + lane % 16) * 2 + (ks % 2)] =
            xs * xv[rt][ct][i] - acc[rt][ct][i];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < RW * C; i += 64 * WR * WC) {
    double v = Rl[i];
#pragma unroll
    for (int w = 1; w < WR; w++) {
      v += Rl[(size_t)w * RW * C + i];
      Rl[(size_t)w * RW * C + i] = 0.0;
    }
    Rl[i] = v;
  }
  __syncthreads();
  // W_k = inv(L_kk) R_k in FP64 and both stores, as in k_trsm_mixed
  d4 w64[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; a++)
#pragma unroll
    for (int b = 0; b < CT; b++) w64[a][b] = (d4){0, 0, 0, 0};
  const double* __restrict__ Li = J.LinvP + (size_t)k * NB * NB + (size_t)(wr * RT) * 128 + lane * 2;
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
}


hipError_t launch_trsm_mixed(const JobTable& tab, int64_t nslabs, int C, hipStream_t st) {
  bool last = false;  // some job of the table leaves its last block to k_trsm_mixed_last
  for (int i = 0; i < tab.njobs; i++) last = last || mixed_last_block_split(tab.j[i].n, tab.j[i].K, NB / 4);
  switch (C) {
    case 32:
      k_trsm_mixed<32, 4, 2, 4><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      if (last) k_trsm_mixed_last<32, 4, 2, 4><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      break;
    case 64:
      k_trsm_mixed<64, 4, 2, 4, 2, 4><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      if (last) k_trsm_mixed_last<64, 4, 2, 4><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      break;
    case 128:
      k_trsm_mixed<128, 4, 2, 4, 2, 4><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      if (last) k_trsm_mixed_last<128, 4, 2, 2><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gls
