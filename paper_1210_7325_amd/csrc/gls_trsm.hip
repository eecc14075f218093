// FP64 blocked triangular solve of genotype blocks (a2), the hot kernel.
#include "gls_device.h"

namespace gls {

// Phase timestamps of k_trsm_pair, compiled only into the measurement build
// (trsm_phase_timing.hip): thread 0 of each of the first PHASE_WGS
// work-groups records the constant 100 MHz clock and the shader clock at
// PHASE_POINTS points of each row-block pair.  Without GLS_PHASE_TIMING the
// stamps compile to nothing.
#ifdef GLS_PHASE_TIMING
constexpr int PHASE_WGS = 256, PHASE_PAIRS = 64, PHASE_POINTS = 6;
__device__ unsigned long long g_phase_rt[PHASE_WGS * PHASE_PAIRS * PHASE_POINTS];
__device__ unsigned long long g_phase_cyc[PHASE_WGS * PHASE_PAIRS * PHASE_POINTS];
#define PHASE_STAMP(pair, point)                                                              \
  do {                                                                                        \
    if (threadIdx.x == 0 && blockIdx.x < PHASE_WGS && (pair) < PHASE_PAIRS) {                 \
      const size_t i_ = ((size_t)blockIdx.x * PHASE_PAIRS + (pair)) * PHASE_POINTS + (point); \
      g_phase_rt[i_] = wall_clock64();                                                        \
      g_phase_cyc[i_] = clock64();                                                            \
    }                                                                                         \
  } while (0)
#else
#define PHASE_STAMP(pair, point) ((void)0)
#endif

// ---------------------------------------------------------------------------
// a2: blocked lower triangular solve  W = L^{-1} X  (the trsm of Alg. 5,
// grouped over many right-hand sides as the paper prescribes)
//
// One work-group owns a slab of C columns and walks the row blocks
// k = 0..K-1 (left-looking):
//   R_k = X_k - sum_{j<k} L_kj W_j     FP64 MFMA, operands from the packed
//                                      strip and the slab's own W (a
//                                      register ring per wave, or staged
//                                      through LDS for the whole group)
//   W_k = inv(L_kk) R_k                FP64 MFMA, R_k staged in LDS
// The waves split the NB rows of a block (WR ways) and the C columns (WC
// ways).  X is int8 genotypes, exact in FP64.

// True when the last row block's real rows (n - (K-1) NB of them) all lie in
// the first of the WR wave rows' tiles (RW rows): the rest of that block is
// padding, whose R and W are zero, and k_trsm_last solves it.
__host__ __device__ inline bool last_block_split(int64_t n, int K, int RW) {
  return K > 1 && n - (int64_t)(K - 1) * NB <= RW;
}

// A split last block has at most LAST_RW real rows: one or two 16-row tiles.
constexpr int LAST_RW = NB / 4;
__host__ __device__ inline int last_block_tiles(int64_t n, int K) {
  return n - (int64_t)(K - 1) * NB <= 16 ? 1 : 2;
}

// The off-diagonal sum of a split last block, grown as the walk produces
// W: once blocks k0 .. k0 + NBLK - 1 are stored (and a barrier has made
// them visible to the work-group), the wave adds their terms L_{K-1,j} W_j
// to NR output tiles (row tiles lt0 .. lt0 + NR - 1 of block K-1, column
// tile ct of the slab).  Each tile is one MFMA chain over the k-step pairs
// in increasing order, the order of every other block's GEMM, so the
// results are the same bits for every slab width.  Between calls a chain
// sits in the slab's rows of block K-1 (unused until the last block's
// diagonal step, which reads it from there), so the walk keeps no
// registers for it; W_j comes from the slab, still in the caches, and the
// strip of block K-1 from global memory, P pairs ahead.  This replaces a
// second pass over the slab's whole W after the walk (10 MB per 128-column
// slab from HBM).
template <int CTS, int NR, int NBLK, int P>
__device__ __forceinline__ void last_block_sum(const double* __restrict__ Lstrips, double* __restrict__ Wslab,
                                               int K, int k0, int lt0, int ct, int lane) {
  // P pairs in flight, each pinned where it is issued (left to the
  // scheduler, the refills slid next to their use and three pairs in
  // flight did not cover the latency of the strip's first touch)
  constexpr int NPB = NB / 8, NKP = NBLK * NPB;
  static_assert(P >= 1 && P <= NKP, "prefetch depth");
  // Buffer loads and stores: a wave-uniform base (scalar registers), the
  // lane's 16 bytes as the only vector offset and the step within the
  // operand as a scalar offset, so that no per-lane 64-bit address lives
  // across the walk (the walk's loop needs every vector register).
  auto rsrc = [](const double* base) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, 0x7fffffff, 0x00020000);
  };
  // two resources for the whole walk (the slab, the strip of block K-1);
  // byte offsets within them (< 2^31: a slab is K NB C doubles, the strip's
  // pairs up to block K-2 (K-1) NB^2 doubles)
  const auto Lr = rsrc(Lstrips + strip_offset(K - 1));
  const auto Wr = rsrc(Wslab);
  const int la0 = (k0 * NPB * (NB / 16) + lt0) * 1024;
  const int wb0 = (k0 * NPB * CTS + ct) * 1024;
  const int ac0 = (((K - 1) * NPB + 2 * lt0) * CTS + ct) * 1024;
  const int vo = lane * 16;
  auto ld = [&](__amdgpu_buffer_rsrc_t r, int soff) {
    return __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, vo, soff, 0));
  };
  d4 acc[NR];
#pragma unroll
  for (int r = 0; r < NR; r++) {
    // (the first call starts the chain at zero; the load is issued anyway,
    // so that no branch joins in front of the loop's waits)
    const d2 lo = ld(Wr, ac0 + (2 * r) * CTS * 1024), hi = ld(Wr, ac0 + (2 * r + 1) * CTS * 1024);
    acc[r] = k0 > 0 ? (d4){lo.x, lo.y, hi.x, hi.y} : (d4){0, 0, 0, 0};
  }
  d2 a[P][NR], b[P];
#pragma unroll
  for (int s = 0; s < P; s++) {
#pragma unroll
    for (int r = 0; r < NR; r++) a[s][r] = ld(Lr, la0 + (s * (NB / 16) + r) * 1024);
    b[s] = ld(Wr, wb0 + s * CTS * 1024);
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int kp = 0; kp < NKP; kp++) {
    const int s = kp % P;
#pragma unroll
    for (int r = 0; r < NR; r++) {
      acc[r] = MFMA64(a[s][r].x, b[s].x, acc[r]);
      acc[r] = MFMA64(a[s][r].y, b[s].y, acc[r]);
    }
    if (kp + P < NKP) {
#pragma unroll
      for (int r = 0; r < NR; r++) a[s][r] = ld(Lr, la0 + ((kp + P) * (NB / 16) + r) * 1024);
      b[s] = ld(Wr, wb0 + (kp + P) * CTS * 1024);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int r = 0; r < NR; r++)
#pragma unroll
    for (int h = 0; h < 2; h++)
      __builtin_amdgcn_raw_buffer_store_b128(
          __builtin_bit_cast(__attribute__((ext_vector_type(4))) unsigned, (d2){acc[r][2 * h], acc[r][2 * h + 1]}),
          Wr, vo, ac0 + (2 * r + h) * CTS * 1024, 0);
}

template <int C, int G>
constexpr int staged_ring_doubles(int S) { return S * G * (NB / 16 + C / 16) * 128; }

// The off-diagonal sum acc = sum_{j<k} L_kj W_j for one row block with the
// operands staged through LDS: a stage is two k-step pairs, i.e. 2 (NB/16 +
// C/16) chunks of 1 KB (the strip tiles of all NB rows and the W tiles of
// all C columns), copied by the work-group's waves straight into one of S
// LDS slots, S - 1 stages ahead.  Every wave then reads its own tiles from
// LDS: each operand byte crosses the L1 cache once per work-group, and the
// stages in flight cost no registers.
//
// The barrier sits in the middle of a stage, so that MFMAs are always ready
// on both sides of it: a wave reads the second pair of stage st, runs the
// first pair's MFMAs, waits for its own copies of stage st+1 (vmcnt) and
// for its LDS reads, and passes the barrier, which makes stage st+1 visible
// to everyone and certifies that every wave has read all of stage st; it
// then refills stage st's slot with stage st+S, reads the first pair of
// stage st+1 and runs the second pair of stage st while those reads land.
// The products are the same MFMAs in the same order as the register ring's.
template <int C, int WR, int WC, int G, int S>
__device__ __forceinline__ void gemm_staged_f64(const double* __restrict__ Lk,
                                                const double* __restrict__ Wslab, int npairs,
                                                double* __restrict__ ring_base,
                                                d4 (&acc)[NB / WR / 16][C / WC / 16]) {
  static_assert(G == 2 && S >= 2, "two pairs per stage, split by the barrier");
  constexpr int RT = NB / WR / 16, CT = C / WC / 16, CTS = C / 16, NT = NB / 16;
  constexpr int NW = WR * WC;
  constexpr int CL = G * NT;           // chunks of L per stage
  constexpr int CPS = G * (NT + CTS);  // chunks per stage
  constexpr int LPW = CPS / NW;        // copies per wave and stage
  constexpr int NG = RT * CT;          // MFMA groups (output tiles) per half-stage
  constexpr int NR = RT + CT;          // LDS reads per half-stage
  constexpr int RPG = (NR + NG / 2 - 1) / (NG / 2);  // reads after each of the first NG/2 groups
  static_assert(CPS % NW == 0 && NG >= 2 && LPW <= NG,
                "every wave copies the same number of chunks, at most one after each group");
  double(*ring)[CPS * 128] = reinterpret_cast<double(*)[CPS * 128]>(ring_base);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  // (lets the compiler resolve which chunks a wave copies: no branches in
  // the loop)
  __builtin_assume(wave >= 0 && wave < NW);
  const int wr = wave / WC, wc = wave % WC;
  const int nst = npairs / G;
  // copy i of this wave (chunk c = wave + i NW) of stage st (clamped to the
  // last: the tail copies are never read) into slot st % S
  auto issue_one = [&](int st, int i) {
    const int sl = st % S;
    st = st < nst ? st : nst - 1;
    const int c = wave + i * NW;
    const double* src = c < CL ? Lk + ((size_t)st * CL + c) * 128 + lane * 2
                               : Wslab + ((size_t)st * G * CTS + (c - CL)) * 128 + lane * 2;
    chunk_to_lds(src, &ring[sl][c * 128]);
  };
  // operand fragment r of pair g of stage st: r < RT rows of L, then the W
  // column tiles
  auto read_one = [&](int st, int g, int r, d2 (&a)[RT], d2 (&b)[CT]) {
    const double* __restrict__ slot = ring[st % S];
    if (r < RT)
      a[r] = *reinterpret_cast<const d2*>(slot + (g * NT + wr * RT + r) * 128 + lane * 2);
    else
      b[r - RT] = *reinterpret_cast<const d2*>(slot + (CL + g * CTS + wc * CT + r - RT) * 128 + lane * 2);
  };
  auto mfma_group = [&](int g8, const d2 (&a)[RT], const d2 (&b)[CT]) {
    const int rt = g8 / CT, ct = g8 % CT;
    acc[rt][ct] = MFMA64(a[rt].x, b[ct].x, acc[rt][ct]);
    acc[rt][ct] = MFMA64(a[rt].y, b[ct].y, acc[rt][ct]);
  };
  // all S slots filled, stage 0 visible
#pragma unroll
  for (int st = 0; st < S; st++)
#pragma unroll
    for (int i = 0; i < LPW; i++) issue_one(st, i);
  wait_vm_lgkm0<(S - 1) * LPW>();
  barrier_only();
  d2 a0[RT], b0[CT], a1[RT], b1[CT];
#pragma unroll
  for (int r = 0; r < NR; r++) read_one(0, 0, r, a0, b0);
  // Each half-stage's MFMAs go out one output tile at a time, and the other
  // instructions of the half sit between the tiles: the next half's LDS
  // reads after the first NG/2 tiles, and after the barrier this wave's
  // copies of stage st + S after the last LPW tiles (issued as a block
  // before the MFMAs, they left the matrix pipe idle).
  for (int st = 0; st < nst; st++) {
    wait_lgkm0();
#pragma unroll
    for (int g8 = 0; g8 < NG; g8++) {
      mfma_group(g8, a0, b0);
#pragma unroll
      for (int r = g8 * RPG; r < (g8 + 1) * RPG; r++)
        if (r < NR) read_one(st, 1, r, a1, b1);
      __builtin_amdgcn_sched_barrier(0);
    }
    // stage st+1 is in LDS for every wave; every wave has read all of stage st
    wait_vm_lgkm0<(S - 2) * LPW>();
    barrier_only();
#pragma unroll
    for (int g8 = 0; g8 < NG; g8++) {
      mfma_group(g8, a1, b1);
#pragma unroll
      for (int r = g8 * RPG; r < (g8 + 1) * RPG; r++)  // (past the last stage: reads of a clamped copy, unused)
        if (r < NR) read_one(st + 1, 0, r, a0, b0);
      if (g8 >= NG - LPW) issue_one(st + S, g8 - (NG - LPW));
      __builtin_amdgcn_sched_barrier(0);
    }
    asm volatile("" ::: "memory");
  }
  // the ring shares its LDS with the right-hand side staged next: the tail
  // copies land and every wave is done reading before that is written
  wait_vm_lgkm0<0>();
  barrier_only();
}

template <int C, int WR, int WC, int D, typename TIn, int G = 1, int S = 0>
__global__ __launch_bounds__(64 * WR * WC) void k_trsm(const JobTable tab) {
  constexpr int RW = NB / WR, RT = RW / 16;
  constexpr int CW = C / WC, CT = CW / 16;
  constexpr int CTS = C / 16;  // column tiles per slab
  constexpr int NPB = NB / 8;  // k-step pairs per row block
  static_assert(RT >= 1 && CT >= 1, "tile shape");
  static_assert(NPB % D == 0, "prefetch depth must divide the pairs of a block");
  static_assert(S == 0 || (NPB % G == 0 && S >= 2), "staging");
  // R_k for the diagonal step; with staged operands (S > 0) the same LDS
  // holds the stage ring during the GEMM
  constexpr int RL_DOUBLES = NB * C > staged_ring_doubles<C, G>(S) ? NB * C : staged_ring_doubles<C, G>(S);
  __shared__ __attribute__((aligned(16))) double Rl[RL_DOUBLES];

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

  // the wave index is wave-uniform (kept in scalar registers)
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  const int wr = wave / WC, wc = wave % WC;
  const int64_t col_base = slab * C + wc * CW;

  // when the last row block's real rows fit its first LAST_RW rows, the
  // walk stops one block early, sums that block's GEMM as it goes
  // (last_block_sum) and leaves its diagonal step to k_trsm_last
  static_assert(2 * CTS <= WR * WC, "a wave for each output tile of the last block's sum");
  const bool split = last_block_split(n, K, LAST_RW);
  const int last_tiles = last_block_tiles(n, K);
  const int Kmain = split ? K - 1 : K;
  for (int k = 0; k < Kmain; k++) {
    // this block's right-hand side, loaded early and held as loaded (it is
    // consumed after the GEMM).  When the wave's tile lies inside the matrix
    // (all but the last row block and the last slab) the loads are plain, so
    // they all issue before the first wait; a guarded load is a branch with
    // a wait of its own.
    TIn xv[RT][CT][4];
    if ((int64_t)k * NB + wr * RW + RW <= n && col_base + CW <= ncols) {
#pragma unroll
      for (int ct = 0; ct < CT; ct++) {
        const TIn* __restrict__ xc =
            X + (col_base + ct * 16 + lane % 16) * ldx + (int64_t)k * NB + wr * RW + lane / 16;
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
#pragma unroll
          for (int i = 0; i < 4; i++) xv[rt][ct][i] = xc[rt * 16 + 4 * i];
      }
    } else {
#pragma unroll
      for (int rt = 0; rt < RT; rt++)
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
#pragma unroll
          for (int i = 0; i < 4; i++) {
            const int64_t row = (int64_t)k * NB + wr * RW + rt * 16 + lane / 16 + 4 * i;
            const int64_t col = col_base + ct * 16 + lane % 16;
            xv[rt][ct][i] = (row < n && col < ncols) ? X[col * ldx + row] : (TIn)0;
          }
    }

    d4 acc[RT][CT];
#pragma unroll
    for (int a = 0; a < RT; a++)
#pragma unroll
      for (int b = 0; b < CT; b++) acc[a][b] = (d4){0, 0, 0, 0};

    // sum_{j<k} L_kj W_j: software pipeline with D k-step pairs in flight
    const double* __restrict__ Ls = Lstrips + strip_offset(k) + (size_t)(wr * RT) * 128 + lane * 2;
    const double* __restrict__ Wb = Wslab + (size_t)(wc * CT) * 128 + lane * 2;
    const int npairs = k * NPB;
    if constexpr (S > 0) {
      if (npairs > 0) gemm_staged_f64<C, WR, WC, G, S>(Lstrips + strip_offset(k), Wslab, npairs, Rl, acc);
    } else if (npairs > 0) {
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
              (d2){(double)xv[rt][ct][i] - acc[rt][ct][i], (double)xv[rt][ct][i + 1] - acc[rt][ct][i + 1]};
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
    // W_k's terms of a split last block's sum: one output tile per wave
    // (row tile wave / CTS, column tile wave % CTS); the other waves go on
    // to the next block
    if (split) {
      const int lt0 = wave / CTS;
      if (lt0 < last_tiles) last_block_sum<CTS, 1, 1, 4>(Lstrips, Wslab, K, k, lt0, wave % CTS, lane);
    }
  }
}

// ---------------------------------------------------------------------------
// Two row blocks per off-diagonal sum (128-column slabs).  k_trsm reads the
// slab's earlier W once per row block: sum_k k NB C 8 bytes, almost all of
// the kernel's memory traffic.  Here the work-group takes the row blocks in
// pairs (k, k+1): one pass over W_0..W_{k-1} feeds the GEMMs of both blocks
// (256 rows of L against each W tile), then
//   W_k      = inv(L_kk) R_k
//   acc_{k+1} += L_{k+1,k} W_k            (W_k from LDS)
//   W_{k+1}  = inv(L_{k+1,k+1}) R_{k+1}
// so W is read half as often.  Each wave holds the same 32 rows of both
// blocks (and 64 columns), so every wave has work in the L_{k+1,k} W_k
// step.  Every element's sum runs over the same k-steps in the same order
// as in k_trsm, so the results are the same bits for every slab width.

constexpr int PAIR_WR = 4, PAIR_WC = 2;   // eight waves of 32 (+32) x 64 tiles
constexpr int PAIR_SLOTS = 3;             // stage slots of 48 KB

// The off-diagonal sums of rows blocks k (strip Lk0) and k+1 (strip Lk1)
// over the same npairs k-step pairs of W, operands staged through LDS as in
// gemm_staged_f64: a stage is two pairs, i.e. 2 (2 NB/16 + C/16) chunks of
// 1 KB, copied S - 1 stages ahead; the barrier sits in the middle of the
// stage.  Each half-stage's 32 MFMAs go out in eight groups of four (one
// output tile each), and the other instructions of the half sit between
// the groups: the LDS reads of the next half's operands (two after each of
// the first four groups) and, after the barrier, this wave's copies of
// stage st + S (one after each of groups 2-7).  Issued as a block before
// the MFMAs, they left the matrix pipe idle while both waves of a SIMD
// issued them (about 8% of the loop's cycles).
template <int C, int WR, int WC, int S>
__device__ __forceinline__ void gemm_staged_pair(const double* __restrict__ Lk0, const double* __restrict__ Lk1,
                                                 const double* __restrict__ Wslab, int npairs,
                                                 double* __restrict__ ring_base,
                                                 d4 (&acc0)[NB / WR / 16][C / WC / 16],
                                                 d4 (&acc1)[NB / WR / 16][C / WC / 16]) {
  constexpr int G = 2;
  constexpr int RT = NB / WR / 16, CT = C / WC / 16, CTS = C / 16, NT = NB / 16;
  constexpr int NW = WR * WC;
  constexpr int CL = G * NT;             // chunks of one strip per stage
  constexpr int CPS = 2 * CL + G * CTS;  // chunks per stage
  static_assert(CPS % NW == 0 && CL % NW == 0, "every wave copies the same chunks of each operand");
  constexpr int LPW = CPS / NW;
  constexpr int NG = RT * CT;            // MFMA groups per half-stage
  constexpr int NR = 2 * RT + CT;        // LDS reads per half-stage
  static_assert(NG == 8 && NR == 8 && LPW == 6, "the interleave places 2 reads after groups 0-3 and "
                                                "1 copy after groups 2-7");
  double(*ring)[CPS * 128] = reinterpret_cast<double(*)[CPS * 128]>(ring_base);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  __builtin_assume(wave >= 0 && wave < NW);
  const int wr = wave / WC, wc = wave % WC;
  const int nst = npairs / G;
  // copy i of this wave (chunk c = wave + i NW) of stage st (clamped to the
  // last: the tail copies are never read) into slot st % S: chunks [0, CL)
  // strip k, [CL, 2 CL) strip k+1, then the W tiles
  auto issue_one = [&](int st, int i) {
    const int sl = st % S;
    st = st < nst ? st : nst - 1;
    const int c = wave + i * NW;
    const double* src = i < CL / NW       ? Lk0 + ((size_t)st * CL + c) * 128 + lane * 2
                        : i < 2 * CL / NW ? Lk1 + ((size_t)st * CL + (c - CL)) * 128 + lane * 2
                                          : Wslab + ((size_t)st * G * CTS + (c - 2 * CL)) * 128 + lane * 2;
    chunk_to_lds(src, &ring[sl][c * 128]);
  };
  // operand fragment r of half g of stage st: r < RT rows of strip k,
  // r < 2 RT rows of strip k+1, then the W column tiles
  auto read_one = [&](int st, int g, int r, d2 (&a0)[RT], d2 (&a1)[RT], d2 (&b)[CT]) {
    const double* __restrict__ slot = ring[st % S];
    if (r < RT)
      a0[r] = *reinterpret_cast<const d2*>(slot + (g * NT + wr * RT + r) * 128 + lane * 2);
    else if (r < 2 * RT)
      a1[r - RT] = *reinterpret_cast<const d2*>(slot + (CL + g * NT + wr * RT + r - RT) * 128 + lane * 2);
    else
      b[r - 2 * RT] = *reinterpret_cast<const d2*>(slot + (2 * CL + g * CTS + wc * CT + r - 2 * RT) * 128 + lane * 2);
  };
  // group g8: the four MFMAs of output tile (g8 / CT, g8 % CT) of both blocks
  auto mfma_group = [&](int g8, const d2 (&a0)[RT], const d2 (&a1)[RT], const d2 (&b)[CT]) {
    const int rt = g8 / CT, ct = g8 % CT;
    acc0[rt][ct] = MFMA64(a0[rt].x, b[ct].x, acc0[rt][ct]);
    acc1[rt][ct] = MFMA64(a1[rt].x, b[ct].x, acc1[rt][ct]);
    acc0[rt][ct] = MFMA64(a0[rt].y, b[ct].y, acc0[rt][ct]);
    acc1[rt][ct] = MFMA64(a1[rt].y, b[ct].y, acc1[rt][ct]);
  };
#pragma unroll
  for (int st = 0; st < S; st++)
#pragma unroll
    for (int i = 0; i < LPW; i++) issue_one(st, i);
  wait_vm_lgkm0<(S - 1) * LPW>();
  barrier_only();
  d2 p0[RT], q0[RT], b0[CT], p1[RT], q1[RT], b1[CT];
#pragma unroll
  for (int r = 0; r < NR; r++) read_one(0, 0, r, p0, q0, b0);
  for (int st = 0; st < nst; st++) {
    wait_lgkm0();
#pragma unroll
    for (int g8 = 0; g8 < NG; g8++) {
      mfma_group(g8, p0, q0, b0);
      if (g8 < 4) {
        read_one(st, 1, 2 * g8, p1, q1, b1);
        read_one(st, 1, 2 * g8 + 1, p1, q1, b1);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // stage st+1 is in LDS for every wave; every wave has read all of stage st
    wait_vm_lgkm0<(S - 2) * LPW>();
    barrier_only();
#pragma unroll
    for (int g8 = 0; g8 < NG; g8++) {
      mfma_group(g8, p1, q1, b1);
      if (g8 < 4) {  // (past the last stage: reads of a clamped copy, unused)
        read_one(st + 1, 0, 2 * g8, p0, q0, b0);
        read_one(st + 1, 0, 2 * g8 + 1, p0, q0, b0);
      }
      if (g8 >= 2) issue_one(st + S, g8 - 2);
      __builtin_amdgcn_sched_barrier(0);
    }
    asm volatile("" ::: "memory");
  }
  wait_vm_lgkm0<0>();
  barrier_only();
}

// A zero of each input type in device memory: the load address of elements
// outside the matrix.
__device__ const int8_t kZeroI8 = 0;
__device__ const double kZeroF64 = 0.0;
__device__ __forceinline__ const int8_t* zero_of(const int8_t*) { return &kZeroI8; }
__device__ __forceinline__ const double* zero_of(const double*) { return &kZeroF64; }

// The wave's RT x CT tiles of a row block's right-hand side (rows row0 +
// 16 rt + lane/16 + 4 i of the block, columns col_base + 16 ct + lane%16),
// as loaded.  Both forms issue one load per element and wait for none: plain
// loads when the tile lies inside the matrix, else loads whose address is
// that of a zero for the elements outside (no branch per element, so the
// wait counts agree where the two forms join and a later wait for another
// load does not have to wait for all of these).
template <int RT, int CT, typename TIn>
__device__ __forceinline__ void load_rhs(const TIn* __restrict__ X, int64_t ldx, int64_t n, int64_t ncols,
                                         int64_t row0, int64_t col_base, int lane, TIn (&xv)[RT][CT][4]) {
  if (row0 + RT * 16 <= n && col_base + CT * 16 <= ncols) {
#pragma unroll
    for (int ct = 0; ct < CT; ct++) {
      const TIn* __restrict__ xc = X + (col_base + ct * 16 + lane % 16) * ldx + row0 + lane / 16;
#pragma unroll
      for (int rt = 0; rt < RT; rt++)
#pragma unroll
        for (int i = 0; i < 4; i++) xv[rt][ct][i] = xc[rt * 16 + 4 * i];
    }
  } else {
    // (global address space for both, so that these are global loads, not
    // flat ones, which the LDS wait counter would count too)
    typedef const __attribute__((address_space(1))) TIn* gptr;
    const gptr gX = (gptr)X, zero = (gptr)zero_of(X);
#pragma unroll
    for (int rt = 0; rt < RT; rt++)
#pragma unroll
      for (int ct = 0; ct < CT; ct++)
#pragma unroll
        for (int i = 0; i < 4; i++) {
          const int64_t row = row0 + rt * 16 + lane / 16 + 4 * i;
          const int64_t col = col_base + ct * 16 + lane % 16;
          xv[rt][ct][i] = *((row < n && col < ncols) ? gX + col * ldx + row : zero);
        }
  }
}

// v (the wave's FP64 output tiles of rows wr RW ..) to LDS in the B-operand
// pair layout of a 128-row block, optionally as x - v
template <int RT, int CT, int CTS, typename TIn>
__device__ __forceinline__ void to_pair_layout(double* __restrict__ Rl, int wr_rows, int wc_tile, int lane,
                                               const TIn (&xv)[RT][CT][4], const d4 (&v)[RT][CT], bool minus) {
#pragma unroll
  for (int rt = 0; rt < RT; rt++) {
    const int rowl = wr_rows + rt * 16;
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int i = 0; i < 4; i += 2) {
        const int kp = (rowl / 4 + i) / 2;
        *reinterpret_cast<d2*>(&Rl[((size_t)kp * CTS + wc_tile + ct) * 128 + lane * 2]) =
            minus ? (d2){(double)xv[rt][ct][i] - v[rt][ct][i], (double)xv[rt][ct][i + 1] - v[rt][ct][i + 1]}
                  : (d2){v[rt][ct][i], v[rt][ct][i + 1]};
      }
  }
}

// The dealt tiles of diag_step_dealt: to the slab (rows k NB + 16 t) and,
// when Wl is given, to LDS in the B-operand pair layout.
template <int CT, int CTS>
__device__ __forceinline__ void store_w_dealt(double* __restrict__ Wslab, double* __restrict__ Wl, int k, int wr,
                                              int wc_tile, int lane, const d4 (&w)[2][CT]) {
  constexpr int NT = NB / 16;
#pragma unroll
  for (int h = 0; h < 2; h++) {
    const int t = h == 0 ? wr : NT - 1 - wr;
    const int64_t ks0 = (int64_t)k * (NB / 4) + 4 * t;
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int i = 0; i < 4; i += 2) {
        const d2 v = (d2){w[h][ct][i], w[h][ct][i + 1]};
        // (typed global and LDS stores: generic ones would compile to flat
        // stores, which every later LDS wait would have to wait for too)
        *(__attribute__((address_space(1))) d2*)(Wslab + ((size_t)((ks0 + i) / 2) * CTS + wc_tile + ct) * 128 +
                                                  lane * 2) = v;
        if (Wl) *(__attribute__((address_space(3))) d2*)(&Wl[((size_t)((4 * t + i) / 2) * CTS + wc_tile + ct) * 128 +
                                                           lane * 2]) = v;
      }
  }
}

template <int C, typename TIn>
__global__ __launch_bounds__(64 * PAIR_WR * PAIR_WC) void k_trsm_pair(const JobTable tab) {
  constexpr int WR = PAIR_WR, WC = PAIR_WC, S = PAIR_SLOTS;
  constexpr int RW = NB / WR, RT = RW / 16;
  constexpr int CW = C / WC, CT = CW / 16;
  constexpr int CTS = C / 16;
  constexpr int NPB = NB / 8;  // k-step pairs per row block
  constexpr int RING = S * 2 * (2 * (NB / 16) + CTS) * 128;
  constexpr int RL_DOUBLES = NB * C > RING ? NB * C : RING;
  static_assert(RT == 2 && 2 * WR == NB / 16, "the diagonal steps deal two row tiles to each wave row");
  __shared__ __attribute__((aligned(16))) double Rl[RL_DOUBLES];

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

  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  const int wr = wave / WC, wc = wave % WC;
  const int wr_rows = wr * RW, wc_tile = wc * CT;
  const int64_t col_base = slab * C + wc * CW;

  // a split last block: as in k_trsm, its sum grows pair by pair
  // (last_block_sum, wave w: column tile w) and k_trsm_last does the rest
  static_assert(CTS == WR * WC, "one column tile of the last block's sum per wave");
  const bool split = last_block_split(n, K, LAST_RW);
  const bool last_two_tiles = last_block_tiles(n, K) == 2;
  const int Kmain = split ? K - 1 : K;
  for (int k = 0; k < Kmain; k += 2) {
    const bool two = k + 1 < Kmain;  // a lone last block: its partner's GEMM rows are discarded
    PHASE_STAMP(k / 2, 0);
    d4 acc0[RT][CT], acc1[RT][CT];
#pragma unroll
    for (int a = 0; a < RT; a++)
#pragma unroll
      for (int b = 0; b < CT; b++) acc0[a][b] = acc1[a][b] = (d4){0, 0, 0, 0};
    const int npairs = k * NPB;
    if (npairs > 0)
      gemm_staged_pair<C, WR, WC, S>(Lstrips + strip_offset(k), Lstrips + strip_offset(two ? k + 1 : k), Wslab,
                                     npairs, Rl, acc0, acc1);
    PHASE_STAMP(k / 2, 1);

    // int8 right-hand sides: both blocks' at once, so that block k+1's
    // arrives with block k's, which the staging below waits for anyway
    // (issued later, any wait for a load issued after them would wait for
    // them too; unused for a lone last block).  FP64 ones (8 times the
    // registers) are loaded one block at a time.
    constexpr bool kEarly = sizeof(TIn) == 1;
    TIn xv0[RT][CT][4], xv1[RT][CT][4];
    load_rhs<RT, CT>(X, ldx, n, ncols, (int64_t)k * NB + wr_rows, col_base, lane, xv0);
    if (kEarly) load_rhs<RT, CT>(X, ldx, n, ncols, (int64_t)(k + 1) * NB + wr_rows, col_base, lane, xv1);
    d2 pa[DIAG_PF];
    DIAG_BY_ROW(diag_prefetch<WROW>(LinvP, k, lane, pa));

    // block k: R_k to LDS, W_k = inv(L_kk) R_k, stored (and, when block
    // k+1 follows, put in LDS in place of R_k once every wave is done
    // reading R_k)
    to_pair_layout<RT, CT, CTS>(Rl, wr_rows, wc_tile, lane, xv0, acc0, true);
    __syncthreads();
    DIAG_BY_ROW((diag_step_dealt<CT, CTS, WROW>(LinvP, k, Rl, wc_tile, lane, pa, acc0)));
    if (two) __syncthreads();
    store_w_dealt<CT, CTS>(Wslab, two ? Rl : nullptr, k, wr, wc_tile, lane, acc0);
    PHASE_STAMP(k / 2, 2);
    if (two) {
      // acc_{k+1} += L_{k+1,k} W_k: the last NPB pairs of strip k+1 (from
      // global memory, D pairs ahead) against W_k (from LDS, one pair ahead)
      constexpr int D = 4;
      const double* __restrict__ Ls =
          Lstrips + strip_offset(k + 1) + (size_t)k * NPB * (NB / 16) * 128 + (size_t)(wr * RT) * 128 + lane * 2;
      d2 a[NPB][RT], b[2][CT];
#pragma unroll
      for (int s = 0; s < D; s++)
#pragma unroll
        for (int rt = 0; rt < RT; rt++) a[s][rt] = *reinterpret_cast<const d2*>(Ls + ((size_t)s * (NB / 16) + rt) * 128);
      if (!kEarly) {
        asm volatile("" ::: "memory");  // (after the first pairs of L, so that waiting for those does not wait for it)
        load_rhs<RT, CT>(X, ldx, n, ncols, (int64_t)(k + 1) * NB + wr_rows, col_base, lane, xv1);
      }
      __syncthreads();
      auto read_b = [&](int kp, d2 (&bb)[CT]) {
#pragma unroll
        for (int ct = 0; ct < CT; ct++)
          bb[ct] = *reinterpret_cast<const d2*>(&Rl[((size_t)kp * CTS + wc_tile + ct) * 128 + lane * 2]);
      };
      read_b(0, b[0]);
#pragma unroll
      for (int kp = 0; kp < NPB; kp++) {
        if (kp + D < NPB) {
#pragma unroll
          for (int rt = 0; rt < RT; rt++)
            a[kp + D][rt] = *reinterpret_cast<const d2*>(Ls + ((size_t)(kp + D) * (NB / 16) + rt) * 128);
        }
        if (kp + 1 < NPB) read_b(kp + 1, b[(kp + 1) % 2]);
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
#pragma unroll
          for (int ct = 0; ct < CT; ct++) {
            acc1[rt][ct] = MFMA64(a[kp][rt].x, b[kp % 2][ct].x, acc1[rt][ct]);
            acc1[rt][ct] = MFMA64(a[kp][rt].y, b[kp % 2][ct].y, acc1[rt][ct]);
          }
        // the loads first, then the MFMAs (as in diag_step_dealt)
        if (kp + D < NPB) __builtin_amdgcn_sched_group_barrier(0x020, RT, 0);
        if (kp + 1 < NPB) __builtin_amdgcn_sched_group_barrier(0x100, CT, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 2 * RT * CT, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
      PHASE_STAMP(k / 2, 3);
      // block k+1: R_{k+1} replaces W_k in LDS once every wave is done
      // reading it
      DIAG_BY_ROW(diag_prefetch<WROW>(LinvP, k + 1, lane, pa));
      __syncthreads();
      to_pair_layout<RT, CT, CTS>(Rl, wr_rows, wc_tile, lane, xv1, acc1, true);
      __syncthreads();
      DIAG_BY_ROW((diag_step_dealt<CT, CTS, WROW>(LinvP, k + 1, Rl, wc_tile, lane, pa, acc1)));
      store_w_dealt<CT, CTS>(Wslab, nullptr, k + 1, wr, wc_tile, lane, acc1);
      PHASE_STAMP(k / 2, 4);
    }
    // the W stores are visible to the work-group's next copies (and to the
    // last block's sum), and every wave is done reading Rl before the next
    // stage ring overwrites it
    __threadfence_block();
    __syncthreads();
    if (split) {
      if (last_two_tiles) {
        if (two) last_block_sum<CTS, 2, 2, 8>(Lstrips, Wslab, K, k, 0, wave, lane);
        else last_block_sum<CTS, 2, 1, 8>(Lstrips, Wslab, K, k, 0, wave, lane);
      } else {
        if (two) last_block_sum<CTS, 1, 2, 16>(Lstrips, Wslab, K, k, 0, wave, lane);
        else last_block_sum<CTS, 1, 1, 16>(Lstrips, Wslab, K, k, 0, wave, lane);
      }
    }
    PHASE_STAMP(k / 2, 5);
  }
}

// The last row block of every slab when last_block_split holds, after the
// walk (same grid, one work-group per slab): R = X - acc for its real row
// tiles, acc being the off-diagonal sum that last_block_sum left in the
// slab's rows of the block, zero for every other row; then the diagonal
// step W = inv(L_kk) R and the store, as in k_trsm (rows past the real ones
// come out zero, as padding must).  Four wave rows of NB / 4 rows, WC wave
// columns.
template <int C, int WC, typename TIn = int8_t>
__global__ __launch_bounds__(256 * WC) void k_trsm_last(const JobTable tab) {
  constexpr int WR = 4, RW = NB / WR, RT = RW / 16;
  constexpr int CW = C / WC, CT = CW / 16;
  constexpr int CTS = C / 16;
  constexpr int NPB = NB / 8;
  __shared__ __attribute__((aligned(16))) double Rl[NB * C];

  int jb = 0;
  while (jb + 1 < tab.njobs && (int64_t)blockIdx.x >= tab.j[jb + 1].slab0) jb++;
  const JobDesc& J = tab.j[jb];
  const int K = J.K;
  if (!last_block_split(J.n, K, LAST_RW)) return;
  const int k = K - 1;
  const int lt_end = last_block_tiles(J.n, K);
  const int64_t slab = (int64_t)blockIdx.x - J.slab0;
  const TIn* __restrict__ X = reinterpret_cast<const TIn*>(J.X);
  double* __restrict__ Wslab = J.W + slab * (int64_t)K * NB * C;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64), lane = threadIdx.x % 64;
  const int wr = wave / WC, wc = wave % WC;
  const int64_t col_base = slab * C + wc * CW;

  // R_k into LDS in the B-operand pair layout: the first wave row's real
  // tiles x - acc, everything else zero (the sum of a tile past the real
  // ones was never formed: its slab rows are not read into R)
#pragma unroll
  for (int rt = 0; rt < RT; rt++) {
    const int rowl = wr * RW + rt * 16;
    const bool real = wr == 0 && rt < lt_end;
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int i = 0; i < 4; i += 2) {
        const int kp = (rowl / 4 + i) / 2;
        const int64_t col = col_base + ct * 16 + lane % 16;
        const int64_t row = (int64_t)k * NB + rowl + lane / 16 + 4 * i;
        const d2 acc = *reinterpret_cast<const d2*>(
            Wslab + ((size_t)(k * NPB + kp) * CTS + wc * CT + ct) * 128 + lane * 2);
        const double x0 = load_x<TIn>(X, J.ldx, row, col, J.n, J.ncols);
        const double x1 = load_x<TIn>(X, J.ldx, row + 4, col, J.n, J.ncols);
        *reinterpret_cast<d2*>(&Rl[((size_t)kp * CTS + wc * CT + ct) * 128 + lane * 2]) =
            real ? (d2){x0 - acc.x, x1 - acc.y} : (d2){0.0, 0.0};
      }
  }
  __syncthreads();
  // W_k = inv(L_kk) R_k and the store, as in k_trsm
  d4 w[RT][CT];
#pragma unroll
  for (int a = 0; a < RT; a++)
#pragma unroll
    for (int b = 0; b < CT; b++) w[a][b] = (d4){0, 0, 0, 0};
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
        w[rt][ct] = MFMA64(a[rt].x, b[ct].x, w[rt][ct]);
        w[rt][ct] = MFMA64(a[rt].y, b[ct].y, w[rt][ct]);
      }
  }
  // (the stores land on the acc tiles, which every wave read before the
  // barrier above)
#pragma unroll
  for (int rt = 0; rt < RT; rt++) {
    const int64_t ks0 = (int64_t)k * (NB / 4) + (wr * RW + rt * 16) / 4;
#pragma unroll
    for (int ct = 0; ct < CT; ct++)
#pragma unroll
      for (int i = 0; i < 4; i += 2)
        *reinterpret_cast<d2*>(Wslab + ((size_t)((ks0 + i) / 2) * CTS + wc * CT + ct) * 128 + lane * 2) =
            (d2){w[rt][ct][i], w[rt][ct][i + 1]};
  }
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


hipError_t launch_trsm_i8(const JobTable& tab, int64_t nslabs, int C, hipStream_t st) {
  // the last row block goes to k_trsm_last when some job of the table wants it
  bool last = false;
  for (int i = 0; i < tab.njobs; i++) last = last || last_block_split(tab.j[i].n, tab.j[i].K, LAST_RW);
  switch (C) {
    case 16:
      // 8 waves of 16 x 16 tiles, so that a slab walks its row blocks with
      // two waves per SIMD (one wave per SIMD issues FP64 MFMAs at about half
      // rate); a wave's pair of MFMAs is short, so 8 pairs are kept in flight
      k_trsm<16, 8, 1, 8, int8_t><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      if (last) k_trsm_last<16, 1><<<(unsigned)nslabs, 256, 0, st>>>(tab);
      break;
    case 32:
      k_trsm<32, 4, 2, TRSM_DEPTH, int8_t><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      if (last) k_trsm_last<32, 2><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      break;
    case 64:
      k_trsm<64, 4, 2, TRSM_DEPTH, int8_t, 2, 4><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      if (last) k_trsm_last<64, 2><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      break;
    case 128:
      // row blocks in pairs: half the W re-reads of k_trsm (4.8% faster
      // than k_trsm's sixteen waves of 32 x 32 tiles, same bits)
      k_trsm_pair<128, int8_t><<<(unsigned)nslabs, 64 * PAIR_WR * PAIR_WC, 0, st>>>(tab);
      if (last) k_trsm_last<128, 2><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The same solve for FP64 right-hand sides (whole design matrices, as the
// per-problem trsm of Alg. 3 and Alg. 4 whitens them): 16-, 64- and
// 128-column slabs.
hipError_t launch_trsm_f64(const JobTable& tab, int64_t nslabs, int C, hipStream_t st) {
  bool last = false;
  for (int i = 0; i < tab.njobs; i++) last = last || last_block_split(tab.j[i].n, tab.j[i].K, LAST_RW);
  switch (C) {
    case 16:
      k_trsm<16, 8, 1, 8, double><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      if (last) k_trsm_last<16, 1, double><<<(unsigned)nslabs, 256, 0, st>>>(tab);
      break;
    case 64:
      k_trsm<64, 4, 2, TRSM_DEPTH, double, 2, 4><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      if (last) k_trsm_last<64, 2, double><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      break;
    case 128:
      k_trsm_pair<128, double><<<(unsigned)nslabs, 64 * PAIR_WR * PAIR_WC, 0, st>>>(tab);
      if (last) k_trsm_last<128, 2, double><<<(unsigned)nslabs, 512, 0, st>>>(tab);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_slab_to_colmajor(const double* W, int C, int64_t n_pad, int64_t n, int64_t col0,
                                   int64_t ncols, double* out, int64_t ldo, hipStream_t st) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)(ncols < 65535 ? ncols : 65535));
  k_slab_to_colmajor<<<grid, 256, 0, st>>>(W, C, n_pad, n, col0, ncols, out, ldo);
  return hipGetLastError();
}

}  // namespace gls
