// Internal declarations shared by the kernels and the host library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gls {

constexpr int NB = 128;       // row block of the factorization and the solve
constexpr int MAX_C = 128;    // widest slab of genotype columns (16 - 128); workspaces come in multiples of it
constexpr int MAXP = 20;      // p = p_L + p_R <= 20 (Sec. 1)
constexpr int MAXT = 8;       // phenotypes per call
constexpr int MAX_INLINE_JOBS = 16;
constexpr int AS_GROUP_COLS = 64;  // columns per work-group of the assembly and centering kernels
#ifndef GLS_TRSM_DEPTH
#define GLS_TRSM_DEPTH 4
#endif
constexpr int TRSM_DEPTH = GLS_TRSM_DEPTH;  // k-step pairs in flight in the solve's GEMM loop

// One block of columns of one cohort for the triangular-solve kernel.
struct JobDesc {
  int64_t slab0;            // first work-group of this job in the launch
  int64_t n;                // individuals
  int64_t ncols;            // right-hand sides
  const void* X;            // int8 or FP64, column-major
  int64_t ldx;
  const double* Lstrips;    // packed off-diagonal strips of L
  const double* LinvP;      // packed inverted diagonal blocks
  double* W;                // output, slab layout
  int K;                    // row blocks (n_pad / NB)
  // FP32_REFINE form only
  const float* Lstrips32;   // FP32 strips, quad layout
  float* W32;               // FP32 copy of the output for the trailing products, quad layout
  const double* shift;      // per-column centering shift (subtracted from X)
};
struct JobTable {
  int njobs;
  JobDesc j[MAX_INLINE_JOBS];
};

// One block of problems of one cohort for the assembly/solve kernel.
struct AsmDesc {
  int64_t grp0;             // first work-group of this job in the launch
  int64_t n, n_pad;
  const double* W;          // whitened genotypes, slab layout (TRSM_C)
  const double* F;          // row-major n_pad x (pL+t): [W_L | ytil]
  const double* STL;        // pL x pL
  const double* CT;         // pL x t
  int64_t nsnp;
  double* B;
  int64_t ldb;
  int32_t* info;
  int C, pL, pR, t;
  // FP32_REFINE form only
  const double* shift;      // per-column centering shift
  const double* XZ;         // per column: (x - shift)^T [Z_L | Z_y], ld = pL + t
  int icol;                 // intercept column of X_L
};
struct AsmTable {
  int njobs;
  AsmDesc j[MAX_INLINE_JOBS];
};

// Centering pre-pass of the FP32_REFINE form: per genotype column the exact
// dyadic shift s = round(256 mean(x)) / 256 and (x - s)^T Z.
struct XzDesc {
  int64_t grp0;             // first work-group (AS_GROUP_COLS columns each)
  int64_t n;
  int64_t ncols;
  const int8_t* X;
  int64_t ldx;
  const double* Z;          // row-major n_pad x ldf: M^{-1}[X_L | Y]
  const double* z1;         // ldf column sums of Z over its n rows
  double* shift;            // out: ncols
  double* XZ;               // out: ncols x ldf
  int ldf;
};
struct XzTable {
  int njobs;
  XzDesc j[MAX_INLINE_JOBS];
};

hipError_t launch_factor(const double* M, int64_t ldm, int64_t n, int64_t n_pad, int K,
                         double* A, double* Ldiag, double* Linv, double* Lstrips, double* LinvP,
                         float* Lstrips32, int* dinfo, hipStream_t st);
hipError_t launch_unpack_factor(const double* Lstrips, const double* Ldiag, int64_t n, double* L,
                                int64_t ldl, hipStream_t st);
hipError_t launch_trsm_i8(const JobTable& tab, int64_t nslabs, int C, hipStream_t st);
hipError_t launch_trsm_f64(const JobTable& tab, int64_t nslabs, int C, hipStream_t st);
hipError_t launch_slab_to_colmajor(const double* W, int C, int64_t n_pad, int64_t n, int64_t col0,
                                   int64_t ncols, double* out, int64_t ldo, hipStream_t st);
hipError_t launch_fixed_solve(const double* XL, int64_t ldx, const double* Y, int64_t ldy,
                              int64_t n, int64_t n_pad, int K, int pL, int t, const double* Lstrips,
                              const double* LinvP, double* F, double* Z, hipStream_t st);
hipError_t launch_rowmajor_to_colmajor(const double* F, int w, int64_t n, int col0, int ncols,
                                       double* out, int64_t ldo, hipStream_t st);
hipError_t launch_gram(const double* F, int64_t n, int pL, int t, double* STL, double* CT,
                       hipStream_t st);
hipError_t launch_assemble_solve(const AsmTable& tab, int64_t ngroups, bool refine, hipStream_t st);
hipError_t launch_trsm_mixed(const JobTable& tab, int64_t nslabs, int C, hipStream_t st);
hipError_t launch_xz_shift(const XzTable& tab, int64_t ngroups, hipStream_t st);
hipError_t launch_colsum(const double* Z, int64_t n, int ld, double* z1, hipStream_t st);

}  // namespace gls
