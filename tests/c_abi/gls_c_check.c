/*
 * Drives libgls through its C ABI alone (include/gls.h, plain device
 * pointers from hipMalloc, no Python, no torch) and checks the results on
 * the host.  Test infrastructure: built by the package's build step, run by
 * tests/test_gpu_c_abi.py.
 *
 * The problem (Sec. 1, Eq. (1)): b_i = (X_i^T M^-1 X_i)^-1 X_i^T M^-1 y with
 * X_i = (X_L | x_i), M = A A^T / q + I (A n x q with entries in {-1, 0, 1}),
 * X_L = (1 | covariate), genotypes x_i in {0, 1, 2}, all from a fixed
 * linear congruential sequence.  The host reference is the definition
 * written out with a plain Cholesky factor of M (FP64): V = M^-1 [X_L y x_i]
 * by forward and back substitution, then the p x p normal equations solved
 * by Gaussian elimination with partial pivoting.  It prints the largest
 * relative error (max norm per problem) and exits 0 when it is below 1e-10.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "gls.h"

enum { N = 300, Q = 600, PL = 2, T = 1, M_SNP = 97, P = PL + 1 };

static uint64_t lcg_state = 12107325u;
static double unif(void) { /* in [0, 1) */
  lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

#define CHECK_HIP(x)                                                  \
  do {                                                                \
    hipError_t e_ = (x);                                              \
    if (e_ != hipSuccess) {                                           \
      fprintf(stderr, "HIP error %d at line %d\n", (int)e_, __LINE__); \
      return 2;                                                       \
    }                                                                 \
  } while (0)
#define CHECK_GLS(x)                                                            \
  do {                                                                          \
    int r_ = (x);                                                               \
    if (r_ != 0) {                                                              \
      fprintf(stderr, "gls error %d (%s) at line %d\n", r_, gls_strerror(r_), __LINE__); \
      return 3;                                                                 \
    }                                                                           \
  } while (0)

/* lower Cholesky factor in place (column-major, n x n); 0 on success */
static int host_cholesky(double* a, int n) {
  for (int j = 0; j < n; j++) {
    double d = a[j + j * n];
    for (int k = 0; k < j; k++) d -= a[j + k * n] * a[j + k * n];
    if (!(d > 0.0)) return 1;
    d = sqrt(d);
    a[j + j * n] = d;
    for (int i = j + 1; i < n; i++) {
      double v = a[i + j * n];
      for (int k = 0; k < j; k++) v -= a[i + k * n] * a[j + k * n];
      a[i + j * n] = v / d;
    }
  }
  return 0;
}

/* x := M^-1 x with M = L L^T */
static void host_solve(const double* l, int n, double* x) {
  for (int i = 0; i < n; i++) {
    double v = x[i];
    for (int k = 0; k < i; k++) v -= l[i + k * n] * x[k];
    x[i] = v / l[i + i * n];
  }
  for (int i = n - 1; i >= 0; i--) {
    double v = x[i];
    for (int k = i + 1; k < n; k++) v -= l[k + i * n] * x[k];
    x[i] = v / l[i + i * n];
  }
}

/* solve the p x p system a z = r (row-major a), partial pivoting */
static void small_solve(double a[P][P], double r[P], double z[P]) {
  for (int c = 0; c < P; c++) {
    int piv = c;
    for (int i = c + 1; i < P; i++)
      if (fabs(a[i][c]) > fabs(a[piv][c])) piv = i;
    for (int j = 0; j < P; j++) {
      double tmp = a[c][j];
      a[c][j] = a[piv][j];
      a[piv][j] = tmp;
    }
    double tmp = r[c];
    r[c] = r[piv];
    r[piv] = tmp;
    for (int i = c + 1; i < P; i++) {
      const double f = a[i][c] / a[c][c];
      for (int j = c; j < P; j++) a[i][j] -= f * a[c][j];
      r[i] -= f * r[c];
    }
  }
  for (int i = P - 1; i >= 0; i--) {
    double v = r[i];
    for (int j = i + 1; j < P; j++) v -= a[i][j] * z[j];
    z[i] = v / a[i][i];
  }
}

int main(void) {
  double* A = malloc(sizeof(double) * N * Q);
  double* Mh = malloc(sizeof(double) * N * N);
  double* L = malloc(sizeof(double) * N * N);
  double XL[N * PL], Y[N * T];
  int8_t* XR = malloc((size_t)N * M_SNP);
  double B[M_SNP * T * P];
  int32_t info[M_SNP];
  for (int i = 0; i < N * Q; i++) A[i] = floor(unif() * 3.0) - 1.0;
  for (int j = 0; j < N; j++)
    for (int i = 0; i < N; i++) {
      double v = 0.0;
      for (int k = 0; k < Q; k++) v += A[i + k * N] * A[j + k * N];
      Mh[i + j * N] = v / Q + (i == j ? 1.0 : 0.0);
    }
  for (int i = 0; i < N; i++) {
    XL[i] = 1.0;
    XL[i + N] = unif() * 2.0 - 1.0;
    Y[i] = unif() * 2.0 - 1.0;
  }
  for (int i = 0; i < N * M_SNP; i++) XR[i] = (int8_t)(unif() < 0.3) + (int8_t)(unif() < 0.3);

  /* the device side, through the ABI only */
  double *dM, *dXL, *dY, *dB;
  int8_t* dXR;
  int32_t* dinfo;
  CHECK_HIP(hipMalloc((void**)&dM, sizeof(double) * N * N));
  CHECK_HIP(hipMalloc((void**)&dXL, sizeof(double) * N * PL));
  CHECK_HIP(hipMalloc((void**)&dY, sizeof(double) * N * T));
  CHECK_HIP(hipMalloc((void**)&dXR, (size_t)N * M_SNP));
  CHECK_HIP(hipMalloc((void**)&dB, sizeof(double) * M_SNP * T * P));
  CHECK_HIP(hipMalloc((void**)&dinfo, sizeof(int32_t) * M_SNP));
  CHECK_HIP(hipMemcpy(dM, Mh, sizeof(double) * N * N, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dXL, XL, sizeof(double) * N * PL, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dY, Y, sizeof(double) * N * T, hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(dXR, XR, (size_t)N * M_SNP, hipMemcpyHostToDevice));
  gls_handle h = NULL;
  CHECK_GLS(gls_factor(&h, N, dM, N, GLS_FP64, NULL));
  CHECK_GLS(gls_whiten_fixed(h, PL, dXL, N, T, dY, N, 0));
  CHECK_GLS(gls_solve_block(h, M_SNP, 1, dXR, N, dB, P, dinfo));
  CHECK_HIP(hipDeviceSynchronize());
  CHECK_HIP(hipMemcpy(B, dB, sizeof(B), hipMemcpyDeviceToHost));
  CHECK_HIP(hipMemcpy(info, dinfo, sizeof(info), hipMemcpyDeviceToHost));
  gls_free(h);

  /* the host reference: Eq. (1) by its definition */
  memcpy(L, Mh, sizeof(double) * N * N);
  if (host_cholesky(L, N)) {
    fprintf(stderr, "host Cholesky failed\n");
    return 4;
  }
  double* V = malloc(sizeof(double) * N * (P + 1));
  double worst = 0.0;
  for (int s = 0; s < M_SNP; s++) {
    if (info[s] != 0) {
      fprintf(stderr, "problem %d: info %d\n", s, info[s]);
      return 5;
    }
    /* columns of X_i, then y */
    for (int i = 0; i < N; i++) {
      V[i] = XL[i];
      V[i + N] = XL[i + N];
      V[i + 2 * N] = XR[i + s * N];
      V[i + 3 * N] = Y[i];
    }
    double X[N * P];
    memcpy(X, V, sizeof(X));
    for (int c = 0; c < P + 1; c++) host_solve(L, N, V + c * N);
    double S[P][P], r[P], b[P];
    for (int a = 0; a < P; a++) {
      for (int c = 0; c < P; c++) {
        double v = 0.0;
        for (int i = 0; i < N; i++) v += X[i + a * N] * V[i + c * N];
        S[a][c] = v;
      }
      double v = 0.0;
      for (int i = 0; i < N; i++) v += X[i + a * N] * V[i + P * N];
      r[a] = v;
    }
    small_solve(S, r, b);
    double num = 0.0, den = 0.0;
    for (int a = 0; a < P; a++) {
      num = fmax(num, fabs(B[s * T * P + a] - b[a]));
      den = fmax(den, fabs(b[a]));
    }
    worst = fmax(worst, num / den);
  }
  printf("c-abi check: n=%d p=%d m=%d max rel err %.3e\n", N, P, M_SNP, worst);
  free(A);
  free(Mh);
  free(L);
  free(XR);
  free(V);
  hipFree(dM);
  hipFree(dXL);
  hipFree(dY);
  hipFree(dXR);
  hipFree(dB);
  hipFree(dinfo);
  return worst < 1e-10 ? 0 : 1;
}
