// Issue-rate measurement behind the solves' ceilings: throughput of
// v_mfma_f32_16x16x4f32 when each MFMA is followed by NV independent VALU
// instructions of one kind in the same wave (FP32 FMA, FP64 add, FP32 to
// FP64 conversion, FP32 add), and of a plain v_mfma_f64_16x16x4f64 stream,
// with one or two waves per SIMD.  The
// mixed-precision solve folds every FP32 chunk into its FP64 running sum
// with one conversion and one FP64 add per accumulator element, i.e. two
// such VALU instructions per MFMA; this program measures what that mix can
// reach on the device.  Built by the package's build step; prints one line
// per setting.  Not part of the library.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

typedef float f4 __attribute__((ext_vector_type(4)));

#define CHK(x)                                                              \
  do {                                                                      \
    hipError_t e_ = (x);                                                    \
    if (e_ != hipSuccess) {                                                 \
      std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));          \
      std::exit(1);                                                         \
    }                                                                       \
  } while (0)

// Eight independent accumulators; each MFMA is followed by NV VALU
// instructions (written as inline asm so that the compiler keeps their
// number and order; they read and write only their own registers).
template <int MODE, int NV>
__global__ __launch_bounds__(512) void k_mix(float* out, int iters) {
  f4 c[8];
  for (int i = 0; i < 8; i++) c[i] = (f4){0, 0, 0, 0};
  const float a = threadIdx.x * 1e-3f, b = 1.0f + blockIdx.x * 1e-6f;
  float fx[8];
  double dx[8];
  for (int i = 0; i < 8; i++) {
    fx[i] = a + i;
    dx[i] = b + i;
  }
  const float fy = 1.0000001f;
  const double dy = 1.0000000001;
  if (MODE == 5) {
    // FP64 MFMAs only: eight independent 16 x 16 FP64 accumulators
    typedef double d4v __attribute__((ext_vector_type(4)));
    d4v e[8];
    for (int i = 0; i < 8; i++) e[i] = (d4v){0, 0, 0, 0};
    const double da = a, db = b;
    for (int it = 0; it < iters; it++) {
#pragma unroll
      for (int t = 0; t < 8; t++)
        asm volatile("v_mfma_f64_16x16x4_f64 %0, %1, %2, %0" : "+v"(e[t]) : "v"(da), "v"(db));
    }
    asm volatile("s_nop 7\n s_nop 7\n s_nop 7\n s_nop 7" ::: "memory");
    double sum = 0;
    for (int i = 0; i < 8; i++) sum += e[i][0] + e[i][1] + e[i][2] + e[i][3];
    out[blockIdx.x * blockDim.x + threadIdx.x] = (float)sum;
    return;
  }
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int t = 0; t < 8; t++) {
      asm volatile("v_mfma_f32_16x16x4_f32 %0, %1, %2, %0" : "+v"(c[t]) : "v"(a), "v"(b));
#pragma unroll
      for (int v = 0; v < NV; v++) {
        const int j = (t * NV + v) % 8;
        if (MODE == 1) asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(fx[j]) : "v"(fy));
        if (MODE == 2) asm volatile("v_add_f64 %0, %0, %1" : "+v"(dx[j]) : "v"(dy));
        if (MODE == 3) asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(dx[j]) : "v"(fx[j]));
        if (MODE == 4) asm volatile("v_add_f32 %0, %0, %1" : "+v"(fx[j]) : "v"(fy));
      }
    }
  }
  // the last MFMAs' results are complete before they are read below
  asm volatile("s_nop 7\n s_nop 7\n s_nop 7" ::: "memory");
  float s = 0;
  for (int i = 0; i < 8; i++) s += c[i][0] + c[i][1] + c[i][2] + c[i][3] + fx[i] + (float)dx[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

static const char* kind(int mode) {
  switch (mode) {
    case 0: return "none";
    case 5: return "(FP64 MFMA)";
    case 1: return "v_fma_f32";
    case 2: return "v_add_f64";
    case 3: return "v_cvt_f64_f32";
    default: return "v_add_f32";
  }
}

template <int MODE, int NV>
static void run(int threads, int grid, float* out, int iters) {
  hipEvent_t e0, e1;
  CHK(hipEventCreate(&e0));
  CHK(hipEventCreate(&e1));
  k_mix<MODE, NV><<<grid, threads>>>(out, iters);  // warm-up
  CHK(hipGetLastError());
  CHK(hipDeviceSynchronize());
  CHK(hipEventRecord(e0));
  k_mix<MODE, NV><<<grid, threads>>>(out, iters);
  CHK(hipGetLastError());
  CHK(hipEventRecord(e1));
  CHK(hipEventSynchronize(e1));
  float ms = 0;
  CHK(hipEventElapsedTime(&ms, e0, e1));
  const double mfma = (double)grid * (threads / 64) * iters * 8;
  std::printf("valu %-14s per_mfma %d waves_per_simd %d: %.3f ms, %.1f TFLOP/s of %s MFMA\n",
              kind(MODE), NV, threads / 256, ms, mfma * 2048 / (ms * 1e-3) / 1e12,
              MODE == 5 ? "FP64" : "FP32");
  CHK(hipEventDestroy(e0));
  CHK(hipEventDestroy(e1));
}

int main() {
  int dev = 0, cus = 0;
  CHK(hipGetDevice(&dev));
  CHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int grid = 4 * cus, iters = 2000;
  float* out = nullptr;
  CHK(hipMalloc(&out, sizeof(float) * (size_t)grid * 512));
  for (int threads : {256, 512}) {
    run<5, 0>(threads, grid, out, iters / 2);
    run<0, 0>(threads, grid, out, iters);
    run<1, 1>(threads, grid, out, iters);
    run<1, 2>(threads, grid, out, iters);
    run<1, 4>(threads, grid, out, iters);
    run<2, 1>(threads, grid, out, iters);
    run<2, 2>(threads, grid, out, iters);
    run<2, 4>(threads, grid, out, iters);
    run<3, 1>(threads, grid, out, iters);
    run<3, 2>(threads, grid, out, iters);
    run<4, 1>(threads, grid, out, iters);
    run<4, 2>(threads, grid, out, iters);
    run<4, 4>(threads, grid, out, iters);
  }
  CHK(hipFree(out));
  return 0;
}
