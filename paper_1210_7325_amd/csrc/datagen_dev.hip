// Synthetic genotypes generated on the device: the GPU twin of datagen.c
// (same counter-based splitmix64 draws, same IEEE double operations in the
// same order, no contraction), so column j is bit-identical to the host
// generator's.  Input generation only; none of the GLS method's arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

__device__ __host__ static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

__device__ static inline double unit_draw(uint64_t ckey, uint64_t i) {
  return (double)(mix64(ckey + (i + 1) * GOLDEN) >> 11) * 0x1.0p-53;
}

// One thread per 4 consecutive individuals of one column.
__global__ void k_gen_genotypes(uint64_t skm, uint64_t skg, double lo, double span, int64_t n,
                                int64_t col0, int64_t ncols, int8_t* __restrict__ out, int64_t ld) {
  const int64_t j = blockIdx.y + (int64_t)gridDim.y * blockIdx.z;
  if (j >= ncols) return;
  const int64_t r0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  if (r0 >= n) return;
  const uint64_t col = (uint64_t)(col0 + j);
  const double f = __dadd_rn(lo, __dmul_rn(span, unit_draw(mix64(skm ^ ((col + 1) * GOLDEN)), 0)));
  const uint64_t ck = mix64(skg ^ ((col + 1) * GOLDEN));
  int8_t* o = out + j * ld;
  for (int e = 0; e < 4 && r0 + e < n; e++) {
    const uint64_t r = (uint64_t)(r0 + e);
    const double u1 = unit_draw(ck, 2 * r), u2 = unit_draw(ck, 2 * r + 1);
    o[r] = (int8_t)((u1 < f) + (u2 < f));
  }
}

extern "C" int gen_genotypes_dev(uint64_t seed, uint64_t stream_maf, uint64_t stream_g, double lo,
                                 double hi, int64_t n, int64_t col0, int64_t ncols, int8_t* out,
                                 int64_t ld, void* stream) {
  if (n < 0 || ncols < 0 || ld < n || (!out && ncols > 0)) return -1;
  if (ncols == 0 || n == 0) return 0;
  const uint64_t skm = mix64(mix64(seed) + stream_maf);
  const uint64_t skg = mix64(mix64(seed) + stream_g);
  const double span = hi - lo;
  const int64_t ythreads = (n + 3) / 4;
  const int64_t gy = ncols < 65535 ? ncols : 65535;
  const int64_t gz = (ncols + gy - 1) / gy;
  dim3 grid((unsigned)((ythreads + 255) / 256), (unsigned)gy, (unsigned)gz);
  k_gen_genotypes<<<grid, 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(
      skm, skg, lo, span, n, col0, ncols, out, ld);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}
