/*
 * Synthetic GWAS inputs: counter-based genotype generator (host, OpenMP).
 *
 * This file holds input generation only; it performs none of the GLS
 * method's arithmetic.  It is the C twin of paper_1210_7325_amd/datagen.py
 * and must agree with it bit for bit (same integer hashing, same IEEE
 * double operations in the same order; built with -ffp-contract=off).
 *
 * Random numbers: the splitmix64 output function (Steele, Lea, Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014) applied
 * to a counter.  A draw is addressed by (seed, stream, column, index), so
 * any genotype column can be regenerated independently of block sizes.
 *
 *   K(seed, stream)      = mix64(mix64(seed) + stream)
 *   Kc(seed, stream, j)  = mix64(K ^ ((j + 1) * GOLDEN))
 *   draw(..., i)         = mix64(Kc + (i + 1) * GOLDEN)
 *   uniform              = (draw >> 11) * 2^-53          in [0, 1)
 *
 * Genotype of individual r in column j: g = [u(2r) < f_j] + [u(2r+1) < f_j]
 * ~ Binomial(2, f_j), with the minor-allele frequency
 * f_j = lo + (hi - lo) * u_maf(j) drawn from its own stream.
 */
#include <stdint.h>
#include <stddef.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream) {
  return mix64(mix64(seed) + stream);
}

static inline uint64_t column_key(uint64_t skey, uint64_t col) {
  return mix64(skey ^ ((col + 1) * GOLDEN));
}

static inline double unit_draw(uint64_t ckey, uint64_t i) {
  return (double)(mix64(ckey + (i + 1) * GOLDEN) >> 11) * 0x1.0p-53;
}

/* Minor-allele frequencies of columns col0 .. col0+ncols-1. */
void gen_maf(uint64_t seed, uint64_t stream, double lo, double hi,
             int64_t col0, int64_t ncols, double* out) {
  uint64_t sk = stream_key(seed, stream);
  for (int64_t j = 0; j < ncols; j++) {
    double u = unit_draw(column_key(sk, (uint64_t)(col0 + j)), 0);
    out[j] = lo + (hi - lo) * u;
  }
}

/* Genotype block: out[j*ld + r] for r < n, j < ncols (column-major int8),
 * column index col0 + j, frequencies from gen_maf(seed, stream_maf, lo, hi). */
void gen_genotypes(uint64_t seed, uint64_t stream_maf, uint64_t stream_g,
                   double lo, double hi, int64_t n, int64_t col0,
                   int64_t ncols, int8_t* out, int64_t ld) {
  uint64_t skm = stream_key(seed, stream_maf);
  uint64_t skg = stream_key(seed, stream_g);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < ncols; j++) {
    uint64_t col = (uint64_t)(col0 + j);
    double f = lo + (hi - lo) * unit_draw(column_key(skm, col), 0);
    uint64_t ck = column_key(skg, col);
    int8_t* o = out + j * ld;
    for (int64_t r = 0; r < n; r++) {
      double u1 = unit_draw(ck, 2 * (uint64_t)r);
      double u2 = unit_draw(ck, 2 * (uint64_t)r + 1);
      o[r] = (int8_t)((u1 < f) + (u2 < f));
    }
  }
}

/* Raw uniforms of one stream: out[j*ld + i] = u(seed, stream, col0+j, i). */
void gen_uniforms(uint64_t seed, uint64_t stream, int64_t nidx, int64_t col0,
                  int64_t ncols, double* out, int64_t ld) {
  uint64_t sk = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < ncols; j++) {
    uint64_t ck = column_key(sk, (uint64_t)(col0 + j));
    for (int64_t i = 0; i < nidx; i++) out[j * ld + i] = unit_draw(ck, (uint64_t)i);
  }
}

/* Fill callback for a streamed solve: the genotypes of problems
 * snp0 .. snp0+nsnp-1 (p_R columns each) into buf (column j at buf + j*ld). */
typedef struct {
  uint64_t seed, stream_maf, stream_g;
  double lo, hi;
  int64_t n, p_R;
} gen_fill_ctx;

int gen_fill_genotypes(void* ctx, int64_t snp0, int64_t nsnp, int8_t* buf, int64_t ld) {
  const gen_fill_ctx* c = (const gen_fill_ctx*)ctx;
  gen_genotypes(c->seed, c->stream_maf, c->stream_g, c->lo, c->hi, c->n, snp0 * c->p_R,
                nsnp * c->p_R, buf, ld);
  return 0;
}
