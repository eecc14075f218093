/*
 * gls.h - C ABI of the MI355X solver for sequences of generalized
 * least-squares problems (Fabregat-Traver, Aulchenko, Bientinesi,
 * "Solving Sequences of Generalized Least-Squares Problems on
 * Multi-threaded Architectures").
 *
 * The library computes, for i = 1..m (Sec. 1, Eq. (1)),
 *
 *     b_i = (X_i^T M^{-1} X_i)^{-1} X_i^T M^{-1} y,   X_i = (X_L | X_{R_i}),
 *
 * following the structure of the paper's in-core algorithm (Sec. 2, the
 * algorithm "hp-gwas"): M = L L^T is factored once, the fixed block X_L
 * and y are whitened once, each block of genotype columns is whitened by
 * one large triangular solve, and the small SPD systems S_i b_i = c_i of
 * size p = p_L + p_R are assembled from the fixed and per-problem parts
 * (Fig. 1) and solved.
 *
 * Conventions (all entry points):
 *  - Every array pointer is a DEVICE pointer, column-major, owned by the
 *    caller.  The library never writes to an input and never frees
 *    caller memory.
 *  - A handle (gls_handle) is opaque and owns device memory: the factor
 *    of M in the kernels' packed layouts, the whitened fixed block and its
 *    products, and a workspace for whitened genotype columns.
 *  - Work is enqueued on the handle's HIP stream (hipStream_t passed as
 *    void*; NULL = the null stream).  Unless stated otherwise a call only
 *    enqueues work: inputs must stay alive, and outputs are valid, once
 *    the stream has passed the call.
 *  - Return codes: 0 success; -k argument k (1-based) invalid; positive
 *    values are the GLS_E_* codes below.  No exception crosses the ABI.
 *  - A handle is not thread-safe.  Distinct handles (also those made by
 *    gls_fork) may be used concurrently on distinct streams.
 *  - Limits: n > p (Sec. 2: X of full rank with n > p), 1 <= p_L,
 *    1 <= p_R, p = p_L + p_R <= 20 (Sec. 1), 1 <= t <= 8 phenotypes.
 */
#ifndef GLS_H
#define GLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gls_handle_s* gls_handle;

/* Arithmetic of the genotype whitening.
 * GLS_FP64: every step in FP64.  Max relative error of b_i (per problem and
 *   phenotype, max-norm) against the FP64 definition: ~3e-14 at the
 *   workloads' conditioning; the target is 1e-10.
 * GLS_FP32_REFINE: the off-diagonal products of the triangular solve in
 *   FP32 matrix cores (FP32 sums over 32 k-values, each two FP32 chains
 *   of 16 added in FP32, then an FP64 running sum), everything else in
 *   FP64, and one FP64 refinement step of the
 *   normal equations per problem.  Not part of the paper, whose routines
 *   are FP64 only.  The FP32-rounded operands leave an error that grows
 *   with kappa(L) = sqrt(kappa(M)) and that the refinement cannot remove
 *   where it enters X_R^T M^-1 X_R, so the stated bound on the max relative
 *   error of b_i depends on the 2-norm condition number of M:
 *       kappa(M) <= 10     1e-8   (measured 3.7e-9 at kappa 3.6)
 *       kappa(M) <= 60     3e-8   (measured 2.4e-8 at kappa 51)
 *       kappa(M) <= 250    6e-8   (measured 4.1e-8 at kappa 209)
 *       kappa(M) <= 1000   1e-7   (measured 4.9e-8 at kappa 799)
 *   (1,000 problems at n = 1,200 each, M = h Phi + (1-h) I + 1e-3 I).  No
 *   bound is stated beyond kappa(M) = 1000: use GLS_FP64 there. */
typedef enum { GLS_FP64 = 0, GLS_FP32_REFINE = 1 } gls_precision;

enum {
  GLS_OK = 0,
  GLS_E_NOT_SPD = 1,     /* gls_factor: M is not positive definite        */
  GLS_E_STATE = 2,       /* call out of order (e.g. solve before whiten)  */
  GLS_E_OOM = 3,         /* device allocation failed                      */
  GLS_E_HIP = 4,         /* a HIP runtime call failed                     */
  GLS_E_UNSUPPORTED = 5, /* valid but unsupported request                 */
  GLS_E_IO = 6,          /* a file could not be opened or read            */
  GLS_E_ABORTED = 7,     /* a stream callback returned nonzero            */
  GLS_E_TOO_LARGE = 8    /* block exceeds gls_solve_block_noalloc's scratch */
};

/* Factor M = L L^T (Cholesky; the potrf of Alg. 3-5, done once per
 * cohort).  M: n x n SPD, leading dimension ldm >= n; only its lower
 * triangle is read.  prec: a gls_precision value.  stream: hipStream_t or
 * NULL.  On success *out receives a new handle bound to `stream`.
 * SYNCHRONOUS: returns after the factorization has finished, so M may be
 * freed on return.  If M is not positive definite the return value is
 * GLS_E_NOT_SPD, *out still receives a handle (to be released with
 * gls_free) and gls_last_info() gives the order of the first non-positive
 * leading minor (LAPACK potrf convention).  Other errors leave *out NULL. */
int gls_factor(gls_handle* out, int64_t n, const double* M, int64_t ldm,
               int prec, void* stream);

/* Whiten the fixed part once (Alg. 5, the trsm of X_L, the trsv of y, the
 * syrk S_TL = W_L^T W_L and the gemv C_T = W_L^T ytil, with W_L = L^{-1} X_L,
 * ytil = L^{-1} y).  X_L: n x p_L (ldx >= n); Y: n x t phenotypes sharing M
 * (ldy >= n).  intercept_col: index of the all-ones column of X_L, or -1;
 * the FP32_REFINE form uses it to center genotypes exactly (it requires
 * one, else GLS_E_UNSUPPORTED).  Asynchronous.  May be called again to
 * replace the fixed part. */
int gls_whiten_fixed(gls_handle h, int64_t p_L, const double* X_L, int64_t ldx,
                     int64_t t, const double* Y, int64_t ldy,
                     int64_t intercept_col);

/* Solve one block of problems (the loop body of Alg. 5 / Alg. 8: one
 * large trsm over the block, then per problem the gemv/dot assembly of
 * S_i and c_i and the posv).  X_R: int8 genotypes, n x (nsnp*p_R),
 * ldxr >= n; problem i owns columns i*p_R .. i*p_R+p_R-1.
 * B: output, element (r, j, i) = component r of b_i for phenotype j at
 * B[(i*t + j)*ldb + r], ldb >= p, components ordered (b_L; b_R) like the
 * columns of X_i.  info: int32[nsnp] or NULL; info[i] = 0, or k > 0 if the
 * k-th leading minor of S_i is not positive (X_i rank deficient), in which
 * case b_i is set to NaN.  Asynchronous; needs gls_whiten_fixed first.
 * The workspace grows (synchronously) when a block is larger than any
 * before; gls_reserve avoids that inside a timed or captured loop. */
int gls_solve_block(gls_handle h, int64_t nsnp, int64_t p_R,
                    const int8_t* X_R, int64_t ldxr, double* B, int64_t ldb,
                    int32_t* info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and results as gls_solve_block, bit for bit, but the
 * whitened-column workspace is a fixed array of GLS_NOALLOC_SCRATCH_BYTES in
 * the library's device code, one per device, held from its first use until
 * the process ends, instead of the handle's own (grown) workspace.  The call
 * allocates and frees nothing.  The block may need at most that many bytes:
 * W is 8 * n_pad * c bytes (n_pad = n rounded up to a multiple of 128,
 * c = nsnp*p_R rounded up to a multiple of 128), and the FP32_REFINE form
 * adds 4 * n_pad * c + 8 * c + 224 * c bytes (each part rounded up to 256
 * bytes); e.g. at n = 10,000 up to 1,536 columns (FP64) or 1,024 (FP32_REFINE).
 * A larger block returns GLS_E_TOO_LARGE before any device work.  The first
 * call on a device looks up the array's address there (hipGetSymbolAddress,
 * with that device made current for the lookup).  Every call on one device
 * uses the same array: calls whose work overlaps on the device (for example
 * on different streams, or from different handles) race and give undefined
 * results; calls ordered on one stream are safe.  Argument checks and the
 * other error codes as gls_solve_block.  Asynchronous on h's stream. */
#define GLS_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int gls_solve_block_noalloc(gls_handle h, int64_t nsnp, int64_t p_R, const int8_t* X_R,
                            int64_t ldxr, double* B, int64_t ldb, int32_t* info);

/* Pre-size the workspace for blocks of up to max_cols = nsnp*p_R genotype
 * columns (rounded up to a multiple of 128).  Synchronous allocation. */
int gls_reserve(gls_handle h, int64_t max_cols);

/* Release the handle and all device memory it owns (after synchronizing
 * its stream).  NULL is ignored.  A factor shared with forked handles is
 * released with the last of them. */
void gls_free(gls_handle h);

/* A new handle that shares h's factor and fixed part (read-only) but has
 * its own workspace and is bound to `stream`, so blocks can be solved
 * concurrently on several streams.  The fixed part must have been set on
 * h before forking.  Synchronizes h's stream once. */
int gls_fork(gls_handle h, void* stream, gls_handle* out);

/* Rebind h to another stream (ordering with the old stream is the
 * caller's business). */
int gls_set_stream(gls_handle h, void* stream);

/* Device bytes a handle holds for a cohort of n individuals, p_L fixed
 * columns, p_R genotype columns per problem, t phenotypes and blocks of up
 * to max_nsnp problems in precision prec (factor, fixed part and workspace;
 * the transient buffer of gls_factor is counted too).  Used for admission
 * by memory footprint.  0 for invalid sizes. */
size_t gls_footprint_bytes(int64_t n, int64_t p_L, int64_t p_R, int64_t t, int64_t max_nsnp,
                           int prec);

/* Order of the first non-positive leading minor found by gls_factor, 0 if
 * none.  Returns -1 for a NULL handle. */
int gls_last_info(gls_handle h);

/* Static description of a return code. */
const char* gls_strerror(int code);

/* ---- inspection ------------------------------------------------------- */

/* Copy L (lower triangle; the strict upper triangle is set to zero) into
 * the caller's n x n device array (ldl >= n).  Asynchronous. */
int gls_copy_factor(gls_handle h, double* L, int64_t ldl);

/* Copy the whitened fixed part: WL n x p_L (ldwl >= n), Yt n x t
 * (ldyt >= n), S_TL p_L x p_L and C_T p_L x t (both packed, ld = p_L).
 * Any pointer may be NULL.  Asynchronous. */
int gls_copy_fixed(gls_handle h, double* WL, int64_t ldwl, double* Yt,
                   int64_t ldyt, double* S_TL, double* C_T);

/* W = L^{-1} X for int8 X (n x ncols, ldx >= n), written to the caller's
 * n x ncols FP64 array (ldw >= n): the genotype whitening step on its own
 * (Alg. 5, the trsm of the X_R block), in the handle's precision.
 * Asynchronous. */
int gls_whiten_block(gls_handle h, int64_t ncols, const int8_t* X, int64_t ldx,
                     double* W, int64_t ldw);

/* W = L^{-1} X for FP64 X (n x ncols, ldx >= n) into the caller's n x ncols
 * FP64 array (ldw >= n): the triangular solve of whole design matrices, as
 * the per-problem trsm of Alg. 3 and Alg. 4 applies it to all p columns of
 * X_i (and as the fixed part's X_L and y are whitened).  FP64 handles only
 * (GLS_E_UNSUPPORTED for GLS_FP32_REFINE).  Same kernels as the genotype
 * solve, with FP64 right-hand sides in 16-, 64- or 128-column slabs (a
 * 32-column setting uses 64).  Asynchronous; grows the workspace like
 * gls_solve_block. */
int gls_whiten_block_f64(gls_handle h, int64_t ncols, const double* X, int64_t ldx, double* W,
                         int64_t ldw);

/* ---- tuning and measurement -------------------------------------------- */

/* Columns of genotypes per work-group of the triangular-solve kernel: 16
 * (FP64 only; GLS_E_UNSUPPORTED in FP32_REFINE), 32, 64 or 128, or 0 (the
 * default) to choose per launch: the narrowest width whose slabs still
 * number at most one per compute unit, else 128 — a slab's walk down the
 * row blocks takes about the same time whatever runs beside it, so small
 * launches finish sooner in narrow slabs and full launches run best in wide
 * ones — except that 64 is kept when a 128-column slab of the launch's
 * largest cohort would take longer than the launch's 64-column slabs spread
 * over the compute units (launches mixing cohorts of different n).  With
 * the automatic width, the work of a gls_solve_block call, or of a
 * gls_solve_multi call whose items share one cohort, that needs more slabs
 * than there are compute units goes out in rounds: one launch of the
 * columns that give one slab per compute unit, then the rest at the width
 * chosen for it (an item may be split between two launches).  Other
 * values return -2.  A performance knob only: every column is
 * whitened by the same sequence of operations whatever its slab, so results
 * are bitwise independent of it.  Items of one gls_solve_multi call must
 * share the setting. */
int gls_set_slab_cols(gls_handle h, int cols);

/* Kernel timing.  While enabled, every launch of the triangular-solve
 * kernel (kind 0) and of the assembly/solve kernel (kind 1) made through h
 * (for gls_solve_multi: through the first item's handle) is bracketed by a
 * pair of HIP events on the stream it is launched on.  Enabling or
 * disabling synchronizes h's stream and clears the record.
 * gls_kernel_time synchronizes on the recorded events and returns the sum
 * of the bracketed durations in milliseconds and the number of launches. */
int gls_set_kernel_timing(gls_handle h, int enable);
int gls_kernel_time(gls_handle h, int kind, double* ms, int64_t* launches);

/* The same record one launch at a time, in launch order.  For each of the
 * first `cap` recorded launches of `kind`: ms[i] its bracketed duration in
 * milliseconds, cols[i] the genotype columns (right-hand sides, nsnp * p_R
 * summed over the launch's work items) it processed, slab[i] its columns
 * per work-group of the triangular solve.  *count receives the number of
 * recorded launches of that kind, which may exceed cap (cap = 0 only counts).
 * The caller owns the three arrays (host memory, cap entries each).
 * Synchronizes on the recorded events of the returned launches.
 * Errors: -1 h NULL, -2 kind not 0 or 1, -3 cap < 0, -4 an array NULL with
 * cap > 0, -7 count NULL, GLS_E_HIP. */
int gls_kernel_launches(gls_handle h, int kind, int64_t cap, double* ms, int64_t* cols, int* slab,
                        int64_t* count);

/* ---- streamed genotypes (out-of-core, Sec. 4, Alg. 8) -------------------
 * Solves problems [snp_begin, snp_end) of h's cohort in blocks of `block`
 * problems whose genotypes live on the host (or on disk) and are produced
 * on demand by `fill`, with double buffering: while block j is solved on
 * h's stream, block j+1 is filled into pinned host memory and copied to the
 * device on a second stream, and the b of block j-1, which the device wrote
 * straight into pinned host memory, is handed to `sink` (Alg. 8: async read
 * of the next block, wait for the current one, compute, async write, wait
 * for the previous).
 * fill(fill_ctx, snp0, nsnp, buf, ld) writes the n x (nsnp*p_R) int8
 *   genotypes of problems snp0.. into pinned host memory buf (column j at
 *   buf + j*ld, ld = n); it returns 0, or nonzero to abort the stream.
 * sink(sink_ctx, snp0, nsnp, b, info) receives host pointers to the
 *   (nsnp, t, p) results and nsnp info codes of those problems, valid during
 *   the call; sinks are called in block order; nonzero aborts.
 * A callback's abort makes the call return GLS_E_ABORTED once the device
 *   work in flight has drained.
 * fill and sink work per block; the device solves superblocks of several
 * consecutive blocks (at least one slab of columns per compute unit per
 * launch), which changes no result bit.
 * snp_begin may be any block boundary of an earlier run: a stream that was
 * aborted resumes after the last block its sink accepted and yields the
 * same bits.  SYNCHRONOUS.  The library allocates (and frees) two pinned
 * input and output buffers, two device input buffers and one stream.
 * stats (nullable) receives wall, fill, sink and wait times. */
typedef int (*gls_fill_fn)(void* fill_ctx, int64_t snp0, int64_t nsnp, int8_t* buf, int64_t ld);
typedef int (*gls_sink_fn)(void* sink_ctx, int64_t snp0, int64_t nsnp, const double* b,
                           const int32_t* info);
typedef struct {
  double wall_ms;       /* whole call                                        */
  double fill_ms;       /* time inside fill                                  */
  double sink_ms;       /* time inside sink                                  */
  double wait_ms;       /* host time blocked on device work (exposed compute) */
  int64_t blocks;
  int64_t bytes_h2d;
  int64_t bytes_d2h;    /* results handed to the host (the assembly writes them
                           straight into pinned host memory)                */
} gls_stream_stats;

int gls_solve_stream(gls_handle h, int64_t snp_begin, int64_t snp_end, int64_t block,
                     int64_t p_R, gls_fill_fn fill, void* fill_ctx, gls_sink_fn sink,
                     void* sink_ctx, gls_stream_stats* stats);

/* ---- genotypes from a file (disk-backed out-of-core, Sec. 4, Alg. 8) ----
 * A ready-made fill callback for gls_solve_stream that reads the genotypes
 * from a file, as the paper's out-of-core algorithm reads the next block
 * from disk while the current one is solved.  The file holds X_R
 * column-major as int8 with leading dimension n: problem s, genotype column
 * q at byte  offset + (s*p_R + q)*n; a block of problems is one contiguous
 * range.  HOST code only (no device work, no HIP call).
 * gls_file_open(out, path, n, p_R, offset, direct, threads) opens path for
 *   reading; with direct != 0 it also opens it with O_DIRECT (page cache
 *   bypassed; pieces whose file offset or length are not multiples of 4096
 *   bytes, and files that refuse direct reads, go through the buffered
 *   descriptor; destinations that refuse direct transfers, such as the
 *   runtime's pinned buffers on some systems, are served through an aligned
 *   bounce buffer per reader).  Each fill splits its range over `threads`
 *   (1..64) reader threads.  Returns 0, a negative argument index, GLS_E_OOM
 *   or GLS_E_IO (cannot open).
 * gls_file_fill has the gls_fill_fn signature (pass the source as fill_ctx);
 *   it requires ld == n and returns nonzero on an I/O error or a read past
 *   the end of the file, which aborts the stream.
 * gls_file_stats reports the bytes read and the wall time spent in fills.
 * gls_file_close closes the file and releases the source (NULL is a no-op).
 * A source may serve one stream at a time. */
typedef struct gls_file_source_s* gls_file_source;
int gls_file_open(gls_file_source* out, const char* path, int64_t n, int64_t p_R, int64_t offset,
                  int direct, int threads);
int gls_file_fill(void* source, int64_t snp0, int64_t nsnp, int8_t* buf, int64_t ld);
int gls_file_stats(gls_file_source src, int64_t* bytes, double* ms);
void gls_file_close(gls_file_source src);

/* ---- results to a file (disk-backed out-of-core, Sec. 4, Alg. 8) --------
 * A ready-made sink callback for gls_solve_stream that writes b (and info)
 * to files asynchronously, the output half of the paper's out-of-core
 * algorithm: the write of a block's results overlaps the solve of the
 * following blocks, and a buffer is reused only once its previous write
 * has completed.  HOST code only (no device work, no HIP call).
 * gls_writer_open(out, b_path, info_path, t, p, snp_base, depth) creates
 *   (or overwrites in place) b_path, where problem s's (t, p) results go at
 *   byte offset (s - snp_base) * t * p * 8 (FP64, phenotype-major within a
 *   problem, the layout of gls_solve_block's B), and info_path (nullable),
 *   where info[s] goes at (s - snp_base) * 4 (int32).  depth (1..64) is the
 *   number of copied blocks that may wait to be written.  Returns 0, a
 *   negative argument index, GLS_E_OOM or GLS_E_IO (cannot create a file).
 * gls_writer_sink has the gls_sink_fn signature (pass the writer as
 *   sink_ctx): it copies the block into a free buffer, waiting while all
 *   depth buffers are still being written, queues the write and returns;
 *   nonzero (which aborts the stream) after a failed write.  Blocks may
 *   come in any order; each lands at its own offset.
 * gls_writer_close drains the queue, flushes both files to the device
 *   (fdatasync), closes them and releases the writer (NULL is a no-op); it
 *   returns GLS_E_IO if any write or the flush failed.  The nullable
 *   outputs receive the bytes written, the time in pwrite, the time sinks
 *   waited for a free buffer and the time of the close itself, in ms.
 * A writer may serve one stream at a time. */
typedef struct gls_file_writer_s* gls_file_writer;
int gls_writer_open(gls_file_writer* out, const char* b_path, const char* info_path, int64_t t,
                    int64_t p, int64_t snp_base, int depth);
int gls_writer_sink(void* writer, int64_t snp0, int64_t nsnp, const double* b, const int32_t* info);
int gls_writer_close(gls_file_writer w, int64_t* bytes, double* write_ms, double* wait_ms,
                     double* close_ms);

/* ---- several cohorts in one launch (serving) ----------------------------
 * One work item per block of problems of one handle.  All items are
 * whitened by one launch of the triangular-solve kernel and assembled and
 * solved by one more (in rounds, as described under gls_set_slab_cols,
 * when the items share one cohort and need more slabs than there are
 * compute units; in launches of at most 16 items otherwise), on `stream`
 * (not the handles' own streams; the caller orders them).  Each item needs its own handle (or fork), because
 * the item uses the handle's workspace.  Results equal gls_solve_block's
 * for the same item bit for bit.  The library records, per handle, the
 * stream of the last launch that used its workspace; growing the workspace
 * (a later, larger block) and gls_free wait for that launch as well as for
 * the handle's own stream.
 * Phenotypes with distinct covariance matrices (the phenotype index of
 * Eq. (1) with its own M_j, e.g. M_j = h_j Phi + (1 - h_j) I): factor each
 * M_j into its own handle, whiten X_L and y_j on it, and pass one item per
 * phenotype whose X_R points at the same genotype block; one launch then
 * solves the block for every phenotype (X_R is only read). */
typedef struct {
  gls_handle h;
  int64_t nsnp;
  int64_t p_R;
  const int8_t* X_R;
  int64_t ldxr;
  double* B;
  int64_t ldb;
  int32_t* info;
} gls_work;

int gls_solve_multi(const gls_work* items, int64_t count, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GLS_H */
