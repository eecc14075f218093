// Host-side internals shared by the translation units of the C ABI.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "gls.h"

namespace gls {

// Device memory a block's launch writes besides its inputs and outputs: the
// whitened columns in the solve's slab layout and, in the FP32_REFINE form,
// their FP32 copy, the per-column centering shifts and products with Z.
struct Workspace {
  double* W;
  float* W32;
  double* shift;
  double* XZ;
};

// Bytes of workspace a block of ncols genotype columns needs on handle h
// (columns rounded up to a multiple of the widest slab, each part aligned
// to 256 bytes).
size_t workspace_bytes(gls_handle h, int64_t ncols);

// The device h's cohort was factored on.
int handle_device(gls_handle h);

// gls_solve_block with the workspace carved out of caller-provided device
// memory (scratch, scratch_bytes) instead of the handle's own: no device
// memory is allocated or freed.  Returns GLS_E_TOO_LARGE when the block needs
// more than scratch_bytes; argument errors as gls_solve_block.
int solve_block_in(gls_handle h, int64_t nsnp, int64_t p_R, const int8_t* X_R, int64_t ldxr,
                   double* B, int64_t ldb, int32_t* info, void* scratch, size_t scratch_bytes);

}  // namespace gls
