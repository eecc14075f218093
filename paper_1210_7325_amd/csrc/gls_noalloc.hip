// The no-allocation form of gls_solve_block (include/gls.h,
// gls_solve_block_noalloc): the whitened-column workspace lives in a fixed
// device array of this file instead of memory the handle allocates.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gls.h"
#include "gls_host.h"

namespace {

// The scratch array.  In host code its name is a host-side stand-in, not a
// device address; kernels and copies get the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[GLS_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on device dev, looked up once per device with
// that device current (each device holds its own copy of the array).
int scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return GLS_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) {
      (void)hipGetLastError();
      return GLS_E_HIP;
    }
    if (cur != dev && hipSetDevice(dev) != hipSuccess) {
      (void)hipGetLastError();
      return GLS_E_HIP;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return GLS_E_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GLS_OK;
}

}  // namespace

extern "C" int gls_solve_block_noalloc(gls_handle h, int64_t nsnp, int64_t p_R, const int8_t* X_R,
                                       int64_t ldxr, double* B, int64_t ldb, int32_t* info) {
  if (!h) return -1;
  void* ptr = nullptr;
  const int rc = scratch_on(gls::handle_device(h), &ptr);
  if (rc) return rc;
  return gls::solve_block_in(h, nsnp, p_R, X_R, ldxr, B, ldb, info, ptr, GLS_NOALLOC_SCRATCH_BYTES);
}
