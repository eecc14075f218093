// Measurement build of the triangular solve (not part of the library):
// gls_trsm.hip with the phase timestamps of k_trsm_pair compiled in, linked
// with the library's other units into libgls_phase.so.  The kernels compute
// the same results; thread 0 of each work-group stores two clocks at six
// points of each row-block pair (loop top, after the off-diagonal GEMM,
// after W_k, after the L_{k+1,k} W_k update, after W_{k+1}, after the
// closing barrier).  paper_1210_7325_amd/phase_timing.py reads them.
#define GLS_PHASE_TIMING 1
#include "gls_trsm.hip"

// The last launch's stamps: rt and cyc receive PHASE_WGS x PHASE_PAIRS x
// PHASE_POINTS values each (host memory owned by the caller, row-major by
// work-group, pair, point); dims receives the three sizes.  0 or -1.
extern "C" int gls_phase_times(unsigned long long* rt, unsigned long long* cyc, int* dims) {
  if (!rt || !cyc || !dims) return -1;
  dims[0] = gls::PHASE_WGS;
  dims[1] = gls::PHASE_PAIRS;
  dims[2] = gls::PHASE_POINTS;
  if (hipDeviceSynchronize() != hipSuccess) return -1;
  if (hipMemcpyFromSymbol(rt, HIP_SYMBOL(gls::g_phase_rt), sizeof(gls::g_phase_rt)) != hipSuccess) return -1;
  if (hipMemcpyFromSymbol(cyc, HIP_SYMBOL(gls::g_phase_cyc), sizeof(gls::g_phase_cyc)) != hipSuccess) return -1;
  return 0;
}
