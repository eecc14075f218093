// Host side of the C ABI declared in include/gls.h: argument checks,
// device memory ownership, stream ordering and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "gls.h"
#include "gls_host.h"
#include "gls_internal.h"

using namespace gls;

namespace {

struct Cohort {
  std::atomic<int> refs{1};
  int64_t n = 0, n_pad = 0;
  int K = 0;
  int prec = GLS_FP64;
  int info = 0;
  double* Lstrips = nullptr;   // off-diagonal strips, fragment layout
  double* LinvP = nullptr;     // inverted diagonal blocks, fragment layout
  double* Ldiag = nullptr;     // diagonal blocks of L, column-major NB x NB
  float* Lstrips32 = nullptr;  // FP32 copy of the strips (FP32_REFINE)
  // fixed part
  bool fixed = false;
  int64_t pL = 0, t = 0, icol = -1;
  double* F = nullptr;         // row-major n_pad x (pL+t): [W_L | ytil] = L^{-1}[X_L | Y]
  double* STL = nullptr;       // pL x pL
  double* CT = nullptr;        // pL x t
  double* Z = nullptr;         // FP32_REFINE: row-major n_pad x (pL+t), M^{-1}[X_L | Y]
  double* z1 = nullptr;        // FP32_REFINE: column sums of Z (pL+t)
  int cus = 256;               // compute units of the device the cohort lives on
  int device = 0;              // the device current at gls_factor
};

}  // namespace

struct TimedLaunch {
  hipEvent_t a = nullptr, b = nullptr;
  int kind = 0;
  int slab = 0;                // columns per work-group of the launch
  int64_t cols = 0;            // genotype columns (right-hand sides) the launch processed
};

struct gls_handle_s {
  Cohort* c = nullptr;
  hipStream_t stream = nullptr;
  int C = 0;                   // columns per work-group of the triangular solve; 0 = per launch
  double* W = nullptr;         // workspace: whitened genotype columns, slab layout
  int64_t Wcols = 0;           // capacity in columns (multiple of 64)
  float* W32 = nullptr;        // FP32_REFINE: FP32 copy of W (quad layout)
  double* shift = nullptr;     // FP32_REFINE: per-column centering shift
  double* XZ = nullptr;        // FP32_REFINE: per column (x - s)^T Z, MAXP + MAXT wide
  hipEvent_t ws_used = nullptr;  // recorded on the stream of every launch that used the workspace
  bool timing = false;         // bracket kernel launches with events
  std::vector<TimedLaunch> timed;
  size_t ntimed = 0;
};

namespace {

int hip_code(hipError_t e) {
  if (e == hipSuccess) return GLS_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return GLS_E_OOM;
  return GLS_E_HIP;
}

#define HIPCHK(x)                         \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return hip_code(e_); \
  } while (0)

template <typename T>
int dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  const hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
  // a failed allocation also sets the runtime's last error; clear it so the
  // launch checks of later calls do not report it again
  if (e != hipSuccess) (void)hipGetLastError();
  return hip_code(e);
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

void cohort_free(Cohort* c) {
  if (!c) return;
  dfree(c->Lstrips);
  dfree(c->LinvP);
  dfree(c->Ldiag);
  dfree(c->Lstrips32);
  dfree(c->F);
  dfree(c->STL);
  dfree(c->CT);
  dfree(c->Z);
  dfree(c->z1);
  delete c;
}

int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }

size_t strips_count(int K) { return (size_t)K * (size_t)(K - 1) / 2 * (size_t)NB * NB; }

// Wait until no launch still uses h's workspace: the last launch that used
// it may have gone to another stream than the handle's (gls_solve_multi).
int workspace_idle(gls_handle h) {
  if (h->ws_used) HIPCHK(hipEventSynchronize(h->ws_used));
  HIPCHK(hipStreamSynchronize(h->stream));
  return GLS_OK;
}

// Record that work just enqueued on st uses h's workspace.
int workspace_used(gls_handle h, hipStream_t st) {
  if (!h->ws_used) HIPCHK(hipEventCreateWithFlags(&h->ws_used, hipEventDisableTiming));
  HIPCHK(hipEventRecord(h->ws_used, st));
  return GLS_OK;
}

int ensure_workspace(gls_handle h, int64_t ncols) {
  const int64_t need = round_up(std::max<int64_t>(ncols, 1), MAX_C);
  if (need <= h->Wcols) return GLS_OK;
  if (int rc = workspace_idle(h)) return rc;
  dfree(h->W);
  dfree(h->W32);
  dfree(h->shift);
  dfree(h->XZ);
  h->Wcols = 0;
  int rc = dalloc(&h->W, (size_t)h->c->n_pad * (size_t)need);
  if (rc) return rc;
  if (h->c->prec == GLS_FP32_REFINE) {
    if ((rc = dalloc(&h->W32, (size_t)h->c->n_pad * (size_t)need))) return rc;
    if ((rc = dalloc(&h->shift, (size_t)need))) return rc;
    if ((rc = dalloc(&h->XZ, (size_t)need * (MAXP + MAXT)))) return rc;
  }
  h->Wcols = need;
  return GLS_OK;
}

// The workspace a launch writes: the handle's own, or caller-provided memory
// (the no-allocation entry point).
Workspace own_workspace(gls_handle h) { return Workspace{h->W, h->W32, h->shift, h->XZ}; }

JobDesc make_job(gls_handle h, const Workspace& ws, int64_t slab0, int64_t ncols, const void* X,
                 int64_t ldx) {
  JobDesc j;
  j.slab0 = slab0;
  j.n = h->c->n;
  j.ncols = ncols;
  j.X = X;
  j.ldx = ldx;
  j.Lstrips = h->c->Lstrips;
  j.LinvP = h->c->LinvP;
  j.W = ws.W;
  j.K = h->c->K;
  j.Lstrips32 = h->c->Lstrips32;
  j.W32 = ws.W32;
  j.shift = ws.shift;
  return j;
}

XzDesc make_xz(gls_handle h, const Workspace& ws, int64_t grp0, int64_t ncols, const int8_t* X,
               int64_t ldx) {
  XzDesc x;
  x.grp0 = grp0;
  x.n = h->c->n;
  x.ncols = ncols;
  x.X = X;
  x.ldx = ldx;
  x.Z = h->c->Z;
  x.z1 = h->c->z1;
  x.shift = ws.shift;
  x.XZ = ws.XZ;
  x.ldf = (int)(h->c->pL + h->c->t);
  return x;
}

AsmDesc make_asm(gls_handle h, const Workspace& ws, int C, int64_t grp0, int64_t nsnp, int64_t pR,
                 double* B, int64_t ldb, int32_t* info) {
  AsmDesc a;
  a.grp0 = grp0;
  a.n = h->c->n;
  a.n_pad = h->c->n_pad;
  a.W = ws.W;
  a.F = h->c->F;
  a.STL = h->c->STL;
  a.CT = h->c->CT;
  a.nsnp = nsnp;
  a.B = B;
  a.ldb = ldb;
  a.info = info;
  a.C = C;
  a.pL = (int)h->c->pL;
  a.pR = (int)pR;
  a.t = (int)h->c->t;
  a.shift = ws.shift;
  a.XZ = ws.XZ;
  a.icol = (int)h->c->icol;
  return a;
}

// Argument checks shared by gls_solve_block and gls_solve_multi; `base`
// is the ABI position of the nsnp argument.
int check_block(gls_handle h, int64_t nsnp, int64_t pR, const int8_t* X_R, int64_t ldxr,
                double* B, int64_t ldb, int base) {
  if (!h) return -(base - 1);
  if (nsnp < 0) return -base;
  if (!h->c->fixed) return GLS_E_STATE;
  const int64_t p = h->c->pL + pR;
  if (pR < 1 || pR > 16 || p > MAXP || h->c->n <= p) return -(base + 1);
  if (nsnp > 0 && !X_R) return -(base + 2);
  if (ldxr < h->c->n) return -(base + 3);
  if (nsnp > 0 && !B) return -(base + 4);
  if (ldb < p) return -(base + 5);
  return GLS_OK;
}

// Brackets one kernel launch with a pair of events when timing is on.
struct TimedScope {
  gls_handle h;
  TimedLaunch* p = nullptr;
  TimedScope(gls_handle h_, int kind, int64_t cols, int slab) : h(h_) {
    if (!h || !h->timing) return;
    if (h->ntimed == h->timed.size()) {
      TimedLaunch t;
      if (hipEventCreate(&t.a) != hipSuccess || hipEventCreate(&t.b) != hipSuccess) return;
      h->timed.push_back(t);
    }
    p = &h->timed[h->ntimed++];
    p->kind = kind;
    p->cols = cols;
    p->slab = slab;
    (void)hipEventRecord(p->a, h->stream);
  }
  void end() {
    if (p) (void)hipEventRecord(p->b, h->stream);
    p = nullptr;
  }
  ~TimedScope() { end(); }
};

// Slab width of one launch.  A slab's walk down the row blocks takes a time
// that grows with its width and with K^2 (K row blocks of its cohort), so a
// launch of few columns is fastest with the narrowest slabs that still give
// at most one work-group per compute unit (measured at n = 10^4, FP64: 576
// to 4,096 columns in 9.9 ms with 16-column slabs against 22.9 ms with 64;
// 8,192 columns in 16.4 ms with 32 against 23.3 ms).  Past 64 columns per
// CU, 128-column slabs are about 6% faster per column (32,768 columns: FP64
// 50.0 ms against 52.6 ms with 64, FP32_REFINE 32.2 ms against 34.6 ms), but
// a 128-column slab takes twice as long as a 64-column one: they are chosen
// only when the 64-column slabs of the launch, spread over the CUs, would
// take at least two of its longest slab, so that no slab of a large cohort
// becomes the critical path of a launch that mixes cohorts.  The
// FP32_REFINE kernel has no 16-column form.  A width set on the handle
// overrides the choice.
int slab_cols_for(const gls_work* items, int64_t count) {
  const gls_handle h = items[0].h;
  if (h->C != 0) return h->C;
  int64_t s16 = 0, s32 = 0, s64 = 0, work64 = 0, kmax2 = 0;
  for (int64_t i = 0; i < count; i++) {
    const int64_t ncols = items[i].nsnp * items[i].p_R;
    const int64_t k2 = (int64_t)items[i].h->c->K * items[i].h->c->K;
    s16 += (ncols + 15) / 16;
    s32 += (ncols + 31) / 32;
    s64 += (ncols + 63) / 64;
    work64 += (ncols + 63) / 64 * k2;
    if (ncols > 0) kmax2 = std::max(kmax2, k2);
  }
  const int64_t cus = h->c->cus;
  if (h->c->prec != GLS_FP32_REFINE && s16 <= cus) return 16;
  if (s32 <= cus) return 32;
  if (s64 <= cus || work64 < 2 * cus * kmax2) return 64;
  return 128;
}

// Launch the kernels of up to MAX_INLINE_JOBS checked work items (same slab
// width setting and precision) on stream st; timing events go through
// handle th (none if th is NULL).  ws: the workspace of a single item, or
// NULL for each item's own (grown here when too small).
int launch_items(const gls_work* items, int64_t count, hipStream_t st, gls_handle th,
                 const Workspace* ws = nullptr, int C_set = 0) {
  if (!ws) {
    for (int64_t i = 0; i < count; i++) {
      int rc = ensure_workspace(items[i].h, items[i].nsnp * items[i].p_R);
      if (rc) return rc;
    }
  } else if (count != 1) {
    return GLS_E_UNSUPPORTED;
  }
  const int C = C_set ? C_set : slab_cols_for(items, count);
  const bool refine = items[0].h->c->prec == GLS_FP32_REFINE;
  JobTable tab;
  AsmTable at;
  XzTable xt;
  tab.njobs = at.njobs = xt.njobs = 0;
  int64_t slabs = 0, groups = 0, xgroups = 0, cols = 0;
  for (int64_t i = 0; i < count; i++) {
    const gls_work& w = items[i];
    if (w.nsnp == 0) continue;
    const int64_t ncols = w.nsnp * w.p_R;
    cols += ncols;
    const Workspace wsi = ws ? *ws : own_workspace(w.h);
    if (refine) {
      xt.j[xt.njobs++] = make_xz(w.h, wsi, xgroups, ncols, w.X_R, w.ldxr);
      xgroups += (ncols + AS_GROUP_COLS - 1) / AS_GROUP_COLS;
    }
    tab.j[tab.njobs++] = make_job(w.h, wsi, slabs, ncols, w.X_R, w.ldxr);
    slabs += (ncols + C - 1) / C;
    at.j[at.njobs++] = make_asm(w.h, wsi, C, groups, w.nsnp, w.p_R, w.B, w.ldb, w.info);
    const int64_t per_group = (AS_GROUP_COLS / 16) * (16 / w.p_R);  // problems per assembly work-group
    groups += (w.nsnp + per_group - 1) / per_group;
  }
  if (tab.njobs == 0) return GLS_OK;
  hipStream_t keep = th ? th->stream : nullptr;
  if (th) th->stream = st;  // timing events go to the launch stream
  hipError_t e = hipSuccess;
  if (refine) {
    TimedScope tx(th, 1, cols, C);
    e = launch_xz_shift(xt, xgroups, st);
  }
  if (e == hipSuccess) {
    TimedScope t0(th, 0, cols, C);
    e = refine ? launch_trsm_mixed(tab, slabs, C, st) : launch_trsm_i8(tab, slabs, C, st);
  }
  if (e == hipSuccess) {
    TimedScope t1(th, 1, cols, C);
    e = launch_assemble_solve(at, groups, refine, st);
  }
  if (th) th->stream = keep;
  if (e == hipSuccess && !ws) {
    for (int64_t i = 0; i < count; i++)
      if (items[i].nsnp > 0)
        if (int rc = workspace_used(items[i].h, st)) return rc;
  }
  return hip_code(e);
}

// Launch the work items of one call in rounds of at most one work-group per
// compute unit.  A launch whose slabs outnumber the compute units runs a
// second, partly empty round of whole slab walks (a walk takes as long
// whatever runs beside it); here the columns that fill one round form one
// launch and the rest the next, whose slab width is chosen for its own size
// (a narrower slab walks its row blocks faster): at n = 10^4, 16,960
// columns in 256 64-column slabs and then 36 16-column ones instead of 265
// 64-column slabs.  An item can be split between two launches: they are
// ordered on stream st, so both parts use the item's workspace in turn.
// Items of several cohorts (whose slab walks differ in length, which one
// launch balances by itself) and handles with a fixed width are launched as
// they are, in groups of MAX_INLINE_JOBS.
int launch_rounds(const gls_work* items, int64_t count, hipStream_t st, gls_handle th) {
  bool split = items[0].h->C == 0;
  for (int64_t i = 1; i < count; i++) split = split && items[i].h->c == items[0].h->c;
  if (!split) {
    for (int64_t a = 0; a < count; a += MAX_INLINE_JOBS) {
      int rc = launch_items(items + a, std::min<int64_t>(count - a, MAX_INLINE_JOBS), st, th);
      if (rc) return rc;
    }
    return GLS_OK;
  }
  std::vector<gls_work> rest(items, items + count);
  const int64_t cus = items[0].h->c->cus;
  const int64_t t = items[0].h->c->t;
  size_t at = 0;
  while (at < rest.size()) {
    const int C = slab_cols_for(&rest[at], (int64_t)(rest.size() - at));
    gls_work batch[MAX_INLINE_JOBS];
    int nb = 0;
    int64_t slabs = 0;
    while (at < rest.size() && nb < MAX_INLINE_JOBS) {
      gls_work& w = rest[at];
      const int64_t s = (w.nsnp * w.p_R + C - 1) / C;
      if (slabs + s <= cus) {
        batch[nb++] = w;
        slabs += s;
        at++;
        continue;
      }
      // the item's first problems fill the round; the rest stays for the next
      const int64_t take = (cus - slabs) * C / w.p_R;
      if (take > 0) {
        gls_work a = w;
        a.nsnp = take;
        batch[nb++] = a;
        w.nsnp -= take;
        w.X_R += take * w.p_R * w.ldxr;
        w.B += take * t * w.ldb;
        w.info += take;
      }
      break;
    }
    if (nb == 0) return GLS_E_UNSUPPORTED;  // (a problem wider than a round: not reachable, p_R <= 16)
    int rc = launch_items(batch, nb, st, th, nullptr, C);
    if (rc) return rc;
  }
  return GLS_OK;
}

}  // namespace

namespace gls {

size_t workspace_bytes(gls_handle h, int64_t ncols) {
  const size_t cols = (size_t)round_up(std::max<int64_t>(ncols, 1), MAX_C);
  const size_t n_pad = (size_t)h->c->n_pad;
  size_t b = round_up((int64_t)(n_pad * cols * sizeof(double)), 256);
  if (h->c->prec == GLS_FP32_REFINE) {
    b += round_up((int64_t)(n_pad * cols * sizeof(float)), 256);
    b += round_up((int64_t)(cols * sizeof(double)), 256);
    b += round_up((int64_t)(cols * (MAXP + MAXT) * sizeof(double)), 256);
  }
  return b;
}

int handle_device(gls_handle h) { return h->c->device; }

int solve_block_in(gls_handle h, int64_t nsnp, int64_t p_R, const int8_t* X_R, int64_t ldxr,
                   double* B, int64_t ldb, int32_t* info, void* scratch, size_t scratch_bytes) {
  int rc = check_block(h, nsnp, p_R, X_R, ldxr, B, ldb, 2);
  if (rc) return rc;
  if (nsnp == 0) return GLS_OK;
  const int64_t ncols = nsnp * p_R;
  if (workspace_bytes(h, ncols) > scratch_bytes) return GLS_E_TOO_LARGE;
  // carve the workspace out of the caller's memory, in the order and with the
  // 256-byte alignment workspace_bytes counts
  const size_t cols = (size_t)round_up(std::max<int64_t>(ncols, 1), MAX_C);
  const size_t n_pad = (size_t)h->c->n_pad;
  char* p = static_cast<char*>(scratch);
  Workspace ws{reinterpret_cast<double*>(p), nullptr, nullptr, nullptr};
  p += round_up((int64_t)(n_pad * cols * sizeof(double)), 256);
  if (h->c->prec == GLS_FP32_REFINE) {
    ws.W32 = reinterpret_cast<float*>(p);
    p += round_up((int64_t)(n_pad * cols * sizeof(float)), 256);
    ws.shift = reinterpret_cast<double*>(p);
    p += round_up((int64_t)(cols * sizeof(double)), 256);
    ws.XZ = reinterpret_cast<double*>(p);
  }
  gls_work w{h, nsnp, p_R, X_R, ldxr, B, ldb, info};
  return launch_items(&w, 1, h->stream, nullptr, &ws);
}

}  // namespace gls

extern "C" {

const char* gls_strerror(int code) {
  switch (code) {
    case GLS_OK: return "success";
    case GLS_E_NOT_SPD: return "matrix M is not positive definite";
    case GLS_E_STATE: return "call out of order for this handle";
    case GLS_E_OOM: return "device memory allocation failed";
    case GLS_E_HIP: return "HIP runtime error";
    case GLS_E_UNSUPPORTED: return "unsupported request";
    case GLS_E_IO: return "file could not be opened or read";
    case GLS_E_ABORTED: return "a stream callback asked to stop";
    case GLS_E_TOO_LARGE: return "block too large for the fixed scratch of the no-allocation entry point";
    default: return code < 0 ? "invalid argument" : "unknown error";
  }
}

size_t gls_footprint_bytes(int64_t n, int64_t p_L, int64_t p_R, int64_t t, int64_t max_nsnp,
                           int prec) {
  if (n < 1 || p_L < 0 || p_R < 1 || t < 0 || max_nsnp < 0) return 0;
  const int64_t max_cols = max_nsnp * p_R;
  const int K = (int)((n + NB - 1) / NB);
  const size_t n_pad = (size_t)K * NB;
  size_t b = 0;
  b += strips_count(K) * 8;                        // strips
  b += 2 * (size_t)K * NB * NB * 8;                // inverted + plain diagonal blocks
  b += n_pad * n_pad * 8 + (size_t)K * NB * NB * 8;  // factorization work (transient)
  const size_t w = (size_t)(p_L + t);
  b += n_pad * w * 8 + (w * w) * 8;  // fixed part
  b += n_pad * (size_t)round_up(std::max<int64_t>(max_cols, 1), MAX_C) * 8;  // workspace
  if (prec == GLS_FP32_REFINE) {
    b += strips_count(K) * 4;                                   // FP32 strips
    b += n_pad * w * 8 + (w + MAXP + MAXT) * 8;                 // Z, its padding, its column sums
    const size_t cols = (size_t)round_up(std::max<int64_t>(max_cols, 1), MAX_C);
    b += n_pad * cols * 4 + cols * 8 + cols * (MAXP + MAXT) * 8;  // W32, shift, XZ
  }
  return b;
}

int gls_factor(gls_handle* out, int64_t n, const double* M, int64_t ldm, int prec, void* stream) {
  if (!out) return -1;
  *out = nullptr;
  if (n < 2 || n > (int64_t)1 << 20) return -2;
  if (!M) return -3;
  if (ldm < n) return -4;
  if (prec != GLS_FP64 && prec != GLS_FP32_REFINE) return -5;

  Cohort* c = new (std::nothrow) Cohort();
  if (!c) return GLS_E_OOM;
  c->n = n;
  c->K = (int)((n + NB - 1) / NB);
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess) c->device = dev;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      c->cus = cus;
    (void)hipGetLastError();
  }
  c->n_pad = (int64_t)c->K * NB;
  c->prec = prec;
  gls_handle h = new (std::nothrow) gls_handle_s();
  if (!h) { delete c; return GLS_E_OOM; }
  h->c = c;
  h->stream = reinterpret_cast<hipStream_t>(stream);

  double* A = nullptr;
  double* Linv = nullptr;
  int* dinfo = nullptr;
  const int K = c->K;
  const size_t blk = (size_t)K * NB * NB;
  int rc = GLS_OK;
  auto fail = [&](int code) {
    dfree(A);
    dfree(Linv);
    dfree(dinfo);
    cohort_free(c);
    delete h;
    return code;
  };
  if ((rc = dalloc(&A, (size_t)c->n_pad * c->n_pad))) return fail(rc);
  if ((rc = dalloc(&Linv, blk))) return fail(rc);
  if ((rc = dalloc(&dinfo, 1))) return fail(rc);
  if ((rc = dalloc(&c->Ldiag, blk))) return fail(rc);
  if ((rc = dalloc(&c->LinvP, blk))) return fail(rc);
  if ((rc = dalloc(&c->Lstrips, std::max<size_t>(strips_count(K), 1)))) return fail(rc);
  if (prec == GLS_FP32_REFINE && (rc = dalloc(&c->Lstrips32, std::max<size_t>(strips_count(K), 1))))
    return fail(rc);

  hipError_t e = hipMemsetAsync(dinfo, 0, sizeof(int), h->stream);
  if (e == hipSuccess)
    e = launch_factor(M, ldm, n, c->n_pad, K, A, c->Ldiag, Linv, c->Lstrips, c->LinvP,
                      c->Lstrips32, dinfo, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&c->info, dinfo, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(hip_code(e));
  dfree(A);
  dfree(Linv);
  dfree(dinfo);
  *out = h;
  return c->info != 0 ? GLS_E_NOT_SPD : GLS_OK;
}

int gls_last_info(gls_handle h) { return h ? h->c->info : -1; }

int gls_set_stream(gls_handle h, void* stream) {
  if (!h) return -1;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  return GLS_OK;
}

int gls_whiten_fixed(gls_handle h, int64_t p_L, const double* X_L, int64_t ldx, int64_t t,
                     const double* Y, int64_t ldy, int64_t intercept_col) {
  if (!h) return -1;
  Cohort* c = h->c;
  if (p_L < 1 || p_L > MAXP - 1 || p_L >= c->n) return -2;
  if (!X_L) return -3;
  if (ldx < c->n) return -4;
  if (t < 1 || t > MAXT) return -5;
  if (!Y) return -6;
  if (ldy < c->n) return -7;
  if (intercept_col < -1 || intercept_col >= p_L) return -8;
  if (c->info != 0) return GLS_E_STATE;
  if (c->refs.load() != 1) return GLS_E_STATE;  // shared with forks: read-only
  if (c->prec == GLS_FP32_REFINE && intercept_col < 0) return GLS_E_UNSUPPORTED;

  HIPCHK(hipStreamSynchronize(h->stream));
  dfree(c->F);
  dfree(c->STL);
  dfree(c->CT);
  dfree(c->Z);
  dfree(c->z1);
  c->fixed = false;
  const int64_t w = p_L + t;
  int rc;
  if ((rc = dalloc(&c->F, (size_t)c->n_pad * w))) return rc;
  if ((rc = dalloc(&c->STL, (size_t)p_L * p_L))) return rc;
  if ((rc = dalloc(&c->CT, (size_t)p_L * t))) return rc;
  // Z carries MAXP + MAXT doubles of zeros past its last row: the centering
  // pre-pass reads a fixed number of entries from every row
  if (c->prec == GLS_FP32_REFINE && (rc = dalloc(&c->Z, (size_t)c->n_pad * w + MAXP + MAXT))) return rc;
  if (c->prec == GLS_FP32_REFINE && (rc = dalloc(&c->z1, (size_t)w))) return rc;
  if (c->prec == GLS_FP32_REFINE)
    HIPCHK(hipMemsetAsync(c->Z + (size_t)c->n_pad * w, 0, sizeof(double) * (MAXP + MAXT), h->stream));
  c->pL = p_L;
  c->t = t;
  c->icol = intercept_col;
  HIPCHK(launch_fixed_solve(X_L, ldx, Y, ldy, c->n, c->n_pad, c->K, (int)p_L, (int)t, c->Lstrips,
                            c->LinvP, c->F, c->Z, h->stream));
  HIPCHK(launch_gram(c->F, c->n, (int)p_L, (int)t, c->STL, c->CT, h->stream));
  if (c->prec == GLS_FP32_REFINE) HIPCHK(launch_colsum(c->Z, c->n, (int)w, c->z1, h->stream));
  c->fixed = true;
  return GLS_OK;
}

int gls_reserve(gls_handle h, int64_t max_cols) {
  if (!h) return -1;
  if (max_cols < 0) return -2;
  return ensure_workspace(h, max_cols);
}

int gls_solve_block(gls_handle h, int64_t nsnp, int64_t p_R, const int8_t* X_R, int64_t ldxr,
                    double* B, int64_t ldb, int32_t* info) {
  int rc = check_block(h, nsnp, p_R, X_R, ldxr, B, ldb, 2);
  if (rc) return rc;
  if (nsnp == 0) return GLS_OK;
  gls_work w{h, nsnp, p_R, X_R, ldxr, B, ldb, info};
  return launch_rounds(&w, 1, h->stream, h);
}

int gls_solve_multi(const gls_work* items, int64_t count, void* stream) {
  if (count < 0) return -2;
  if (count == 0) return GLS_OK;
  if (!items) return -1;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int C = items[0].h ? items[0].h->C : 0;
  const int prec = items[0].h ? items[0].h->c->prec : GLS_FP64;
  for (int64_t i = 0; i < count; i++) {
    const gls_work& w = items[i];
    int rc = check_block(w.h, w.nsnp, w.p_R, w.X_R, w.ldxr, w.B, w.ldb, 2);
    if (rc) return rc < 0 ? -1 : rc;
    // one slab width and one precision per launch
    if (w.h->C != C || w.h->c->prec != prec) return GLS_E_UNSUPPORTED;
    for (int64_t j = 0; j < i; j++)
      if (items[j].h == w.h) return -1;  // each item needs its own workspace
  }
  return launch_rounds(items, count, st, items[0].h);
}

int gls_fork(gls_handle h, void* stream, gls_handle* out) {
  if (!out) return -3;
  *out = nullptr;
  if (!h) return -1;
  if (!h->c->fixed) return GLS_E_STATE;
  HIPCHK(hipStreamSynchronize(h->stream));
  gls_handle g = new (std::nothrow) gls_handle_s();
  if (!g) return GLS_E_OOM;
  g->c = h->c;
  g->c->refs.fetch_add(1);
  g->stream = reinterpret_cast<hipStream_t>(stream);
  g->C = h->C;
  *out = g;
  return GLS_OK;
}

void gls_free(gls_handle h) {
  if (!h) return;
  (void)workspace_idle(h);
  if (h->ws_used) (void)hipEventDestroy(h->ws_used);
  dfree(h->W);
  dfree(h->W32);
  dfree(h->shift);
  dfree(h->XZ);
  for (auto& p : h->timed) {
    if (p.a) (void)hipEventDestroy(p.a);
    if (p.b) (void)hipEventDestroy(p.b);
  }
  if (h->c->refs.fetch_sub(1) == 1) cohort_free(h->c);
  delete h;
}

int gls_copy_factor(gls_handle h, double* L, int64_t ldl) {
  if (!h) return -1;
  if (!L) return -2;
  if (ldl < h->c->n) return -3;
  if (h->c->info != 0) return GLS_E_STATE;
  HIPCHK(launch_unpack_factor(h->c->Lstrips, h->c->Ldiag, h->c->n, L, ldl, h->stream));
  return GLS_OK;
}

int gls_copy_fixed(gls_handle h, double* WL, int64_t ldwl, double* Yt, int64_t ldyt, double* S_TL,
                   double* C_T) {
  if (!h) return -1;
  Cohort* c = h->c;
  if (WL && ldwl < c->n) return -3;
  if (Yt && ldyt < c->n) return -5;
  if (!c->fixed) return GLS_E_STATE;
  const int w = (int)(c->pL + c->t);
  if (WL) HIPCHK(launch_rowmajor_to_colmajor(c->F, w, c->n, 0, (int)c->pL, WL, ldwl, h->stream));
  if (Yt) HIPCHK(launch_rowmajor_to_colmajor(c->F, w, c->n, (int)c->pL, (int)c->t, Yt, ldyt, h->stream));
  if (S_TL)
    HIPCHK(hipMemcpyAsync(S_TL, c->STL, sizeof(double) * c->pL * c->pL, hipMemcpyDeviceToDevice,
                          h->stream));
  if (C_T)
    HIPCHK(hipMemcpyAsync(C_T, c->CT, sizeof(double) * c->pL * c->t, hipMemcpyDeviceToDevice,
                          h->stream));
  return GLS_OK;
}

int gls_whiten_block(gls_handle h, int64_t ncols, const int8_t* X, int64_t ldx, double* W,
                     int64_t ldw) {
  if (!h) return -1;
  if (ncols < 0) return -2;
  if (ncols > 0 && !X) return -3;
  if (ldx < h->c->n) return -4;
  if (ncols > 0 && !W) return -5;
  if (ldw < h->c->n) return -6;
  if (h->c->info != 0) return GLS_E_STATE;
  if (ncols == 0) return GLS_OK;
  int rc = ensure_workspace(h, ncols);
  if (rc) return rc;
  JobTable tab;
  tab.njobs = 1;
  tab.j[0] = make_job(h, own_workspace(h), 0, ncols, X, ldx);
  const gls_work item{h, ncols, 1, X, ldx, nullptr, 0, nullptr};
  const int C = slab_cols_for(&item, 1);
  TimedScope t0(h, 0, ncols, C);
  if (h->c->prec == GLS_FP32_REFINE) {
    // plain L^{-1} X: no centering shift
    HIPCHK(hipMemsetAsync(h->shift, 0, sizeof(double) * ncols, h->stream));
    HIPCHK(launch_trsm_mixed(tab, (ncols + C - 1) / C, C, h->stream));
  } else {
    HIPCHK(launch_trsm_i8(tab, (ncols + C - 1) / C, C, h->stream));
  }
  t0.end();
  HIPCHK(launch_slab_to_colmajor(h->W, C, h->c->n_pad, h->c->n, 0, ncols, W, ldw, h->stream));
  return workspace_used(h, h->stream);
}

int gls_whiten_block_f64(gls_handle h, int64_t ncols, const double* X, int64_t ldx, double* W,
                         int64_t ldw) {
  if (!h) return -1;
  if (ncols < 0) return -2;
  if (ncols > 0 && !X) return -3;
  if (ldx < h->c->n) return -4;
  if (ncols > 0 && !W) return -5;
  if (ldw < h->c->n) return -6;
  if (h->c->info != 0) return GLS_E_STATE;
  if (h->c->prec != GLS_FP64) return GLS_E_UNSUPPORTED;
  if (ncols == 0) return GLS_OK;
  int rc = ensure_workspace(h, ncols);
  if (rc) return rc;
  JobTable tab;
  tab.njobs = 1;
  tab.j[0] = make_job(h, own_workspace(h), 0, ncols, X, ldx);
  const gls_work item{h, ncols, 1, nullptr, ldx, nullptr, 0, nullptr};
  int C = slab_cols_for(&item, 1);
  if (C == 32) C = 64;  // FP64 right-hand sides come in 16-, 64- and 128-column slabs
  TimedScope t0(h, 0, ncols, C);
  HIPCHK(launch_trsm_f64(tab, (ncols + C - 1) / C, C, h->stream));
  t0.end();
  HIPCHK(launch_slab_to_colmajor(h->W, C, h->c->n_pad, h->c->n, 0, ncols, W, ldw, h->stream));
  return workspace_used(h, h->stream);
}

int gls_set_slab_cols(gls_handle h, int cols) {
  if (!h) return -1;
  if (cols != 0 && cols != 16 && cols != 32 && cols != 64 && cols != 128) return -2;
  if (h->c->prec == GLS_FP32_REFINE && cols == 16) return GLS_E_UNSUPPORTED;
  h->C = cols;
  return GLS_OK;
}

int gls_set_kernel_timing(gls_handle h, int enable) {
  if (!h) return -1;
  HIPCHK(hipStreamSynchronize(h->stream));
  h->ntimed = 0;
  h->timing = enable != 0;
  return GLS_OK;
}

int gls_kernel_time(gls_handle h, int kind, double* ms, int64_t* launches) {
  if (!h) return -1;
  if (kind != 0 && kind != 1) return -2;
  if (!ms) return -3;
  if (!launches) return -4;
  double sum = 0.0;
  int64_t cnt = 0;
  for (size_t i = 0; i < h->ntimed; i++) {
    const TimedLaunch& p = h->timed[i];
    if (p.kind != kind) continue;
    HIPCHK(hipEventSynchronize(p.b));
    float f = 0.f;
    HIPCHK(hipEventElapsedTime(&f, p.a, p.b));
    sum += f;
    cnt++;
  }
  *ms = sum;
  *launches = cnt;
  return GLS_OK;
}

int gls_kernel_launches(gls_handle h, int kind, int64_t cap, double* ms, int64_t* cols, int* slab,
                        int64_t* count) {
  if (!h) return -1;
  if (kind != 0 && kind != 1) return -2;
  if (cap < 0) return -3;
  if (cap > 0 && (!ms || !cols || !slab)) return -4;
  if (!count) return -7;
  int64_t cnt = 0;
  for (size_t i = 0; i < h->ntimed; i++) {
    const TimedLaunch& p = h->timed[i];
    if (p.kind != kind) continue;
    if (cnt < cap) {
      HIPCHK(hipEventSynchronize(p.b));
      float f = 0.f;
      HIPCHK(hipEventElapsedTime(&f, p.a, p.b));
      ms[cnt] = f;
      cols[cnt] = p.cols;
      slab[cnt] = p.slab;
    }
    cnt++;
  }
  *count = cnt;
  return GLS_OK;
}

int gls_solve_stream(gls_handle h, int64_t snp_begin, int64_t snp_end, int64_t block, int64_t p_R,
                     gls_fill_fn fill, void* fill_ctx, gls_sink_fn sink, void* sink_ctx,
                     gls_stream_stats* stats) {
  using clk = std::chrono::steady_clock;
  auto ms_since = [](clk::time_point t0) {
    return std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  };
  const auto t_start = clk::now();
  if (!h) return -1;
  if (snp_begin < 0) return -2;
  if (snp_end < snp_begin) return -3;
  if (block < 1) return -4;
  if (!fill) return -6;
  if (!sink) return -8;
  if (!h->c->fixed) return GLS_E_STATE;
  const int64_t n = h->c->n, t = h->c->t, p = h->c->pL + p_R;
  if (p_R < 1 || p_R > 16 || p > MAXP || n <= p) return -5;
  gls_stream_stats st{};
  if (snp_end == snp_begin) {
    if (stats) *stats = st;
    return GLS_OK;
  }
  // I/O happens per block of `block` problems; the device solves
  // superblocks of `group` consecutive blocks so that one launch has at
  // least one slab per CU (results do not depend on the grouping)
  const int64_t target_cols = h->c->cus * (int64_t)(h->C ? h->C : MAX_C);
  const int64_t group = std::max<int64_t>(1, (target_cols + block * p_R - 1) / (block * p_R));
  const int64_t sbk = group * block;  // problems per superblock
  const int64_t cols = sbk * p_R;
  int rc = ensure_workspace(h, cols);
  if (rc) return rc;

  // Results go from the assembly kernel straight into pinned host memory
  // (mapped into the device's address space): a device-to-host copy would
  // be a copy kernel, and with the solve kernel holding every compute unit
  // it could not start before the next superblock's solve had finished,
  // which kept the host from handing over results and filling the next
  // input while the device worked.
  int8_t* hin[2] = {nullptr, nullptr};
  int8_t* din[2] = {nullptr, nullptr};
  double* hB[2] = {nullptr, nullptr};
  int32_t* hinfo[2] = {nullptr, nullptr};
  hipStream_t s_in = nullptr;
  hipEvent_t ev_in[2] = {nullptr, nullptr}, ev_comp[2] = {nullptr, nullptr};
  const size_t in_bytes = (size_t)n * cols, out_n = (size_t)sbk * t * p;
  auto cleanup = [&]() {
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (s_in) (void)hipStreamSynchronize(s_in);
    for (int i = 0; i < 2; i++) {
      if (hin[i]) (void)hipHostFree(hin[i]);
      if (hB[i]) (void)hipHostFree(hB[i]);
      if (hinfo[i]) (void)hipHostFree(hinfo[i]);
      dfree(din[i]);
      if (ev_in[i]) (void)hipEventDestroy(ev_in[i]);
      if (ev_comp[i]) (void)hipEventDestroy(ev_comp[i]);
    }
    if (s_in) (void)hipStreamDestroy(s_in);
  };
#define STREAM_CHK(x)               \
  do {                              \
    hipError_t e_ = (x);            \
    if (e_ != hipSuccess) {         \
      cleanup();                    \
      return hip_code(e_);          \
    }                               \
  } while (0)
  for (int i = 0; i < 2; i++) {
    STREAM_CHK(hipHostMalloc(reinterpret_cast<void**>(&hin[i]), in_bytes, hipHostMallocDefault));
    STREAM_CHK(hipHostMalloc(reinterpret_cast<void**>(&hB[i]), out_n * sizeof(double), hipHostMallocDefault));
    STREAM_CHK(hipHostMalloc(reinterpret_cast<void**>(&hinfo[i]), sbk * sizeof(int32_t), hipHostMallocDefault));
    STREAM_CHK(hipMalloc(reinterpret_cast<void**>(&din[i]), in_bytes));
    STREAM_CHK(hipEventCreateWithFlags(&ev_in[i], hipEventDisableTiming));
    STREAM_CHK(hipEventCreateWithFlags(&ev_comp[i], hipEventDisableTiming));
  }
  STREAM_CHK(hipStreamCreateWithFlags(&s_in, hipStreamNonBlocking));

  const int64_t nsb = (snp_end - snp_begin + sbk - 1) / sbk;
  auto sb_snp0 = [&](int64_t j) { return snp_begin + j * sbk; };
  auto sb_len = [&](int64_t j) { return std::min<int64_t>(sbk, snp_end - sb_snp0(j)); };
  auto drain = [&](int64_t j) -> int {
    const int sj = (int)(j % 2);
    const auto tw = clk::now();
    hipError_t e = hipEventSynchronize(ev_comp[sj]);
    st.wait_ms += ms_since(tw);
    if (e != hipSuccess) return hip_code(e);
    const int64_t len = sb_len(j);
    for (int64_t o = 0; o < len; o += block) {
      const int64_t nb = std::min<int64_t>(block, len - o);
      const auto ts = clk::now();
      const int r = sink(sink_ctx, sb_snp0(j) + o, nb, hB[sj] + (size_t)o * t * p, hinfo[sj] + o);
      st.sink_ms += ms_since(ts);
      if (r) return GLS_E_ABORTED;
      st.blocks++;
    }
    st.bytes_d2h += (int64_t)(len * (t * p * sizeof(double) + sizeof(int32_t)));
    return GLS_OK;
  };
  for (int64_t j = 0; j < nsb; j++) {
    const int sj = (int)(j % 2);
    const int64_t len = sb_len(j);
    // pinned input sj is free once the copy of superblock j-2 has completed
    if (j >= 2) {
      const auto tw = clk::now();
      STREAM_CHK(hipEventSynchronize(ev_in[sj]));
      st.wait_ms += ms_since(tw);
    }
    for (int64_t o = 0; o < len; o += block) {
      const int64_t nb = std::min<int64_t>(block, len - o);
      const auto tf = clk::now();
      const int fr = fill(fill_ctx, sb_snp0(j) + o, nb, hin[sj] + (size_t)o * p_R * n, n);
      st.fill_ms += ms_since(tf);
      if (fr) {
        cleanup();
        return GLS_E_ABORTED;
      }
    }
    // device input sj is free once the solve of superblock j-2 has finished
    if (j >= 2) STREAM_CHK(hipStreamWaitEvent(s_in, ev_comp[sj], 0));
    STREAM_CHK(hipMemcpyAsync(din[sj], hin[sj], (size_t)n * len * p_R, hipMemcpyHostToDevice, s_in));
    STREAM_CHK(hipEventRecord(ev_in[sj], s_in));
    st.bytes_h2d += n * len * p_R;
    // solve on the handle's stream after the copy; the pinned output sj was
    // handed over (drained) after superblock j-2, before this one was issued
    STREAM_CHK(hipStreamWaitEvent(h->stream, ev_in[sj], 0));
    gls_work w{h, len, p_R, din[sj], n, hB[sj], p, hinfo[sj]};
    rc = launch_rounds(&w, 1, h->stream, h);
    if (rc) {
      cleanup();
      return rc;
    }
    STREAM_CHK(hipEventRecord(ev_comp[sj], h->stream));
    // hand over the previous superblock while this one computes
    if (j >= 1 && (rc = drain(j - 1))) {
      cleanup();
      return rc;
    }
  }
  if ((rc = drain(nsb - 1))) {
    cleanup();
    return rc;
  }
#undef STREAM_CHK
  cleanup();
  st.wall_ms = ms_since(t_start);
  if (stats) *stats = st;
  return GLS_OK;
}

}  // extern "C"
