// Genotypes from a file: a ready-made fill callback for gls_solve_stream
// (the disk-backed out-of-core form, Sec. 4, Alg. 8, where the next block is
// read from disk while the current one is solved).
//
// File layout: X_R column-major int8 with leading dimension n, problem s and
// genotype column q at byte  offset + (s * p_R + q) * n.  A block of
// consecutive problems is therefore one contiguous byte range, read with
// pread by `threads` reader threads in parallel.  With `direct`, the file is
// also opened with O_DIRECT (no page cache: the disk's own speed); pieces
// whose file offset or length are not multiples of 4096 bytes go through the
// buffered descriptor instead.  Pinned host buffers of the HIP runtime may
// refuse direct I/O into them (the kernel cannot map their pages for the
// transfer); the first such refusal switches the source to reading through
// an aligned bounce buffer per thread (still O_DIRECT) and copying.
#include <fcntl.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <chrono>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "gls.h"

namespace {

constexpr int64_t kAlign = 4096;
constexpr int64_t kBounce = int64_t(4) << 20;  // bounce buffer per reader thread

}  // namespace

struct gls_file_source_s {
  int fd = -1;         // buffered descriptor
  int fd_direct = -1;  // O_DIRECT descriptor, -1 if not requested or not available
  int64_t n = 0, p_R = 0, offset = 0;
  int threads = 1;
  std::atomic<bool> bounce{false};  // direct reads go through an aligned bounce buffer
  std::atomic<int64_t> bytes{0};
  std::atomic<int64_t> ns{0};
};

namespace {

// pread the whole range [off, off + len) into dst through descriptor fd;
// returns 0, or the errno of a failed call (EIO for end of file).
int pread_all(int fd, int8_t* dst, int64_t off, int64_t len) {
  while (len > 0) {
    const int64_t chunk = std::min<int64_t>(len, int64_t(1) << 30);
    const ssize_t r = pread(fd, dst, (size_t)chunk, (off_t)off);
    if (r < 0 && errno == EINTR) continue;
    if (r < 0) return errno ? errno : EIO;
    if (r == 0) return EIO;  // end of file before the range was read
    dst += r;
    off += r;
    len -= r;
  }
  return 0;
}

// Direct read of an aligned range through an aligned bounce buffer.
int pread_bounce(int fd, int8_t* dst, int64_t off, int64_t len) {
  void* tmp = nullptr;
  if (posix_memalign(&tmp, kAlign, (size_t)kBounce) != 0) return ENOMEM;
  int8_t* b = static_cast<int8_t*>(tmp);
  int err = 0;
  for (int64_t done = 0; done < len && !err; done += kBounce) {
    const int64_t c = std::min<int64_t>(kBounce, len - done);
    err = pread_all(fd, b, off + done, c);
    if (!err) std::memcpy(dst + done, b, (size_t)c);
  }
  free(tmp);
  return err;
}

// Read len bytes at file offset off into dst; 0 on success.
int read_range(gls_file_source_s* s, int8_t* dst, int64_t off, int64_t len) {
  const bool direct = s->fd_direct >= 0 && off % kAlign == 0 && len % kAlign == 0;
  if (!direct) return pread_all(s->fd, dst, off, len) ? 1 : 0;
  if (!s->bounce.load() && reinterpret_cast<uintptr_t>(dst) % kAlign == 0) {
    const int err = pread_all(s->fd_direct, dst, off, len);
    if (!err) return 0;
    if (err != EFAULT && err != EINVAL) return 1;
    s->bounce = true;  // this memory refuses direct I/O: bounce from now on
  }
  const int err = pread_bounce(s->fd_direct, dst, off, len);
  if (err == EINVAL) return pread_all(s->fd, dst, off, len) ? 1 : 0;  // no direct I/O on this file
  return err ? 1 : 0;
}

}  // namespace

extern "C" {

int gls_file_open(gls_file_source* out, const char* path, int64_t n, int64_t p_R, int64_t offset,
                  int direct, int threads) {
  if (!out) return -1;
  *out = nullptr;
  if (!path) return -2;
  if (n < 1) return -3;
  if (p_R < 1 || p_R > 16) return -4;
  if (offset < 0) return -5;
  if (threads < 1 || threads > 64) return -7;
  gls_file_source_s* s = new (std::nothrow) gls_file_source_s;
  if (!s) return GLS_E_OOM;
  s->fd = open(path, O_RDONLY | O_CLOEXEC);
  if (s->fd < 0) {
    delete s;
    return GLS_E_IO;
  }
  if (direct) s->fd_direct = open(path, O_RDONLY | O_CLOEXEC | O_DIRECT);  // may fail: buffered only
  s->n = n;
  s->p_R = p_R;
  s->offset = offset;
  s->threads = threads;
  *out = s;
  return GLS_OK;
}

int gls_file_fill(void* source, int64_t snp0, int64_t nsnp, int8_t* buf, int64_t ld) {
  gls_file_source_s* s = static_cast<gls_file_source_s*>(source);
  if (!s || !buf || snp0 < 0 || nsnp < 0 || ld != s->n) return 1;
  if (nsnp == 0) return 0;
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t len = nsnp * s->p_R * s->n;
  const int64_t off = s->offset + snp0 * s->p_R * s->n;
  // split into pieces on 4096-byte boundaries of the file (so that aligned
  // blocks stay aligned piece by piece)
  const int nt = (int)std::min<int64_t>(s->threads, (len + (1 << 20) - 1) >> 20);
  std::vector<int64_t> cut(nt + 1);
  cut[0] = 0;
  cut[nt] = len;
  for (int i = 1; i < nt; i++) {
    int64_t c = len / nt * i;
    c -= (off + c) % kAlign;  // piece boundaries at aligned file offsets
    cut[i] = std::max(cut[i - 1], c);
  }
  std::atomic<int> bad{0};
  auto work = [&](int i) {
    if (cut[i + 1] > cut[i] && read_range(s, buf + cut[i], off + cut[i], cut[i + 1] - cut[i])) bad = 1;
  };
  if (nt <= 1) {
    work(0);
  } else {
    std::vector<std::thread> pool;
    pool.reserve(nt - 1);
    for (int i = 1; i < nt; i++) pool.emplace_back(work, i);
    work(0);
    for (auto& th : pool) th.join();
  }
  s->bytes += len;
  s->ns += std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
  return bad.load() ? 1 : 0;
}

int gls_file_stats(gls_file_source src, int64_t* bytes, double* ms) {
  if (!src) return -1;
  if (bytes) *bytes = src->bytes.load();
  if (ms) *ms = (double)src->ns.load() * 1e-6;
  return GLS_OK;
}

void gls_file_close(gls_file_source src) {
  if (!src) return;
  if (src->fd_direct >= 0) close(src->fd_direct);
  if (src->fd >= 0) close(src->fd);
  delete src;
}

}  // extern "C"
