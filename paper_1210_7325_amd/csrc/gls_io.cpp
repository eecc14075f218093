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
//
// Results to a file: a ready-made sink callback for gls_solve_stream (the
// output half of Alg. 8: the asynchronous write of block j's b while later
// blocks are computed, and the wait for the previous write before a buffer
// is reused).  The sink copies the block into one of `depth` buffers and
// returns; a writer thread writes the buffers in order with pwrite.  When
// all buffers are waiting to be written, the sink blocks until the oldest
// write completes.
#include <fcntl.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <cerrno>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
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

// pwrite the whole range; returns 0 or the errno of a failed call.
int pwrite_all(int fd, const void* src, int64_t off, int64_t len) {
  const char* p = static_cast<const char*>(src);
  while (len > 0) {
    const int64_t chunk = std::min<int64_t>(len, int64_t(1) << 30);
    const ssize_t r = pwrite(fd, p, (size_t)chunk, (off_t)off);
    if (r < 0 && errno == EINTR) continue;
    if (r <= 0) return errno ? errno : EIO;
    p += r;
    off += r;
    len -= r;
  }
  return 0;
}

struct WriteJob {
  int64_t snp0 = 0, nsnp = 0;
  std::vector<double> b;
  std::vector<int32_t> info;
};

}  // namespace

struct gls_file_writer_s {
  int fd_b = -1, fd_info = -1;
  int64_t t = 0, p = 0, base = 0;
  int depth = 2;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<WriteJob> pending;  // copied blocks waiting to be written, in order
  std::vector<WriteJob> spare;   // buffers free for reuse
  int inflight = 0;              // jobs taken by the writer thread, not yet done
  bool stop = false;
  int err = 0;                   // first write error (errno)
  std::thread th;
  std::atomic<int64_t> bytes{0};
  std::atomic<int64_t> write_ns{0};
  std::atomic<int64_t> wait_ns{0};
  std::atomic<int64_t> close_ns{0};

  void run() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv.wait(lk, [&] { return stop || !pending.empty(); });
      if (pending.empty()) return;  // stop requested and nothing left
      WriteJob j = std::move(pending.front());
      pending.pop_front();
      inflight++;
      lk.unlock();
      const auto t0 = std::chrono::steady_clock::now();
      int e = 0;
      if (!err) {
        const int64_t row = t * p * (int64_t)sizeof(double);
        e = pwrite_all(fd_b, j.b.data(), (j.snp0 - base) * row, j.nsnp * row);
        if (!e && fd_info >= 0)
          e = pwrite_all(fd_info, j.info.data(), (j.snp0 - base) * (int64_t)sizeof(int32_t),
                         j.nsnp * (int64_t)sizeof(int32_t));
      }
      write_ns += std::chrono::duration_cast<std::chrono::nanoseconds>(
                      std::chrono::steady_clock::now() - t0).count();
      if (!e) bytes += j.nsnp * (t * p * (int64_t)sizeof(double) + (fd_info >= 0 ? 4 : 0));
      lk.lock();
      if (e && !err) err = e;
      spare.push_back(std::move(j));
      inflight--;
      cv.notify_all();
    }
  }
};

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

int gls_writer_open(gls_file_writer* out, const char* b_path, const char* info_path, int64_t t,
                    int64_t p, int64_t snp_base, int depth) {
  if (!out) return -1;
  *out = nullptr;
  if (!b_path) return -2;
  if (t < 1) return -4;
  if (p < 1) return -5;
  if (snp_base < 0) return -6;
  if (depth < 1 || depth > 64) return -7;
  gls_file_writer_s* w = new (std::nothrow) gls_file_writer_s;
  if (!w) return GLS_E_OOM;
  w->fd_b = open(b_path, O_WRONLY | O_CREAT | O_CLOEXEC, 0644);
  if (w->fd_b >= 0 && info_path) w->fd_info = open(info_path, O_WRONLY | O_CREAT | O_CLOEXEC, 0644);
  if (w->fd_b < 0 || (info_path && w->fd_info < 0)) {
    if (w->fd_b >= 0) close(w->fd_b);
    delete w;
    return GLS_E_IO;
  }
  w->t = t;
  w->p = p;
  w->base = snp_base;
  w->depth = depth;
  try {
    w->th = std::thread([w] { w->run(); });
  } catch (...) {
    close(w->fd_b);
    if (w->fd_info >= 0) close(w->fd_info);
    delete w;
    return GLS_E_OOM;
  }
  *out = w;
  return GLS_OK;
}

int gls_writer_sink(void* writer, int64_t snp0, int64_t nsnp, const double* b, const int32_t* info) {
  gls_file_writer_s* w = static_cast<gls_file_writer_s*>(writer);
  if (!w || snp0 < w->base || nsnp < 0 || (nsnp > 0 && !b)) return 1;
  if (nsnp == 0) return 0;
  std::unique_lock<std::mutex> lk(w->mu);
  const auto t0 = std::chrono::steady_clock::now();
  // wait(previous): a buffer is free once its write has completed
  w->cv.wait(lk, [&] { return w->err || (int)w->pending.size() + w->inflight < w->depth; });
  w->wait_ns += std::chrono::duration_cast<std::chrono::nanoseconds>(
                    std::chrono::steady_clock::now() - t0).count();
  if (w->err) return 1;
  WriteJob j;
  if (!w->spare.empty()) {
    j = std::move(w->spare.back());
    w->spare.pop_back();
  }
  lk.unlock();
  try {
    j.b.assign(b, b + nsnp * w->t * w->p);
    if (info)
      j.info.assign(info, info + nsnp);
    else
      j.info.assign((size_t)nsnp, 0);
  } catch (...) {
    return 1;
  }
  j.snp0 = snp0;
  j.nsnp = nsnp;
  lk.lock();
  w->pending.push_back(std::move(j));  // async_write(b of this block)
  w->cv.notify_all();
  return 0;
}

int gls_writer_close(gls_file_writer w, int64_t* bytes, double* write_ms, double* wait_ms,
                     double* close_ms) {
  if (!w) return GLS_OK;
  const auto t0 = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(w->mu);
    w->stop = true;
  }
  w->cv.notify_all();
  w->th.join();
  int rc = w->err ? GLS_E_IO : GLS_OK;
  if (fdatasync(w->fd_b) != 0 && rc == GLS_OK) rc = GLS_E_IO;
  if (w->fd_info >= 0 && fdatasync(w->fd_info) != 0 && rc == GLS_OK) rc = GLS_E_IO;
  close(w->fd_b);
  if (w->fd_info >= 0) close(w->fd_info);
  w->close_ns += std::chrono::duration_cast<std::chrono::nanoseconds>(
                     std::chrono::steady_clock::now() - t0).count();
  if (bytes) *bytes = w->bytes.load();
  if (write_ms) *write_ms = (double)w->write_ns.load() * 1e-6;
  if (wait_ms) *wait_ms = (double)w->wait_ns.load() * 1e-6;
  if (close_ms) *close_ms = (double)w->close_ns.load() * 1e-6;
  delete w;
  return rc;
}

}  // extern "C"
