// gls_stream: the GPU half of the paper's multi-level buffering (Sec. 3.1).
//
// Two device buffers alternate roles: while block b is solved in buffer
// alpha on the compute stream, block b+1 is copied from page-locked host
// memory into buffer beta on the copy stream.  Roles rotate by index, never
// by copying.  Unlike the paper's design, the whitened block never returns to
// the host: the per-SNP products and solves run on the GPU right after the
// triangular product, and only b, sigma2, v and status go back.
#include <hip/hip_runtime.h>

#include <fcntl.h>
#include <unistd.h>

#include <algorithm>
#include <cerrno>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <mutex>
#include <thread>
#include <vector>

#include "gls_internal.hpp"

using namespace gls;

namespace {

struct EventPool {
  std::vector<hipEvent_t> ev;
  ~EventPool() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  hipError_t make(size_t count) {
    ev.assign(count, nullptr);
    for (auto& e : ev) {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
    }
    return hipSuccess;
  }
};

// Element of a packed-dosage column: one byte holding four samples' 2-bit
// codes.  A distinct type so that the stream templates pick the right
// staging buffer and block solver.
struct Packed2 {
  uint8_t bits;
};

// Elements per column of the SNP matrix in each input format.
int64_t col_elems(const Ctx* c, const double*) { return c->n; }
int64_t col_elems(const Ctx* c, const uint8_t*) { return c->n; }
int64_t col_elems(const Ctx* c, const Packed2*) { return (c->n + 3) / 4; }

// rows: elements per column (dense in dst)
template <typename T>
hipError_t h2d_block(T* dst, int64_t rows, const T* src, int64_t ld, int64_t cols, hipStream_t s) {
  if (ld == rows) return hipMemcpyAsync(dst, src, sizeof(T) * rows * cols, hipMemcpyHostToDevice, s);
  return hipMemcpy2DAsync(dst, sizeof(T) * rows, src, sizeof(T) * ld, sizeof(T) * rows, cols, hipMemcpyHostToDevice,
                          s);
}

double* stage(Ctx* c, int i, const double*) { return c->buf[i]; }
uint8_t* stage(Ctx* c, int i, const uint8_t*) { return c->ub[i]; }
Packed2* stage(Ctx* c, int i, const Packed2*) { return reinterpret_cast<Packed2*>(c->ub[i]); }

gls_status solve_block(Ctx* c, int mb, const double* X, int64_t ld, double* b, int64_t ldb, double* s2, double* v,
                       int* st, hipStream_t s) {
  return block_forward(c, mb, X, ld, b, ldb, s2, v, st, s);
}
gls_status solve_block(Ctx* c, int mb, const uint8_t* X, int64_t ld, double* b, int64_t ldb, double* s2, double* v,
                       int* st, hipStream_t s) {
  return block_forward_u8(c, mb, X, ld, b, ldb, s2, v, st, s);
}
gls_status solve_block(Ctx* c, int mb, const Packed2* X, int64_t ld, double* b, int64_t ldb, double* s2, double* v,
                       int* st, hipStream_t s) {
  return block_forward_u2(c, mb, reinterpret_cast<const uint8_t*>(X), ld, b, ldb, s2, v, st, s);
}

// Block schedule of a stream of `total` columns: starts of the blocks plus
// `total` at the end.  Full blocks of bc, except that a stream of large blocks
// (bc >= 2,048) starts with short ones, bc / 8 growing by a quarter per block
// (multiples of 64): the first copy (and read), which nothing overlaps, is an
// eighth as long, and each later one still fits under the solve before it
// (a solve takes longer per SNP than its copy).  Results do not depend on the
// blocking.
std::vector<int64_t> block_schedule(int64_t bc, int64_t total) {
  std::vector<int64_t> bstart;
  int64_t pos = 0, len = (bc >= 2048) ? std::max<int64_t>(64, bc / 8 / 64 * 64) : bc;
  while (pos < total) {
    bstart.push_back(pos);
    pos += std::min(len, total - pos);
    len = std::min(bc, (len * 5 / 4 + 63) / 64 * 64);
  }
  bstart.push_back(total);
  return bstart;
}

// The streams a study runs on: the caller's pair, or, without a copy stream,
// the handle's own pair (checked at setup not to share a hardware queue),
// after the work already queued on the caller's compute stream.
struct RunStreams {
  hipStream_t sc = nullptr, sx = nullptr;
};

hipError_t run_streams(Ctx* c, void* compute_stream, void* copy_stream, RunStreams* r) {
  const hipStream_t caller = static_cast<hipStream_t>(compute_stream);
  if (copy_stream || (c->opts.flags & GLS_STREAM_SERIAL)) {   // serial: every copy on the compute stream
    r->sc = caller;
    r->sx = copy_stream ? static_cast<hipStream_t>(copy_stream) : caller;
    return hipSuccess;
  }
  r->sc = c->own_st[0];
  r->sx = c->own_st[1];
  hipError_t e = hipEventRecord(c->ev_join, caller);
  if (e == hipSuccess) e = hipStreamWaitEvent(r->sc, c->ev_join, 0);
  if (e == hipSuccess) e = hipStreamWaitEvent(r->sx, c->ev_join, 0);
  return e;
}

}  // namespace

template <typename T>
static gls_status stream_run(gls_handle h, int64_t m, int64_t col0, const T* XR_host, int64_t ld_xr, double* b_host,
                             double* sigma2_host, double* v_host, int32_t* status_host, const RunStreams& rs,
                             gls_stream_stats* stats_out) {
  Ctx* c = h;
  if (m < 0 || col0 < 0 || col0 > m) return arg_fail("gls_stream: need 0 <= col0 <= m");
  if (col0 == m) {   // nothing to stream: no pointer is used
    if (stats_out) *stats_out = gls_stream_stats{};
    return GLS_OK;
  }
  const int64_t rows = col_elems(c, XR_host);
  if (!XR_host || ld_xr < rows) return arg_fail("gls_stream: the SNP matrix is NULL or its ld is below a column");
  if (!b_host || !sigma2_host || !v_host || !status_host) return arg_fail("gls_stream: NULL host output");
  hipStream_t sc = rs.sc;
  // serial mode: every copy on the compute stream, so nothing overlaps
  hipStream_t sx = (c->opts.flags & GLS_STREAM_SERIAL) ? sc : rs.sx;
  const int64_t bc = c->bc;
  const int p = c->p;
  const std::vector<int64_t> bstart = block_schedule(bc, m - col0);
  const int64_t nblk = (int64_t)bstart.size() - 1;
  gls_stream_stats st{};
  if (nblk == 0) {
    if (stats_out) *stats_out = st;
    return GLS_OK;
  }
  EventPool pool;
  hipError_t e;
  // per block: compute start/stop; plus wall start/stop
  if ((e = pool.make(2 * nblk + 2)) != hipSuccess) return hip_fail(e, "gls_stream: event create");
  hipEvent_t wall0 = pool.ev[2 * nblk], wall1 = pool.ev[2 * nblk + 1];

  auto cols_of = [&](int64_t blk) { return bstart[blk + 1] - bstart[blk]; };
  auto src_of = [&](int64_t blk) { return XR_host + (col0 + bstart[blk]) * ld_xr; };

  if ((e = hipEventRecord(wall0, sx)) != hipSuccess) return hip_fail(e, "gls_stream: record");
  if ((e = h2d_block(stage(c, 0, XR_host), rows, src_of(0), ld_xr, cols_of(0), sx)) != hipSuccess)
    return hip_fail(e, "gls_stream: H2D");
  if ((e = hipEventRecord(c->ev_copy[0], sx)) != hipSuccess) return hip_fail(e, "gls_stream: record");
  st.h2d_bytes += sizeof(T) * rows * cols_of(0);

  for (int64_t blk = 0; blk < nblk; ++blk) {
    const int cur = (int)(blk & 1), nxt = cur ^ 1;
    const int64_t cols = cols_of(blk);
    const int64_t col = col0 + bstart[blk];
    if (blk + 1 < nblk && sx != sc) {
      // beta may only be overwritten once the solve that last read it is done
      if (blk >= 1 && (e = hipStreamWaitEvent(sx, c->ev_comp[nxt], 0)) != hipSuccess)
        return hip_fail(e, "gls_stream: wait");
      if ((e = h2d_block(stage(c, nxt, XR_host), rows, src_of(blk + 1), ld_xr, cols_of(blk + 1), sx)) != hipSuccess)
        return hip_fail(e, "gls_stream: H2D");
      if ((e = hipEventRecord(c->ev_copy[nxt], sx)) != hipSuccess) return hip_fail(e, "gls_stream: record");
      st.h2d_bytes += sizeof(T) * rows * cols_of(blk + 1);
    }
    if (sx == sc && blk >= 1) {   // serial: this block's copy only now, behind the previous results
      if ((e = h2d_block(stage(c, cur, XR_host), rows, src_of(blk), ld_xr, cols, sc)) != hipSuccess)
        return hip_fail(e, "gls_stream: H2D");
      if ((e = hipEventRecord(c->ev_copy[cur], sc)) != hipSuccess) return hip_fail(e, "gls_stream: record");
      st.h2d_bytes += sizeof(T) * rows * cols;
    }
    if ((e = hipStreamWaitEvent(sc, c->ev_copy[cur], 0)) != hipSuccess) return hip_fail(e, "gls_stream: wait");
    if ((e = hipEventRecord(pool.ev[2 * blk], sc)) != hipSuccess) return hip_fail(e, "gls_stream: record");
    gls_status r = solve_block(c, (int)cols, stage(c, cur, XR_host), rows, c->ob, p, c->os2, c->ov, c->ost, sc);
    if (r != GLS_OK) return r;
    if ((e = hipEventRecord(c->ev_comp[cur], sc)) != hipSuccess) return hip_fail(e, "gls_stream: record");
    if ((e = hipEventRecord(pool.ev[2 * blk + 1], sc)) != hipSuccess) return hip_fail(e, "gls_stream: record");
    // results of this block; same stream, so the next block's kernels wait for them
    struct {
      void* dst;
      const void* src;
      size_t bytes;
    } d2h[4] = {{b_host + col * p, c->ob, sizeof(double) * p * cols},
                {sigma2_host + col, c->os2, sizeof(double) * cols},
                {v_host + col, c->ov, sizeof(double) * cols},
                {status_host + col, c->ost, sizeof(int32_t) * cols}};
    for (int q = 0; q < 4; ++q) {
      if ((e = hipMemcpyAsync(d2h[q].dst, d2h[q].src, d2h[q].bytes, hipMemcpyDeviceToHost, sc)) != hipSuccess) {
        char what[160];
        snprintf(what, sizeof what, "gls_stream: D2H %d of block %lld (%zu bytes to %p)", q, (long long)blk,
                 d2h[q].bytes, d2h[q].dst);
        return hip_fail(e, what);
      }
    }
    st.d2h_bytes += (sizeof(double) * (p + 2) + sizeof(int32_t)) * cols;
  }
  if ((e = hipEventRecord(wall1, sc)) != hipSuccess) return hip_fail(e, "gls_stream: record");
  if ((e = hipStreamSynchronize(sc)) != hipSuccess) return hip_fail(e, "gls_stream: synchronize");
  if ((e = hipStreamSynchronize(sx)) != hipSuccess) return hip_fail(e, "gls_stream: synchronize");
  float ms = 0.f;
  if ((e = hipEventElapsedTime(&ms, wall0, wall1)) != hipSuccess) return hip_fail(e, "gls_stream: elapsed");
  st.wall_ms = ms;
  for (int64_t blk = 0; blk < nblk; ++blk) {
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, pool.ev[2 * blk], pool.ev[2 * blk + 1])) != hipSuccess)
      return hip_fail(e, "gls_stream: elapsed");
    st.compute_ms += t;
  }
  st.blocks = nblk;
  if (stats_out) *stats_out = st;
  return GLS_OK;
}

// A failed stream drains both streams before returning, so that no copy into
// the caller's host buffers is still in flight.
template <typename T>
static gls_status stream_impl(gls_handle h, int64_t m, int64_t col0, const T* XR_host, int64_t ld_xr, double* b_host,
                              double* sigma2_host, double* v_host, int32_t* status_host, void* compute_stream,
                              void* copy_stream, gls_stream_stats* stats_out) {
  Ctx* c = h;
  if (!c || !c->ready) return arg_fail("gls_stream: handle is not set up"), GLS_ERR_STATE;
  RunStreams rs;
  hipError_t e = run_streams(c, compute_stream, copy_stream, &rs);
  if (e != hipSuccess) return hip_fail(e, "gls_stream: stream order");
  const gls_status r = stream_run(h, m, col0, XR_host, ld_xr, b_host, sigma2_host, v_host, status_host, rs,
                                  stats_out);
  if (r != GLS_OK) {
    (void)hipStreamSynchronize(rs.sc);
    (void)hipStreamSynchronize(rs.sx);
  }
  return r;
}

extern "C" gls_status gls_stream(gls_handle h, int64_t m, int64_t col0, const double* XR_host, int64_t ld_xr,
                                 double* b_host, double* sigma2_host, double* v_host, int32_t* status_host,
                                 void* compute_stream, void* copy_stream, gls_stream_stats* stats_out) {
  return stream_impl(h, m, col0, XR_host, ld_xr, b_host, sigma2_host, v_host, status_host, compute_stream,
                     copy_stream, stats_out);
}

extern "C" gls_status gls_stream_u8(gls_handle h, int64_t m, int64_t col0, const uint8_t* G_host, int64_t ld_g,
                                    double* b_host, double* sigma2_host, double* v_host, int32_t* status_host,
                                    void* compute_stream, void* copy_stream, gls_stream_stats* stats_out) {
  return stream_impl(h, m, col0, G_host, ld_g, b_host, sigma2_host, v_host, status_host, compute_stream,
                     copy_stream, stats_out);
}

extern "C" gls_status gls_stream_u2(gls_handle h, int64_t m, int64_t col0, const uint8_t* G2_host, int64_t ld_g2,
                                    double* b_host, double* sigma2_host, double* v_host, int32_t* status_host,
                                    void* compute_stream, void* copy_stream, gls_stream_stats* stats_out) {
  return stream_impl(h, m, col0, reinterpret_cast<const Packed2*>(G2_host), ld_g2, b_host, sigma2_host, v_host,
                     status_host, compute_stream, copy_stream, stats_out);
}

// ---------------------------------------------------------------------------
// gls_stream_backward: the adjoint of a streamed study.  The SNP blocks take
// the forward stream's route (two device buffers, the next block copied on
// the copy stream while the current one is worked on), and each block's
// cotangents go up on the compute stream just before its adjoint, which
// recomputes the whitened block from the copy it has just received.

static gls_status stream_backward_run(Ctx* c, int64_t m, int64_t col0, const double* XR_host, int64_t ld_xr,
                                      const double* bbar_host, const double* s2bar_host, const double* vbar_host,
                                      double* XR_grad_host, const RunStreams& rs, gls_stream_stats* stats_out) {
  const int64_t rows = c->n;
  const hipStream_t sc = rs.sc;
  const hipStream_t sx = (c->opts.flags & GLS_STREAM_SERIAL) ? sc : rs.sx;
  const int p = c->p;
  const std::vector<int64_t> bstart = block_schedule(c->bc, m - col0);
  const int64_t nblk = (int64_t)bstart.size() - 1;
  gls_stream_stats st{};
  EventPool pool;
  hipError_t e;
  if ((e = pool.make(2 * nblk + 2)) != hipSuccess) return hip_fail(e, "gls_stream_backward: event create");
  hipEvent_t wall0 = pool.ev[2 * nblk], wall1 = pool.ev[2 * nblk + 1];
  auto cols_of = [&](int64_t blk) { return bstart[blk + 1] - bstart[blk]; };
  auto src_of = [&](int64_t blk) { return XR_host + (col0 + bstart[blk]) * ld_xr; };
  auto copy_x = [&](int64_t blk, int buf, hipStream_t s) -> hipError_t {
    hipError_t r = h2d_block(c->buf[buf], rows, src_of(blk), ld_xr, cols_of(blk), s);
    if (r == hipSuccess) r = hipEventRecord(c->ev_copy[buf], s);
    st.h2d_bytes += (int64_t)sizeof(double) * rows * cols_of(blk);
    return r;
  };

  if ((e = hipEventRecord(wall0, sx)) != hipSuccess) return hip_fail(e, "gls_stream_backward: record");
  if ((e = copy_x(0, 0, sx)) != hipSuccess) return hip_fail(e, "gls_stream_backward: H2D");
  for (int64_t blk = 0; blk < nblk; ++blk) {
    const int cur = (int)(blk & 1), nxt = cur ^ 1;
    const int64_t cols = cols_of(blk);
    const int64_t col = col0 + bstart[blk];
    if (blk + 1 < nblk && sx != sc) {
      // the other buffer may only be overwritten once the adjoint that last read it is done
      if (blk >= 1 && (e = hipStreamWaitEvent(sx, c->ev_comp[nxt], 0)) != hipSuccess)
        return hip_fail(e, "gls_stream_backward: wait");
      if ((e = copy_x(blk + 1, nxt, sx)) != hipSuccess) return hip_fail(e, "gls_stream_backward: H2D");
    }
    if (sx == sc && blk >= 1 && (e = copy_x(blk, cur, sc)) != hipSuccess)
      return hip_fail(e, "gls_stream_backward: H2D");
    // this block's cotangents into the result staging buffers (unused by the adjoint itself)
    struct {
      void* dst;
      const void* src;
      size_t bytes;
    } up[3] = {{c->ob, bbar_host + col * p, sizeof(double) * p * cols},
               {c->os2, s2bar_host + col, sizeof(double) * cols},
               {c->ov, vbar_host + col, sizeof(double) * cols}};
    for (int q = 0; q < 3; ++q) {
      if ((e = hipMemcpyAsync(up[q].dst, up[q].src, up[q].bytes, hipMemcpyHostToDevice, sc)) != hipSuccess)
        return hip_fail(e, "gls_stream_backward: cotangent H2D");
      st.h2d_bytes += (int64_t)up[q].bytes;
    }
    if ((e = hipStreamWaitEvent(sc, c->ev_copy[cur], 0)) != hipSuccess) return hip_fail(e, "gls_stream_backward: wait");
    if ((e = hipEventRecord(pool.ev[2 * blk], sc)) != hipSuccess) return hip_fail(e, "gls_stream_backward: record");
    gls_status r = block_backward(c, (int)cols, c->buf[cur], rows, c->ob, c->os2, c->ov, nullptr, sc);
    if (r != GLS_OK) return r;
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "gls_stream_backward: launch");
    if ((e = hipEventRecord(c->ev_comp[cur], sc)) != hipSuccess) return hip_fail(e, "gls_stream_backward: record");
    if ((e = hipEventRecord(pool.ev[2 * blk + 1], sc)) != hipSuccess) return hip_fail(e, "gls_stream_backward: record");
    if (XR_grad_host) {
      // X_R bar of the block stays in Xb (ld N) until the next block's adjoint; copied out before it on the same
      // stream
      if ((e = hipMemcpy2DAsync(XR_grad_host + col * ld_xr, sizeof(double) * ld_xr, c->Xb, sizeof(double) * c->N,
                                sizeof(double) * rows, cols, hipMemcpyDeviceToHost, sc)) != hipSuccess)
        return hip_fail(e, "gls_stream_backward: D2H of the X_R gradient");
      st.d2h_bytes += (int64_t)sizeof(double) * rows * cols;
    }
  }
  if ((e = hipEventRecord(wall1, sc)) != hipSuccess) return hip_fail(e, "gls_stream_backward: record");
  if ((e = hipStreamSynchronize(sc)) != hipSuccess) return hip_fail(e, "gls_stream_backward: synchronize");
  if ((e = hipStreamSynchronize(sx)) != hipSuccess) return hip_fail(e, "gls_stream_backward: synchronize");
  float ms = 0.f;
  if ((e = hipEventElapsedTime(&ms, wall0, wall1)) != hipSuccess) return hip_fail(e, "gls_stream_backward: elapsed");
  st.wall_ms = ms;
  for (int64_t blk = 0; blk < nblk; ++blk) {
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, pool.ev[2 * blk], pool.ev[2 * blk + 1])) != hipSuccess)
      return hip_fail(e, "gls_stream_backward: elapsed");
    st.compute_ms += t;
  }
  st.blocks = nblk;
  if (stats_out) *stats_out = st;
  return GLS_OK;
}

extern "C" gls_status gls_stream_backward(gls_handle h, int64_t m, int64_t col0, const double* XR_host,
                                          int64_t ld_xr, const double* b_bar_host, const double* sigma2_bar_host,
                                          const double* v_bar_host, double* XR_grad_host, void* compute_stream,
                                          void* copy_stream, gls_stream_stats* stats_out) {
  Ctx* c = h;
  if (!c || !c->ready || !c->grad) {
    set_last_error_str("gls_stream_backward: handle not set up with GLS_KEEP_FOR_GRAD");
    return GLS_ERR_STATE;
  }
  if (m < 0 || col0 < 0 || col0 > m) return arg_fail("gls_stream_backward: need 0 <= col0 <= m");
  if (col0 == m) {
    if (stats_out) *stats_out = gls_stream_stats{};
    return GLS_OK;
  }
  if (!XR_host || ld_xr < c->n) return arg_fail("gls_stream_backward: the SNP matrix is NULL or ld_xr < n");
  if (!b_bar_host || !sigma2_bar_host || !v_bar_host) return arg_fail("gls_stream_backward: NULL cotangent");
  RunStreams rs;
  hipError_t e = run_streams(c, compute_stream, copy_stream, &rs);
  if (e != hipSuccess) return hip_fail(e, "gls_stream_backward: stream order");
  const gls_status r = stream_backward_run(c, m, col0, XR_host, ld_xr, b_bar_host, sigma2_bar_host, v_bar_host,
                                           XR_grad_host, rs, stats_out);
  if (r != GLS_OK) {
    (void)hipStreamSynchronize(rs.sc);
    (void)hipStreamSynchronize(rs.sx);
  }
  return r;
}

// ---------------------------------------------------------------------------
// Streaming from storage: reader thread -> three host buffers -> two device
// buffers.

namespace {

struct FileRing {
  std::mutex mu;
  std::condition_variable cv;
  int64_t filled[3] = {-1, -1, -1};  // block held by each host buffer (-1: none)
  bool free_[3] = {true, true, true};
  bool stop = false;
  int err = 0;                        // errno of a failed read, or -1 for a short read
  double read_ms = 0.0;
  int64_t bytes = 0;
};

bool read_fully(int fd, void* dst, size_t len, off_t off, int* err) {
  char* p = static_cast<char*>(dst);
  while (len > 0) {
    ssize_t r = pread(fd, p, len, off);
    if (r < 0) {
      if (errno == EINTR) continue;
      *err = errno;
      return false;
    }
    if (r == 0) {
      *err = -1;
      return false;
    }
    p += r;
    off += r;
    len -= (size_t)r;
  }
  return true;
}

// three host buffers of one block each; col_bytes: bytes per SNP column
size_t host_ring_bytes(const Ctx* c, int64_t col_bytes) {
  const size_t one = (size_t)col_bytes * (size_t)c->bc;
  return 3 * ((one + 4095) / 4096 * 4096);
}

// The work a file stream does on each block once its columns are in device buffer X (rows elements per column,
// dense), on the compute stream: the forward solve and its results, or the adjoint.
template <typename T>
struct FileForward {
  double* b_host;
  double* sigma2_host;
  double* v_host;
  int32_t* status_host;
  gls_status block(Ctx* c, const T* X, int64_t rows, int64_t, int64_t cols, hipStream_t sc, gls_stream_stats*) const {
    return solve_block(c, (int)cols, X, rows, c->ob, c->p, c->os2, c->ov, c->ost, sc);
  }
  // results of the block, after its timing event
  hipError_t after(Ctx* c, int64_t col, int64_t cols, hipStream_t sc, gls_stream_stats* st) const {
    const int p = c->p;
    hipError_t e;
    if ((e = hipMemcpyAsync(b_host + col * p, c->ob, sizeof(double) * p * cols, hipMemcpyDeviceToHost, sc)) ||
        (e = hipMemcpyAsync(sigma2_host + col, c->os2, sizeof(double) * cols, hipMemcpyDeviceToHost, sc)) ||
        (e = hipMemcpyAsync(v_host + col, c->ov, sizeof(double) * cols, hipMemcpyDeviceToHost, sc)) ||
        (e = hipMemcpyAsync(status_host + col, c->ost, sizeof(int32_t) * cols, hipMemcpyDeviceToHost, sc)))
      return e;
    st->d2h_bytes += (int64_t)(sizeof(double) * (p + 2) + sizeof(int32_t)) * cols;
    return hipSuccess;
  }
};

// FP64 columns of a block for the adjoint: FP64 input as it is, bytes and packed dosages widened into the
// handle's zero-padded FP64 staging buffer.
const double* fp64_columns(Ctx*, const double* X, int64_t rows, int64_t, hipStream_t, int64_t* ld) {
  *ld = rows;
  return X;
}
const double* fp64_columns(Ctx* c, const uint8_t* X, int64_t rows, int64_t cols, hipStream_t s, int64_t* ld) {
  widen_u8(c, X, rows, (int)cols, s);
  *ld = c->N;
  return c->x64;
}
const double* fp64_columns(Ctx* c, const Packed2* X, int64_t rows, int64_t cols, hipStream_t s, int64_t* ld) {
  widen_u2(c, reinterpret_cast<const uint8_t*>(X), rows, (int)cols, s);
  *ld = c->N;
  return c->x64;
}

template <typename T>
struct FileBackward {
  const double* bbar_host;
  const double* s2bar_host;
  const double* vbar_host;
  double* XR_grad_host;   // n x m, ld n, or NULL
  gls_status block(Ctx* c, const T* X, int64_t rows, int64_t col, int64_t cols, hipStream_t sc,
                   gls_stream_stats* st) const {
    const int p = c->p;
    struct {
      void* dst;
      const void* src;
      size_t bytes;
    } up[3] = {{c->ob, bbar_host + col * p, sizeof(double) * p * cols},
               {c->os2, s2bar_host + col, sizeof(double) * cols},
               {c->ov, vbar_host + col, sizeof(double) * cols}};
    for (int q = 0; q < 3; ++q) {
      const hipError_t e = hipMemcpyAsync(up[q].dst, up[q].src, up[q].bytes, hipMemcpyHostToDevice, sc);
      if (e != hipSuccess) return hip_fail(e, "gls_stream_backward_file: cotangent H2D");
      st->h2d_bytes += (int64_t)up[q].bytes;
    }
    int64_t ld = 0;
    const double* Xd = fp64_columns(c, X, rows, cols, sc, &ld);
    return block_backward(c, (int)cols, Xd, ld, c->ob, c->os2, c->ov, nullptr, sc);
  }
  hipError_t after(Ctx* c, int64_t col, int64_t cols, hipStream_t sc, gls_stream_stats* st) const {
    if (!XR_grad_host) return hipSuccess;
    // X_R bar of the block stays in Xb (ld N) until the next block's adjoint, queued behind this copy
    const hipError_t e = hipMemcpy2DAsync(XR_grad_host + col * c->n, sizeof(double) * c->n, c->Xb,
                                          sizeof(double) * c->N, sizeof(double) * c->n, cols, hipMemcpyDeviceToHost, sc);
    if (e == hipSuccess) st->d2h_bytes += (int64_t)sizeof(double) * c->n * cols;
    return e;
  }
};

template <typename T, typename Op>
gls_status stream_file_impl(Ctx* c, int fd, int64_t offset, int64_t m, int64_t col0, char* host, const Op& op,
                            hipStream_t sc, hipStream_t sx_in, gls_stream_stats* stats_out) {
  const int64_t bc = c->bc, rows = col_elems(c, (const T*)nullptr);
  const bool serial = (c->opts.flags & GLS_STREAM_SERIAL) != 0;
  hipStream_t sx = serial ? sc : sx_in;
  const std::vector<int64_t> bstart = block_schedule(bc, m - col0);   // opening ramp as in gls_stream
  const int64_t nblk = (int64_t)bstart.size() - 1;
  gls_stream_stats st{};
  if (nblk == 0) {
    if (stats_out) *stats_out = st;
    return GLS_OK;
  }
  const size_t slot_bytes = host_ring_bytes(c, rows * (int64_t)sizeof(T)) / 3;
  T* hb[3];
  for (int i = 0; i < 3; ++i) hb[i] = reinterpret_cast<T*>(host + i * slot_bytes);
  auto cols_of = [&](int64_t blk) { return bstart[blk + 1] - bstart[blk]; };
  auto file_off = [&](int64_t blk) { return (off_t)(offset + (col0 + bstart[blk]) * rows * (int64_t)sizeof(T)); };

  EventPool pool;
  hipError_t e;
  // per block: compute start/stop, H2D done; plus wall start/stop
  if ((e = pool.make(3 * nblk + 2)) != hipSuccess) return hip_fail(e, "gls_stream_file: event create");
  hipEvent_t wall0 = pool.ev[3 * nblk], wall1 = pool.ev[3 * nblk + 1];
  auto ev_h2d = [&](int64_t blk) { return pool.ev[2 * nblk + blk]; };

  FileRing ring;
  std::thread reader;
  if (!serial) {
    reader = std::thread([&] {
      for (int64_t blk = 0; blk < nblk; ++blk) {
        const int slot = (int)(blk % 3);
        {
          std::unique_lock<std::mutex> lk(ring.mu);
          ring.cv.wait(lk, [&] { return ring.free_[slot] || ring.stop; });
          if (ring.stop) return;
          ring.free_[slot] = false;
        }
        const size_t len = (size_t)(cols_of(blk) * rows) * sizeof(T);
        int err = 0;
        auto t0 = std::chrono::steady_clock::now();
        const bool ok = read_fully(fd, hb[slot], len, file_off(blk), &err);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        std::lock_guard<std::mutex> lk(ring.mu);
        ring.read_ms += ms;
        if (!ok) {
          ring.err = err;
          ring.cv.notify_all();
          return;
        }
        ring.bytes += (int64_t)len;
        ring.filled[slot] = blk;
        ring.cv.notify_all();
      }
    });
  }
  auto finish_reader = [&] {
    if (reader.joinable()) {
      {
        std::lock_guard<std::mutex> lk(ring.mu);
        ring.stop = true;
      }
      ring.cv.notify_all();
      reader.join();
    }
  };
  auto fail = [&](gls_status s) {
    finish_reader();
    (void)hipStreamSynchronize(sc);
    (void)hipStreamSynchronize(sx);
    return s;
  };

  if ((e = hipEventRecord(wall0, sx)) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: record"));
  for (int64_t blk = 0; blk < nblk; ++blk) {
    const int slot = (int)(blk % 3), cur = (int)(blk & 1);
    const int64_t cols = cols_of(blk);
    const int64_t col = col0 + bstart[blk];
    if (serial) {
      int err = 0;
      auto t0 = std::chrono::steady_clock::now();
      const size_t len = (size_t)(cols * rows) * sizeof(T);
      if (!read_fully(fd, hb[slot], len, file_off(blk), &err)) {
        set_last_error_str(err > 0 ? "gls_stream_file: read failed" : "gls_stream_file: file shorter than m columns");
        return fail(GLS_ERR_STATE);
      }
      ring.read_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      ring.bytes += (int64_t)len;
    } else {
      std::unique_lock<std::mutex> lk(ring.mu);
      ring.cv.wait(lk, [&] { return ring.filled[slot] == blk || ring.err != 0; });
      if (ring.err != 0 && ring.filled[slot] != blk) {
        const int err = ring.err;
        lk.unlock();
        set_last_error_str(err > 0 ? "gls_stream_file: read failed" : "gls_stream_file: file shorter than m columns");
        return fail(GLS_ERR_STATE);
      }
    }
    // device buffer cur may be overwritten once the solve two blocks back is done
    if (!serial && blk >= 2 && (e = hipStreamWaitEvent(sx, c->ev_comp[cur], 0)) != hipSuccess)
      return fail(hip_fail(e, "gls_stream_file: wait"));
    if ((e = h2d_block(stage(c, cur, (const T*)nullptr), rows, hb[slot], rows, cols, sx)) != hipSuccess)
      return fail(hip_fail(e, "gls_stream_file: H2D"));
    if ((e = hipEventRecord(ev_h2d(blk), sx)) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: record"));
    st.h2d_bytes += (int64_t)sizeof(T) * rows * cols;
    if ((e = hipStreamWaitEvent(sc, ev_h2d(blk), 0)) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: wait"));
    if ((e = hipEventRecord(pool.ev[2 * blk], sc)) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: record"));
    gls_status r = op.block(c, stage(c, cur, (const T*)nullptr), rows, col, cols, sc, &st);
    if (r != GLS_OK) return fail(r);
    if ((e = hipGetLastError()) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: launch"));
    if ((e = hipEventRecord(c->ev_comp[cur], sc)) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: record"));
    if ((e = hipEventRecord(pool.ev[2 * blk + 1], sc)) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: record"));
    if ((e = op.after(c, col, cols, sc, &st)) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: D2H"));
    if (serial) {
      if ((e = hipStreamSynchronize(sc)) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: synchronize"));
    } else if (blk >= 1) {
      // the previous block's host buffer is free once its copy has landed
      if ((e = hipEventSynchronize(ev_h2d(blk - 1))) != hipSuccess)
        return fail(hip_fail(e, "gls_stream_file: synchronize"));
      std::lock_guard<std::mutex> lk(ring.mu);
      ring.free_[(blk - 1) % 3] = true;
      ring.filled[(blk - 1) % 3] = -1;
      ring.cv.notify_all();
    }
  }
  if ((e = hipEventRecord(wall1, sc)) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: record"));
  if ((e = hipStreamSynchronize(sc)) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: synchronize"));
  if ((e = hipStreamSynchronize(sx)) != hipSuccess) return fail(hip_fail(e, "gls_stream_file: synchronize"));
  finish_reader();
  float ms = 0.f;
  if ((e = hipEventElapsedTime(&ms, wall0, wall1)) != hipSuccess) return hip_fail(e, "gls_stream_file: elapsed");
  st.wall_ms = ms;
  for (int64_t blk = 0; blk < nblk; ++blk) {
    float t = 0.f;
    if ((e = hipEventElapsedTime(&t, pool.ev[2 * blk], pool.ev[2 * blk + 1])) != hipSuccess)
      return hip_fail(e, "gls_stream_file: elapsed");
    st.compute_ms += t;
  }
  st.blocks = nblk;
  st.file_bytes = ring.bytes;
  st.read_ms = ring.read_ms;
  if (stats_out) *stats_out = st;
  return GLS_OK;
}

}  // namespace

namespace {
// bytes per SNP column in a file of elem_bits-bit entries (64, 8 or 2); 0 if invalid
int64_t file_col_bytes(const Ctx* c, int32_t elem_bits) {
  switch (elem_bits) {
    case 64: return 8 * c->n;
    case 8: return c->n;
    case 2: return (c->n + 3) / 4;
    default: return 0;
  }
}
}  // namespace

extern "C" size_t gls_stream_file_host_bytes(gls_handle h, int32_t elem_bits) {
  const Ctx* c = h;
  if (!c || !c->ready || file_col_bytes(c, elem_bits) == 0) return 0;
  return host_ring_bytes(c, file_col_bytes(c, elem_bits));
}

extern "C" gls_status gls_stream_file(gls_handle h, const char* path, int64_t offset, int32_t elem_bits, int64_t m,
                                      int64_t col0, void* host_ws, size_t host_ws_bytes, double* b_host,
                                      double* sigma2_host, double* v_host, int32_t* status_host,
                                      void* compute_stream, void* copy_stream, gls_stream_stats* stats_out) {
  Ctx* c = h;
  if (!c || !c->ready) return arg_fail("gls_stream_file: handle is not set up"), GLS_ERR_STATE;
  if (!path || offset < 0 || m < 0 || col0 < 0 || col0 > m) return arg_fail("gls_stream_file: bad path/offset/m/col0");
  if (file_col_bytes(c, elem_bits) == 0) return arg_fail("gls_stream_file: elem_bits must be 64, 8 or 2");
  if (col0 == m) {   // nothing to read: neither the file nor any buffer is used
    if (stats_out) *stats_out = gls_stream_stats{};
    return GLS_OK;
  }
  if (!host_ws || host_ws_bytes < host_ring_bytes(c, file_col_bytes(c, elem_bits)))
    return arg_fail("gls_stream_file: host_ws smaller than gls_stream_file_host_bytes()");
  if (!b_host || !sigma2_host || !v_host || !status_host) return arg_fail("gls_stream_file: NULL host output");
  const int fd = open(path, O_RDONLY);
  if (fd < 0) return arg_fail("gls_stream_file: cannot open the file");
  gls_status st;
  RunStreams rs;
  const hipError_t e = run_streams(c, compute_stream, copy_stream, &rs);
  if (e != hipSuccess) {
    close(fd);
    return hip_fail(e, "gls_stream_file: stream order");
  }
  const hipStream_t sc = rs.sc, sx = rs.sx;
  char* ring = static_cast<char*>(host_ws);
  if (elem_bits == 64)
    st = stream_file_impl<double>(c, fd, offset, m, col0, ring,
                                  FileForward<double>{b_host, sigma2_host, v_host, status_host}, sc, sx, stats_out);
  else if (elem_bits == 8)
    st = stream_file_impl<uint8_t>(c, fd, offset, m, col0, ring,
                                   FileForward<uint8_t>{b_host, sigma2_host, v_host, status_host}, sc, sx, stats_out);
  else
    st = stream_file_impl<Packed2>(c, fd, offset, m, col0, ring,
                                   FileForward<Packed2>{b_host, sigma2_host, v_host, status_host}, sc, sx, stats_out);
  close(fd);
  return st;
}

extern "C" gls_status gls_stream_backward_file(gls_handle h, const char* path, int64_t offset, int32_t elem_bits,
                                               int64_t m, int64_t col0, void* host_ws, size_t host_ws_bytes,
                                               const double* b_bar_host, const double* sigma2_bar_host,
                                               const double* v_bar_host, double* XR_grad_host, void* compute_stream,
                                               void* copy_stream, gls_stream_stats* stats_out) {
  Ctx* c = h;
  if (!c || !c->ready || !c->grad) {
    set_last_error_str("gls_stream_backward_file: handle not set up with GLS_KEEP_FOR_GRAD");
    return GLS_ERR_STATE;
  }
  if (!path || offset < 0 || m < 0 || col0 < 0 || col0 > m)
    return arg_fail("gls_stream_backward_file: bad path/offset/m/col0");
  if (file_col_bytes(c, elem_bits) == 0) return arg_fail("gls_stream_backward_file: elem_bits must be 64, 8 or 2");
  if (col0 == m) {
    if (stats_out) *stats_out = gls_stream_stats{};
    return GLS_OK;
  }
  if (!host_ws || host_ws_bytes < host_ring_bytes(c, file_col_bytes(c, elem_bits)))
    return arg_fail("gls_stream_backward_file: host_ws smaller than gls_stream_file_host_bytes()");
  if (!b_bar_host || !sigma2_bar_host || !v_bar_host) return arg_fail("gls_stream_backward_file: NULL cotangent");
  const int fd = open(path, O_RDONLY);
  if (fd < 0) return arg_fail("gls_stream_backward_file: cannot open the file");
  RunStreams rs;
  const hipError_t e = run_streams(c, compute_stream, copy_stream, &rs);
  if (e != hipSuccess) {
    close(fd);
    return hip_fail(e, "gls_stream_backward_file: stream order");
  }
  char* ring = static_cast<char*>(host_ws);
  gls_status st;
  if (elem_bits == 64)
    st = stream_file_impl<double>(c, fd, offset, m, col0, ring,
                                  FileBackward<double>{b_bar_host, sigma2_bar_host, v_bar_host, XR_grad_host}, rs.sc,
                                  rs.sx, stats_out);
  else if (elem_bits == 8)
    st = stream_file_impl<uint8_t>(c, fd, offset, m, col0, ring,
                                   FileBackward<uint8_t>{b_bar_host, sigma2_bar_host, v_bar_host, XR_grad_host},
                                   rs.sc, rs.sx, stats_out);
  else
    st = stream_file_impl<Packed2>(c, fd, offset, m, col0, ring,
                                   FileBackward<Packed2>{b_bar_host, sigma2_bar_host, v_bar_host, XR_grad_host},
                                   rs.sc, rs.sx, stats_out);
  close(fd);
  return st;
}
