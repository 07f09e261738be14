// gls_stream: the GPU half of the paper's multi-level buffering (Sec. 3.1).
//
// Two device buffers alternate roles: while block b is solved in buffer
// alpha on the compute stream, block b+1 is copied from page-locked host
// memory into buffer beta on the copy stream.  Roles rotate by index, never
// by copying.  Unlike the paper's design, the whitened block never returns to
// the host: the per-SNP products and solves run on the GPU right after the
// triangular product, and only b, sigma2, v and status go back.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
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

template <typename T>
hipError_t h2d_block(T* dst, int64_t n, const T* src, int64_t ld, int64_t cols, hipStream_t s) {
  if (ld == n) return hipMemcpyAsync(dst, src, sizeof(T) * n * cols, hipMemcpyHostToDevice, s);
  return hipMemcpy2DAsync(dst, sizeof(T) * n, src, sizeof(T) * ld, sizeof(T) * n, cols, hipMemcpyHostToDevice, s);
}

double* stage(Ctx* c, int i, const double*) { return c->buf[i]; }
uint8_t* stage(Ctx* c, int i, const uint8_t*) { return c->ub[i]; }

gls_status solve_block(Ctx* c, int mb, const double* X, int64_t ld, double* b, int64_t ldb, double* s2, double* v,
                       int* st, hipStream_t s) {
  return block_forward(c, mb, X, ld, b, ldb, s2, v, st, s);
}
gls_status solve_block(Ctx* c, int mb, const uint8_t* X, int64_t ld, double* b, int64_t ldb, double* s2, double* v,
                       int* st, hipStream_t s) {
  return block_forward_u8(c, mb, X, ld, b, ldb, s2, v, st, s);
}

}  // namespace

template <typename T>
static gls_status stream_impl(gls_handle h, int64_t m, int64_t col0, const T* XR_host, int64_t ld_xr, double* b_host,
                              double* sigma2_host, double* v_host, int32_t* status_host, void* compute_stream,
                              void* copy_stream, gls_stream_stats* stats_out) {
  Ctx* c = h;
  if (!c || !c->ready) return arg_fail("gls_stream: handle is not set up"), GLS_ERR_STATE;
  if (m < 0 || col0 < 0 || col0 > m) return arg_fail("gls_stream: need 0 <= col0 <= m");
  if (!XR_host || ld_xr < c->n) return arg_fail("gls_stream: XR_host is NULL or ld_xr < n");
  if (!b_host || !sigma2_host || !v_host || !status_host) return arg_fail("gls_stream: NULL host output");
  hipStream_t sc = static_cast<hipStream_t>(compute_stream);
  // serial mode: every copy on the compute stream, so nothing overlaps
  hipStream_t sx = (c->opts.flags & GLS_STREAM_SERIAL) ? sc : static_cast<hipStream_t>(copy_stream);
  const int64_t n = c->n, bc = c->bc;
  const int p = c->p;
  const int64_t nblk = (m - col0 + bc - 1) / bc;
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

  auto cols_of = [&](int64_t blk) { return std::min<int64_t>(bc, m - col0 - blk * bc); };
  auto src_of = [&](int64_t blk) { return XR_host + (col0 + blk * bc) * ld_xr; };

  if ((e = hipEventRecord(wall0, sx)) != hipSuccess) return hip_fail(e, "gls_stream: record");
  if ((e = h2d_block(stage(c, 0, XR_host), n, src_of(0), ld_xr, cols_of(0), sx)) != hipSuccess)
    return hip_fail(e, "gls_stream: H2D");
  if ((e = hipEventRecord(c->ev_copy[0], sx)) != hipSuccess) return hip_fail(e, "gls_stream: record");
  st.h2d_bytes += sizeof(T) * n * cols_of(0);

  for (int64_t blk = 0; blk < nblk; ++blk) {
    const int cur = (int)(blk & 1), nxt = cur ^ 1;
    const int64_t cols = cols_of(blk);
    const int64_t col = col0 + blk * bc;
    if (blk + 1 < nblk && sx != sc) {
      // beta may only be overwritten once the solve that last read it is done
      if (blk >= 1 && (e = hipStreamWaitEvent(sx, c->ev_comp[nxt], 0)) != hipSuccess)
        return hip_fail(e, "gls_stream: wait");
      if ((e = h2d_block(stage(c, nxt, XR_host), n, src_of(blk + 1), ld_xr, cols_of(blk + 1), sx)) != hipSuccess)
        return hip_fail(e, "gls_stream: H2D");
      if ((e = hipEventRecord(c->ev_copy[nxt], sx)) != hipSuccess) return hip_fail(e, "gls_stream: record");
      st.h2d_bytes += sizeof(T) * n * cols_of(blk + 1);
    }
    if (sx == sc && blk >= 1) {   // serial: this block's copy only now, behind the previous results
      if ((e = h2d_block(stage(c, cur, XR_host), n, src_of(blk), ld_xr, cols, sc)) != hipSuccess)
        return hip_fail(e, "gls_stream: H2D");
      if ((e = hipEventRecord(c->ev_copy[cur], sc)) != hipSuccess) return hip_fail(e, "gls_stream: record");
      st.h2d_bytes += sizeof(T) * n * cols;
    }
    if ((e = hipStreamWaitEvent(sc, c->ev_copy[cur], 0)) != hipSuccess) return hip_fail(e, "gls_stream: wait");
    if ((e = hipEventRecord(pool.ev[2 * blk], sc)) != hipSuccess) return hip_fail(e, "gls_stream: record");
    gls_status r = solve_block(c, (int)cols, stage(c, cur, XR_host), n, c->ob, p, c->os2, c->ov, c->ost, sc);
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
