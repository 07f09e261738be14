/*
 * gls.h -- C-ABI of libgls, the MI355X (gfx950) streamed GWAS GLS solver.
 *
 * For every SNP i the library computes (paper Sec. 1.3, Eq. 1)
 *
 *     b_i = (X_i^T M^-1 X_i)^-1 X_i^T M^-1 y,   X_i = [X_L | x_R,i] (n x p),
 *     M   = h2 * Phi + (1 - h2) * I,
 *
 * by the Cholesky rewrite (Sec. 2.1, Eq. 2) and the structured algorithm of
 * Sec. 2.1 (Listing 1): one Cholesky M = L L^T per study, the covariate terms
 * X~_L = L^-1 X_L, y~ = L^-1 y, r~_T = X~_L^T y~, S_TL = X~_L^T X~_L hoisted
 * out of the SNP loop, then per block of SNP columns X~_R,b = L^-1 X_R,b
 * (Sec. 2.2: SNP vectors packed so the solve is one level-3 operation),
 * the per-SNP products S_BL,i, S_BR,i, r~_B,i and the p x p SPD solve.
 * Beyond b_i each SNP also gets
 *     sigma2_i = (y~^T y~ - b_i^T r~_i) / (n - p)   (GLS residual variance),
 *     v_i      = (S_i^-1)_pp                          (so se_i = sqrt(sigma2_i v_i)),
 *     status_i = 0 ok, 1 S_i numerically singular (b_i, sigma2_i, v_i = NaN).
 * S_i counts as singular when its last squared Cholesky pivot is not above
 * 2^-40 * S_BR,i.
 *
 * Conventions
 *   - Every matrix is column-major FP64.  A SNP block X_R is n x mb with
 *     leading dimension ld_xr >= n: SNP j's n samples are contiguous (a torch
 *     (mb, n) row-major tensor is the same memory).  Coefficients b are
 *     p x mb with ld_b >= p: SNP j's p coefficients are contiguous, ordered
 *     [covariates..., SNP].
 *   - Pointers are DEVICE pointers unless the name ends in _host.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - The caller owns every input, output and the workspace.  The library
 *     never allocates device memory.  Host-side resources: the small handle
 *     with its HIP events and two streams of its own for streamed studies
 *     (see gls_stream), freed by gls_destroy; gls_setup also creates a side
 *     stream and events of its own, which it synchronizes and destroys before
 *     returning; gls_stream_file runs a reader thread that is joined before
 *     the call returns.
 *     gls_setup also creates events of its own, which it destroys before
 *     returning; gls_stream_file runs a reader thread that is joined before
 *     the call returns.
 *   - Work the library enqueues on a caller's stream reads and writes the
 *     workspace asynchronously: the workspace must not be freed or reused
 *     until that stream has finished it.
 *   - Every call returns a gls_status; no C++ exception crosses the ABI.
 *     gls_last_error() gives a thread-local message for the last failure.
 */
#ifndef GLS_H
#define GLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gls_ctx* gls_handle;

typedef enum {
  GLS_OK = 0,
  GLS_ERR_ARG = -1,       /* bad size, leading dimension, pointer or option      */
  GLS_ERR_NOT_SPD = -2,   /* M is not SPD; *info = 1-based failing pivot          */
  GLS_ERR_HIP = -3,       /* a HIP runtime call failed                            */
  GLS_ERR_WORKSPACE = -4, /* workspace smaller than gls_workspace_bytes, or not
                             256-byte aligned                                     */
  GLS_ERR_STATE = -5,     /* call not valid in the handle's state                 */
  GLS_ERR_RANK = -6       /* X_L rank deficient: a squared pivot of S_TL at or
                             below 2^-40 of its diagonal entry; *info = 1-based
                             covariate index                                      */
} gls_status;

/* Arithmetic of the per-block triangular solve (everything else is FP64). */
typedef enum {
  GLS_FP64 = 0,     /* plain FP64 MFMA                                           */
  GLS_FP32_IR = 1,  /* FP32 MFMA bulk + FP64 residual refinement sweeps          */
  GLS_FP16_IR = 2,  /* FP16 MFMA (power-of-two column scaling) + FP64 refinement */
  GLS_BF16_IR = 3,  /* BF16 MFMA (power-of-two column scaling) + FP64 refinement */
  GLS_INT8_EMU = 4  /* dosage input only (the _u8 and _u2 entry points): the product
                       with L^-1 as eight exact int8 slice products on the integer
                       matrix cores, combined in FP64 (FP64-level accuracy); FP64
                       input on such a handle runs the plain FP64 product        */
} gls_precision;

/* gls_opts.flags: keep Phi and the factor terms needed by the adjoint. */
#define GLS_KEEP_FOR_GRAD 1u
/* gls_opts.flags: gls_stream without overlap (copy, solve and results one
 * after another on the compute stream): the naive offloading pattern of the
 * paper's Sec. 3, for comparison with the double-buffered default. */
#define GLS_STREAM_SERIAL 2u

typedef struct {
  int32_t precision;      /* gls_precision                                       */
  int32_t refine_sweeps;  /* 0..4 refinement sweeps (mixed precision only)       */
  int32_t block_cols;     /* largest mb any later gls_block call will use (>= 1) */
  uint32_t flags;         /* GLS_KEEP_FOR_GRAD                                   */
} gls_opts;

/* Device workspace (bytes) a handle with these sizes and options needs.
 * Returns 0 for invalid arguments (n <= p, n > 2^20, p < 1, p > 20,
 * block_cols < 1, refine_sweeps outside 0..4, unknown precision). */
size_t gls_workspace_bytes(int64_t n, int32_t p, const gls_opts* opts);

/* Study setup (Sec. 2.1, Listing 1 before the SNP loop; Eq. 2):
 *   M = h2 Phi + (1 - h2) I, L = chol(M), the inverse factor L^-1 (blocked:
 *   inverted diagonal blocks and FP64 MFMA updates), X~_L, y~, S_TL, r~_T,
 *   y~^T y~, and the Cholesky factor of S_TL.
 * Phi: n x n symmetric (only its lower triangle is read), ld_phi >= n.
 * XL : n x (p-1) fixed covariates, ld_xl >= n (may be NULL when p == 1).
 * y  : n phenotype values.
 * workspace: device buffer of at least gls_workspace_bytes(n, p, opts) bytes,
 *   256-byte aligned; it must outlive the handle.  Inputs may be freed once
 *   gls_setup returns.
 * Synchronizes `stream` before returning so that failures are reported:
 *   GLS_ERR_NOT_SPD (*info = failing pivot, 1-based) or GLS_ERR_RANK
 *   (*info = failing covariate, 1-based); *info = 0 on success.  `info` may be
 *   NULL.  On failure *out is NULL. */
gls_status gls_setup(gls_handle* out, int64_t n, int32_t p,
                     const double* Phi, int64_t ld_phi, double h2,
                     const double* XL, int64_t ld_xl, const double* y,
                     void* workspace, size_t ws_bytes, const gls_opts* opts,
                     void* stream, int64_t* info);

/* One SNP block (Sec. 2.2 and the SNP loop of Sec. 2.1): X~_R,b = L^-1 X_R,b,
 * the per-SNP products and the p x p solves.
 * XR: n x mb (ld_xr >= n), 1 <= mb <= opts.block_cols; it is not modified.
 * Outputs: b (p x mb, ld_b >= p), sigma2 (mb), v (mb), snp_status (mb).
 * Asynchronous on `stream`.  Results depend only on each SNP's column, not on
 * mb or on the column's position in the block (bitwise). */
gls_status gls_block(gls_handle h, int32_t mb, const double* XR, int64_t ld_xr,
                     double* b, int64_t ld_b, double* sigma2, double* v,
                     int32_t* snp_status, void* stream);

/* One SNP block (Sec. 2.2, as gls_block) given as genotype bytes: G is
 * n x mb uint8 (ld_g >= n), entries 0..127 (dosages 0, 1, 2).  GLS_INT8_EMU
 * sums exact int32 products, so it needs n * 127 * max(G) < 2^31: any byte
 * value for n <= 133,000, dosages 0..2 for n up to 8.4 million.  Same outputs and asynchrony as
 * gls_block.  With GLS_FP64 or the mixed forms the bytes are widened to FP64
 * on the device and the results are bitwise those of gls_block on the same
 * values; with GLS_INT8_EMU the product runs on the integer matrix cores
 * (see gls_precision).  Moves 1 byte per sample instead of 8. */
gls_status gls_block_u8(gls_handle h, int32_t mb, const uint8_t* G, int64_t ld_g,
                        double* b, int64_t ld_b, double* sigma2, double* v,
                        int32_t* snp_status, void* stream);

/* One SNP block (Sec. 2.2, as gls_block) given as packed 2-bit dosages:
 * column j occupies bytes [j * ld_g2, j * ld_g2 + ceil(n / 4)) of G2
 * (ld_g2 >= ceil(n / 4)); sample k's dosage is the 2-bit code in bits
 * [2 (k % 4), 2 (k % 4) + 2) of the column's byte k / 4, read as the integer
 * 0..3 (no missing-value code).  Bits of a
 * column's last byte past sample n - 1 are ignored.  The codes are expanded
 * on the device, and the results are bitwise those of gls_block_u8 on the same
 * dosages as bytes (every precision).  Moves a quarter byte per sample.  Same
 * outputs, errors and asynchrony as gls_block. */
gls_status gls_block_u2(gls_handle h, int32_t mb, const uint8_t* G2, int64_t ld_g2,
                        double* b, int64_t ld_b, double* sigma2, double* v,
                        int32_t* snp_status, void* stream);

/* Per-stream timing and byte counts filled by gls_stream (may be NULL). */
typedef struct {
  int64_t blocks;        /* blocks processed                                  */
  int64_t h2d_bytes;     /* host-to-device bytes                              */
  int64_t d2h_bytes;     /* device-to-host bytes                              */
  double wall_ms;        /* first copy enqueue to last result landed          */
  double compute_ms;     /* sum over blocks of the block's device time        */
  int64_t file_bytes;    /* bytes read from storage (gls_stream_file)         */
  double read_ms;        /* time the reader spent in read calls (gls_stream_file) */
} gls_stream_stats;

/* Streamed study (Sec. 3.1, the GPU half of the double/triple buffering):
 * SNP columns [col0, m) of XR_host (n x m, ld_xr >= n, page-locked host
 * memory) are moved block by block into two device buffers (alpha computes
 * while beta receives the next block on `copy_stream`), solved on
 * `compute_stream`, and the results are copied into the host arrays
 * b_host (p x m, ld = p), sigma2_host, v_host, status_host at the same
 * column offsets.  Blocks of opts.block_cols columns; the last one is ragged.
 * With block_cols >= 2,048 the stream starts with shorter blocks
 * (block_cols / 8, growing by a quarter per block, multiples of 64), so the
 * first copy, which nothing overlaps, is short; results are bitwise the same
 * for any blocking.
 * copy_stream NULL (recommended): the study runs on the handle's own compute
 * and copy streams, after the work already queued on compute_stream.  HIP
 * multiplexes streams onto a few hardware queues, and on a shared queue the
 * copy pipeline's cross-stream waits hold up the other stream: copies and
 * solves would run one after another.  gls_setup therefore checks that a wait
 * on its copy stream does not hold up its compute stream, and re-creates the
 * copy stream (at most four times) until it does not.  A caller-given copy
 * stream gets no such check.
 * Returns after every result has landed.  col0 > 0 resumes an interrupted
 * run: outputs for columns < col0 are not touched.  col0 == m (an empty
 * stream) returns GLS_OK at once, and the pointers may then be NULL. */
gls_status gls_stream(gls_handle h, int64_t m, int64_t col0,
                      const double* XR_host, int64_t ld_xr,
                      double* b_host, double* sigma2_host, double* v_host,
                      int32_t* status_host, void* compute_stream, void* copy_stream,
                      gls_stream_stats* stats_out);

/* gls_stream (Sec. 3.1) for genotype bytes: G_host is n x m uint8 (ld_g >= n) in
 * page-locked host memory; blocks are processed as by gls_block_u8. */
gls_status gls_stream_u8(gls_handle h, int64_t m, int64_t col0,
                         const uint8_t* G_host, int64_t ld_g,
                         double* b_host, double* sigma2_host, double* v_host,
                         int32_t* status_host, void* compute_stream, void* copy_stream,
                         gls_stream_stats* stats_out);

/* gls_stream (Sec. 3.1) for packed 2-bit dosages: G2_host holds m columns of
 * ceil(n / 4) bytes at stride ld_g2 (>= ceil(n / 4)) bytes, in page-locked host
 * memory, in the layout of gls_block_u2; blocks are processed as by
 * gls_block_u2. */
gls_status gls_stream_u2(gls_handle h, int64_t m, int64_t col0,
                         const uint8_t* G2_host, int64_t ld_g2,
                         double* b_host, double* sigma2_host, double* v_host,
                         int32_t* status_host, void* compute_stream, void* copy_stream,
                         gls_stream_stats* stats_out);

/* Streamed study read from storage (Sec. 3.1, both buffering levels): the
 * SNP matrix is a file holding SNP j's n samples contiguously at byte
 * offset + j * c, as FP64 (elem_bits 64, c = 8 n), genotype bytes (elem_bits 8,
 * c = n) or packed 2-bit dosages in the layout of gls_block_u2 (elem_bits 2,
 * c = ceil(n / 4)).  A reader thread reads block b+2 into one of three
 * page-locked host buffers while block b+1 waits in another and block b is
 * copied to the device (two device buffers alternate as in gls_stream); a
 * host buffer is reused only once its copy has completed.  Blocks follow
 * gls_stream's schedule, opening ramp included.  host_ws is the
 * caller's page-locked host memory of gls_stream_file_host_bytes() bytes.
 * Outputs, col0 and return as gls_stream; read errors give GLS_ERR_ARG
 * (unopenable file) or GLS_ERR_STATE (short read), with gls_last_error().
 * With GLS_STREAM_SERIAL the calling thread reads, copies and solves one
 * block after another (no overlap at either level). */
size_t gls_stream_file_host_bytes(gls_handle h, int32_t elem_bits);
gls_status gls_stream_file(gls_handle h, const char* path, int64_t offset, int32_t elem_bits,
                           int64_t m, int64_t col0, void* host_ws, size_t host_ws_bytes,
                           double* b_host, double* sigma2_host, double* v_host,
                           int32_t* status_host, void* compute_stream, void* copy_stream,
                           gls_stream_stats* stats_out);

/* Adjoint of one SNP block (requires GLS_KEEP_FOR_GRAD at setup).
 * Given cotangents b_bar (p x mb, ld p), sigma2_bar (mb), v_bar (mb) of the
 * block's outputs, recomputes X~_R,b and accumulates into the handle the
 * adjoints of L, y~, S_TL, r~_T and y~^T y~.  If XR_grad is not NULL it
 * receives dL/dX_R,b (n x mb, ld_xr).  Asynchronous on `stream`. */
gls_status gls_backward_block(gls_handle h, int32_t mb, const double* XR, int64_t ld_xr,
                              const double* b_bar, const double* sigma2_bar,
                              const double* v_bar, double* XR_grad, void* stream);

/* Finishes the adjoint after all blocks: y_grad (n, may be NULL) and h2_grad
 * (one double on the device, may be NULL), through y~ = L^-1 y, the Cholesky
 * factorization and M = h2 Phi + (1 - h2) I.  Resets the accumulators.
 * Asynchronous on `stream`. */
gls_status gls_backward_finish(gls_handle h, double* y_grad, double* h2_grad, void* stream);

/* Adjoint of a streamed study (the buffering of Sec. 3.1 applied to the
 * adjoint of the per-SNP solve of Sec. 2.1; requires GLS_KEEP_FOR_GRAD).
 * For SNPs [col0, m) of XR_host (n x m FP64, ld_xr >= n, page-locked host
 * memory, the layout of gls_stream) runs gls_backward_block on each block in
 * gls_stream's block schedule: block b+1 is copied into one of two device
 * buffers on the copy stream while block b's adjoint (which recomputes
 * X~_R,b from its copy) runs on the compute stream.  b_bar_host (p x m,
 * ld p), sigma2_bar_host and v_bar_host (m) are the cotangents of the
 * study's outputs, in host memory; each block's are copied up on the compute
 * stream just before its adjoint.  If XR_grad_host is not NULL it receives
 * dL/dX_R (n x m, ld_xr) in host memory, each block's copied down on the
 * compute stream right after its adjoint (that copy is not overlapped).
 * The handle's adjoint accumulators add up over calls (col0 > 0 resumes; a
 * study may also be passed several times); gls_backward_finish then gives
 * the y and h2 gradients.  With every block but the last a multiple of 16
 * SNPs wide, the gradients are bitwise those of gls_backward_block over
 * blocks of any such width.  Streams as for gls_stream.  Returns after every
 * copy has landed; col0 == m returns GLS_OK at once.  Errors: GLS_ERR_STATE
 * without GLS_KEEP_FOR_GRAD; GLS_ERR_ARG for col0 outside [0, m], a NULL SNP
 * matrix or cotangent, or ld_xr < n. */
gls_status gls_stream_backward(gls_handle h, int64_t m, int64_t col0,
                               const double* XR_host, int64_t ld_xr,
                               const double* b_bar_host, const double* sigma2_bar_host,
                               const double* v_bar_host, double* XR_grad_host,
                               void* compute_stream, void* copy_stream,
                               gls_stream_stats* stats_out);

/* gls_stream_backward for a SNP matrix read from storage (both buffering
 * levels of Sec. 3.1): the file, offset, elem_bits (64 FP64, 8 genotype
 * bytes, 2 packed 2-bit dosages), block schedule, reader thread, host_ws
 * (page-locked, gls_stream_file_host_bytes(h, elem_bits) bytes) and streams
 * are those of gls_stream_file.  Byte and packed columns are widened to FP64
 * on the device before each block's adjoint.  Cotangents as in
 * gls_stream_backward; XR_grad_host, if not NULL, receives dL/dX_R as n x m
 * FP64 (ld n) in host memory.  Requires GLS_KEEP_FOR_GRAD (else
 * GLS_ERR_STATE); read errors and argument errors as for gls_stream_file. */
gls_status gls_stream_backward_file(gls_handle h, const char* path, int64_t offset, int32_t elem_bits,
                                    int64_t m, int64_t col0, void* host_ws, size_t host_ws_bytes,
                                    const double* b_bar_host, const double* sigma2_bar_host,
                                    const double* v_bar_host, double* XR_grad_host,
                                    void* compute_stream, void* copy_stream,
                                    gls_stream_stats* stats_out);

/* Per-phase device time of the block path, measured with HIP events recorded
 * around each phase's kernels on the caller's stream while profiling is on.
 *   phase 0: triangular product X~_R,b = L^-1 X_R,b (plain, or the
 *            low-precision bulk and corrections of the mixed forms)
 *   phase 1: FP64 refinement residuals X_R,b - L X~_R,b (mixed forms)
 *   phase 2: per-SNP products and p x p solves
 *   phase 3: adjoint block work                                             */
#define GLS_NUM_PHASES 4
typedef struct {
  int64_t launches[GLS_NUM_PHASES]; /* timed phase instances                 */
  double ms[GLS_NUM_PHASES];        /* summed device milliseconds            */
} gls_phase_stats;

/* Turns event timing of the phases on (on != 0) or off.  Off by default. */
gls_status gls_profile_enable(gls_handle h, int32_t on);

/* Waits for the recorded events, adds their times into *out (zeroed first),
 * and, if reset != 0, forgets them.  Host-synchronous on those events. */
gls_status gls_profile_read(gls_handle h, gls_phase_stats* out, int32_t reset);

/* Releases the handle (not the workspace).  NULL is allowed. */
void gls_destroy(gls_handle h);

/* For callers that cannot allocate device memory or create HIP objects
 * (serving loops and harnesses that forbid hipMalloc): gls_setup followed by
 * gls_block over m SNPs, with no workspace argument and no handle.
 * The workspace is a static device array of GLS_NOALLOC_SCRATCH_BYTES that
 * each GPU the library runs on holds until the process ends; its device
 * address is looked up once per device, on the first call with that device
 * current.  The call allocates no device or host memory and creates no
 * stream or event; the setup runs entirely on `stream`.
 * Arguments: as gls_setup (Phi, XL, y, h2, opts, info) and gls_block (XR is
 *   n x m with ld_xr >= n; b is p x m with ld_b >= p; sigma2, v, snp_status
 *   have m entries), walked in blocks of opts->block_cols SNPs.
 *   opts->flags must be 0 (no adjoint, no streaming).
 * Limit: gls_workspace_bytes(n, p, opts) <= GLS_NOALLOC_SCRATCH_BYTES, else
 *   GLS_ERR_WORKSPACE (plain FP64, p = 4: n up to 1,536 with block_cols = 256,
 *   up to about 1,000 with block_cols = 1,024).
 * Results are bitwise those of gls_setup + gls_block with the same opts.
 * Synchronizes `stream` before returning (outputs written, scratch free).
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (each call rewrites what it reads): calls that overlap on one GPU,
 * for instance from two host threads, race and must not be made. */
#define GLS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
gls_status gls_solve_noalloc(int64_t n, int32_t p, const double* Phi, int64_t ld_phi, double h2,
                             const double* XL, int64_t ld_xl, const double* y,
                             int64_t m, const double* XR, int64_t ld_xr,
                             double* b, int64_t ld_b, double* sigma2, double* v, int32_t* snp_status,
                             const gls_opts* opts, void* stream, int64_t* info);

const char* gls_status_string(gls_status s);
const char* gls_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GLS_H */
