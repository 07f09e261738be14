// libgls: C-ABI entry points, workspace planning and the host-side drivers
// of the streamed GWAS GLS solver (paper Sec. 2-3), for gfx950.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "gemm_f64.hpp"
#include "gemm_f64_dma.hpp"
#include "gls.h"
#include "adjoint_kernels.hpp"
#include "gls_internal.hpp"
#include "lp_gemm.hpp"
#include "ozaki_i8.hpp"
#include "setup_kernels.hpp"
#include "snp_kernels.hpp"

using namespace gls;

namespace {

thread_local char g_err[512] = "";

void set_err(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

}  // namespace

namespace gls {

gls_status hip_fail(hipError_t e, const char* what) {
  set_err("%s: %s", what, hipGetErrorString(e));
  return GLS_ERR_HIP;
}

gls_status arg_fail(const char* what) {
  set_err("%s", what);
  return GLS_ERR_ARG;
}

void set_last_error_str(const char* what) { set_err("%s", what); }

static size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int64_t padded_n(int64_t n) { return (n + NPAD - 1) / NPAD * NPAD; }

// Launch shapes below take N / tile rows without a remainder.
static_assert(NPAD % NB_LEAF == 0 && NPAD % LP_BM == 0 && NPAD % OZ_BM == 0 && NPAD % DB_BM == 0 && NPAD % 64 == 0,
              "the row padding must be a multiple of every row tile");

// Largest T1 buffer of the recursive factorization: (b - mid) * (mid - a) leaves.
static int64_t recursion_temp_leaves(int a, int b) {
  if (b - a <= 1) return 0;
  int mid = (a + b) / 2;
  int64_t here = (int64_t)(b - mid) * (mid - a);
  return std::max(here, std::max(recursion_temp_leaves(a, mid), recursion_temp_leaves(mid, b)));
}

// Setup products of at least this many output elements use the XCD-aware
// mapping; a node whose panel is this big forms its panel products on the
// direct-load kernel and runs its T = L21 L11^-1 on the side stream.
static bool big_product(int64_t rows, int64_t cols) { return rows * cols >= (int64_t)1024 * 1024; }

// Per recursion depth, the largest (b - mid) x (mid - a) leaf product of a
// node whose T runs on the side stream.
static void side_temp_leaves(int a, int b, int depth, int64_t* most) {
  if (b - a <= 1 || depth >= 16) return;
  const int mid = (a + b) / 2;
  const int64_t here = (int64_t)(b - mid) * (mid - a);
  if (big_product((int64_t)(b - mid) * NB_LEAF, (int64_t)(mid - a) * NB_LEAF)) most[depth] = std::max(most[depth], here);
  side_temp_leaves(a, mid, depth + 1, most);
  side_temp_leaves(mid, b, depth + 1, most);
}

bool plan_workspace(int64_t n, int32_t p, const gls_opts* o, Plan* pl) {
  if (n < 2 || p < 1 || p > PMAX || n <= p || !o || o->block_cols < 1) return false;
  if (o->precision < GLS_FP64 || o->precision > GLS_INT8_EMU) return false;
  if (o->refine_sweeps < 0 || o->refine_sweeps > 4) return false;
  if (n > (int64_t)1 << 20) return false;
  const int64_t N = padded_n(n);
  const int64_t bc = o->block_cols;
  const int Kt = (int)((n + NB_LEAF - 1) / NB_LEAF);   // rows past n are the identity: factored only up to a leaf
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes, 256);
    return at;
  };
  pl->n = n;
  pl->p = p;
  pl->N = N;
  pl->bc = bc;
  pl->leaves = Kt;
  pl->off_info = take(256);
  pl->off_small = take(sizeof(double) * 2048);
  pl->off_gram = take(sizeof(double) * PMAX * PMAX);
  pl->off_L = take(sizeof(double) * N * N);
  pl->off_Linv = take(sizeof(double) * N * N);
  pl->off_W = take(sizeof(double) * N * p);
  // the panel of a recursion node and, for big nodes, its transpose
  // the whitened block (N x bc, padded to a multiple of 64 SNPs for the adjoint's zero SNPs), the setup's panels
  int64_t tmp = std::max<int64_t>(N * ((bc + 63) / 64 * 64), 2 * recursion_temp_leaves(0, Kt) * NB_LEAF * NB_LEAF);
  tmp = std::max<int64_t>(tmp, N * p * (1 + (N + TA_KC - 1) / TA_KC));   // [X_L | y] and its split-k partials
  pl->off_Xt = take(sizeof(double) * tmp);
  {
    int64_t most[16] = {0}, at = 0;
    side_temp_leaves(0, Kt, 0, most);
    for (int d = 0; d < 16; ++d) {
      pl->side_at[d] = at;
      at += most[d] * NB_LEAF * NB_LEAF;
    }
    pl->off_side = take(sizeof(double) * std::max<int64_t>(at, 1));
  }
  pl->off_buf0 = take(sizeof(double) * n * bc);
  pl->off_buf1 = take(sizeof(double) * n * bc);
  pl->off_ob = take(sizeof(double) * p * bc);
  pl->off_os2 = take(sizeof(double) * bc);
  pl->off_ov = take(sizeof(double) * bc);
  pl->off_ost = take(sizeof(int32_t) * bc);
  pl->bcp = (bc + 63) / 64 * 64;
  pl->lp_bytes = o->precision == GLS_FP32_IR ? 4
                 : (o->precision == GLS_FP16_IR || o->precision == GLS_BF16_IR) ? 2 : 0;
  pl->off_ub0 = take((size_t)n * bc);
  pl->off_ub1 = take((size_t)n * bc);
  if (o->precision == GLS_INT8_EMU) {
    pl->off_ubp = take((size_t)N * pl->bcp);
    pl->off_sl = take((size_t)OZ_SLICES * N * N);
    pl->off_ex = take(sizeof(int) * N);
  }
  pl->off_x64 = take(sizeof(double) * N * bc);
  if (pl->lp_bytes) {
    pl->off_Llp = take((size_t)pl->lp_bytes * N * N);
    pl->off_Blp = take((size_t)pl->lp_bytes * N * pl->bcp);
    pl->off_R = take(sizeof(double) * N * pl->bcp);
    pl->off_cs = take(sizeof(double) * pl->bcp);
    pl->off_red = take(sizeof(double) * 2048);
  }
  if (o->flags & GLS_KEEP_FOR_GRAD) {
    const int64_t nc = adj_nc(p);
    pl->off_Phi = take(sizeof(double) * N * N);
    pl->off_Lbar = take(sizeof(double) * N * N);
    pl->off_T1 = take(sizeof(double) * N * N);
    pl->off_T2 = take(sizeof(double) * N * N);
    pl->off_Xtb = take(sizeof(double) * N * pl->bcp);
    pl->off_Xb = take(sizeof(double) * N * pl->bcp);
    pl->off_Cb = take(sizeof(double) * p * pl->bcp);
    pl->off_eb = take(sizeof(double) * pl->bcp);
    pl->off_ct = take(sizeof(double) * nc * pl->bcp);
    pl->off_Wb = take(sizeof(double) * N * p);
    pl->off_W0b = take(sizeof(double) * N * p);
    pl->off_acc = take(sizeof(double) * (nc + 2048));
  }
  pl->total = off;
  return true;
}

}  // namespace gls

// ---------------------------------------------------------------------------
// GEMM launch helpers

namespace gls {

// One tile configuration for every product: 64 x 64 tiles, 16-deep LDS
// slices, four waves each owning a 64 x 16 strip, v_mfma_f64_4x4x4_4b_f64
// (58 TFLOP/s measured on the n = 10,000 per-block product).
constexpr int GBM = 64, GBN = 64, GBK = 16, GWM = 1, GWN = 4;

template <bool TA, bool TB, int MAP, bool VEC>
static void launch_gemm_cfg(GemmArgs g, hipStream_t s) {
  const int Mt = (g.M + GBM - 1) / GBM;
  g.M = Mt * GBM;
  const int Nt = (g.ncols + GBN - 1) / GBN;
  if (Mt == 0 || Nt == 0) return;
  if (MAP == MAP_XCD) {
    hipLaunchKernelGGL((gemm_f64_kernel<GBM, GBN, GBK, GWM, GWN, TA, TB, MAP_XCD, VEC, true>),
                       dim3(XcdMap::grid(g, Mt, Nt)), dim3(64 * GWM * GWN), 0, s, g);
  } else {
    hipLaunchKernelGGL((gemm_f64_kernel<GBM, GBN, GBK, GWM, GWN, TA, TB, MAP_GRID, VEC, true>), dim3(Nt, Mt),
                       dim3(64 * GWM * GWN), 0, s, g);
  }
}

template <int MAP, bool VEC>
static void gemm_map(bool ta, bool tb, const GemmArgs& g, hipStream_t s) {
  if (!ta && !tb) launch_gemm_cfg<false, false, MAP, VEC>(g, s);
  else if (ta && !tb) launch_gemm_cfg<true, false, MAP, VEC>(g, s);
  else if (!ta && tb) launch_gemm_cfg<false, true, MAP, VEC>(g, s);
  else launch_gemm_cfg<true, true, MAP, VEC>(g, s);
}

// The direct-load kernel for a product it takes (false: not launched).
static bool gemm_dma(const GemmArgs& g, hipStream_t s) {
  if (!trmm_dma_ok(g)) return false;
  GemmArgs d = g;
  const int Mt = (g.M + DB_BM - 1) / DB_BM, Nt = (g.ncols + DB_BN - 1) / DB_BN;
  d.M = Mt * DB_BM;   // rows past mvalid are computed from A's padding and not stored
  hipLaunchKernelGGL(trmm_f64_dma_kernel, dim3(XcdMap::grid(d, Mt, Nt)), dim3(DB_THREADS), 0, s, d);
  return true;
}

void gemm(bool ta, bool tb, bool xcd_map, const GemmArgs& g, hipStream_t s) {
  if (!ta && !tb && xcd_map && g.red_q == 0 && gemm_dma(g, s)) return;
  const bool vec = gemm_vec_ok(g, ta, tb);
  if (xcd_map) {
    if (vec) gemm_map<MAP_XCD, true>(ta, tb, g, s);
    else gemm_map<MAP_XCD, false>(ta, tb, g, s);
  } else {
    if (vec) gemm_map<MAP_GRID, true>(ta, tb, g, s);
    else gemm_map<MAP_GRID, false>(ta, tb, g, s);
  }
}

GemmArgs gemm_args(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, int M,
                   int ncols, int K, double alpha) {
  GemmArgs g;
  std::memset(&g, 0, sizeof g);
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.C = C;
  g.ldc = ldc;
  g.Cin = C;
  g.ldcin = ldc;
  g.M = M;
  g.mvalid = M;
  g.ncols = ncols;
  g.K = K;
  g.alpha = alpha;
  g.beta = 0.0;
  return g;
}

static int grid_for(int64_t total) {
  int64_t b = (total + 255) / 256;
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 65536);
}

// Recursive blocked Cholesky with the inverse factor built alongside.
// Leaves [a, b) count NB_LEAF-row diagonal blocks of the N x N matrices.
//   chol([A11 .; A21 A22]):  L11 = chol(A11), L11^-1 (leaf: in LDS)
//                            L21 = A21 L11^-T,  A22 -= L21 L21^T
//                            L22 = chol(A22),   L22^-1
//                            (L^-1)21 = -L22^-1 L21 L11^-1
// Large setup products use the XCD-aware heavy-first mapping; small ones the plain grid.
//
// T = L21 L11^-1 is needed only by the last product of its node, so for big
// nodes it runs on a side stream (forked after L21 is formed, joined before
// that last product) while the main stream factors L22; it then fills the
// compute units that L22's latency-bound small steps leave idle.  Each depth
// has its own T region and join event.
struct SetupSide {
  hipStream_t st = nullptr;   // the caller's side stream (nullptr: none)
  hipEvent_t fork = nullptr;
  hipEvent_t join[16] = {};
  double* base = nullptr;   // side scratch (plan offsets side_at[depth])
  hipError_t err = hipSuccess;   // first failed record or wait
  void check(hipError_t e) {
    if (err == hipSuccess) err = e;
  }
  ~SetupSide() {
    if (st) (void)hipStreamSynchronize(st);
    for (hipEvent_t e : join)
      if (e) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
  }
  hipError_t init(hipStream_t side, double* scratch) {
    st = side;
    base = scratch;
    hipError_t e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    for (int d = 0; d < 16 && e == hipSuccess; ++d) e = hipEventCreateWithFlags(&join[d], hipEventDisableTiming);
    return e;
  }
};

static void chol_inv_rec(Ctx* c, int a, int b, int depth, SetupSide* side, hipStream_t s) {
  const int64_t N = c->N;
  double* L = c->L;
  double* Li = c->Linv;
  if (b - a == 1) {
    const int64_t r = (int64_t)a * NB_LEAF;
    hipLaunchKernelGGL(leaf_potrf_trtri_kernel, dim3(1), dim3(512), 0, s, L + r + r * N, Li + r + r * N, N, (int)r,
                       c->info);
    return;
  }
  const int mid = (a + b) / 2;
  chol_inv_rec(c, a, mid, depth + 1, side, s);
  const int64_t r1 = (int64_t)a * NB_LEAF, r2 = (int64_t)mid * NB_LEAF;
  const int w1 = (mid - a) * NB_LEAF, w2 = (b - mid) * NB_LEAF;
  double* A21 = L + r2 + r1 * N;
  double* A22 = L + r2 + r2 * N;
  const double* Li11 = Li + r1 + r1 * N;
  double* Li21 = Li + r2 + r1 * N;
  const double* Li22 = Li + r2 + r2 * N;
  double* T = c->Xt;  // w2 x w1, ld w2
  if (big_product(w2, w1)) {
    // Both products without transposed operands, so they run on the direct-load kernel:
    //   U = L21^T = L11^-1 A21^T (U, A21^T: w1 x w2, ld w1), L21 = U^T, A22 -= L21 U.
    double* At = c->Xt;
    double* U = c->Xt + (int64_t)w1 * w2;
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((w2 + 31) / 32), (unsigned)((w1 + 31) / 32)), dim3(256), 0, s,
                       At, (int64_t)w1, A21, N, w2, w1);
    {
      GemmArgs g = gemm_args(Li11, N, At, w1, U, w1, w1, w2, w1, 1.0);
      g.a_tri = TRI_LOWER;
      g.a_diag = 0;
      g.map_desc = 1;
      gemm(false, false, true, g, s);
    }
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((w1 + 31) / 32), (unsigned)((w2 + 31) / 32)), dim3(256), 0, s,
                       A21, N, U, (int64_t)w1, w1, w2);
    {  // lower tiles; high row tiles hold the most of them
      GemmArgs g = gemm_args(A21, N, U, w1, A22, N, w2, w2, w1, -1.0);
      g.beta = 1.0;
      g.c_lower = 1;
      g.c_diag = 0;
      g.map_desc = 1;
      gemm(false, false, true, g, s);
    }
  } else {
    hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for((int64_t)w2 * w1)), dim3(256), 0, s, T, (int64_t)w2, A21, N, w2,
                       w1);
    {  // L21 = T * L11^-T   (op(B)[k][j] = Li11[j][k], non-zero for k <= j: upper)
      GemmArgs g = gemm_args(T, w2, Li11, N, A21, N, w2, w1, w1, 1.0);
      g.b_tri = TRI_UPPER;
      g.b_diag = 0;
      gemm(false, true, false, g, s);
    }
    {  // A22 -= L21 L21^T  (lower tiles)
      GemmArgs g = gemm_args(A21, N, A21, N, A22, N, w2, w2, w1, -1.0);
      g.beta = 1.0;
      g.c_lower = 1;
      g.c_diag = 0;
      g.map_desc = 1;
      gemm(false, true, big_product(w2, w2), g, s);
    }
  }
  const bool on_side = big_product(w2, w1) && depth < 16 && side->st != nullptr;
  if (on_side) {   // T = L21 L11^-1 on the side stream, into this depth's region
    T = side->base + c->plan.side_at[depth];
    side->check(hipEventRecord(side->fork, s));
    side->check(hipStreamWaitEvent(side->st, side->fork, 0));
    GemmArgs g = gemm_args(A21, N, Li11, N, T, w2, w2, w1, w1, 1.0);
    g.b_tri = TRI_LOWER;
    g.b_diag = 0;
    gemm(false, false, true, g, side->st);
    side->check(hipEventRecord(side->join[depth], side->st));
  }
  chol_inv_rec(c, mid, b, depth + 1, side, s);
  if (on_side) {
    side->check(hipStreamWaitEvent(s, side->join[depth], 0));
  } else {  // T = L21 L11^-1   (op(B) = Li11 lower: non-zero for k >= j)
    GemmArgs g = gemm_args(A21, N, Li11, N, T, w2, w2, w1, w1, 1.0);
    g.b_tri = TRI_LOWER;
    g.b_diag = 0;
    gemm(false, false, big_product(w2, w1), g, s);
  }
  {  // (L^-1)21 = -L22^-1 T   (op(A) = Li22 lower: non-zero for k <= i)
    GemmArgs g = gemm_args(Li22, N, T, w2, Li21, N, w2, w1, w2, -1.0);
    g.a_tri = TRI_LOWER;
    g.a_diag = 0;
    g.map_desc = 1;
    gemm(false, false, big_product(w2, w1), g, s);
  }
}

template <int P>
static void tri_apply_p(Ctx* c, const double* V, double* part, double* W, hipStream_t s) {
  const int N = (int)c->N;
  hipLaunchKernelGGL(tri_apply_partial_kernel<P>, dim3(N / 64, (N + TA_KC - 1) / TA_KC), dim3(256), 0, s, c->Linv, N,
                     V, part);
  hipLaunchKernelGGL(tri_apply_sum_kernel, dim3(grid_for((int64_t)N * P)), dim3(256), 0, s, part, N, P, W);
}

// W (N x p) = L^-1 V for the covariate block V (N x p, ld N); part holds
// ceil(N / TA_KC) partial N x p blocks.
static void tri_apply(Ctx* c, const double* V, double* part, double* W, hipStream_t s) {
  switch (c->p) {
#define GLS_P_CASE(P) \
  case P: tri_apply_p<P>(c, V, part, W, s); break;
    GLS_P_CASE(1) GLS_P_CASE(2) GLS_P_CASE(3) GLS_P_CASE(4) GLS_P_CASE(5) GLS_P_CASE(6) GLS_P_CASE(7)
    GLS_P_CASE(8) GLS_P_CASE(9) GLS_P_CASE(10) GLS_P_CASE(11) GLS_P_CASE(12) GLS_P_CASE(13) GLS_P_CASE(14)
    GLS_P_CASE(15) GLS_P_CASE(16) GLS_P_CASE(17) GLS_P_CASE(18) GLS_P_CASE(19) GLS_P_CASE(20)
#undef GLS_P_CASE
    default: break;
  }
}

// X~ (rows x mb, ld N) = L^-1 X   for an n x mb block X (ld ldx) summed over
// its first K rows: K = n, or n rounded up to 16 when X's rows n..K-1 are
// zero.  rows = N, or n rounded up to the product's 128-row tiles when only
// the sample rows (and the zero rows up to that tile edge) are read later.
void whiten_fp64(Ctx* c, const double* X, int64_t ldx, int mb, int K, int rows, double* Xt, hipStream_t s) {
  GemmArgs g = gemm_args(c->Linv, c->N, X, ldx, Xt, c->N, rows, mb, K, 1.0);
  g.a_tri = TRI_LOWER;
  g.a_diag = 0;
  g.map_desc = 1;
  gemm(false, false, true, g, s);
}

// The same product with the per-SNP sums fused into its epilogue: instead of
// X~, c->Xt receives for each 128-row tile t and SNP j the sums of x~ times
// [X~_L | y~] and of x~^2 over the tile's rows ((t (p + 1) + q) mb + j).
// Returns false, launching nothing, when the direct-load kernel does not
// take the shape.
static bool whiten_fp64_fused(Ctx* c, const double* X, int64_t ldx, int mb, int K, int rows, hipStream_t s) {
  GemmArgs g = gemm_args(c->Linv, c->N, X, ldx, c->Xt, c->N, rows, mb, K, 1.0);
  g.a_tri = TRI_LOWER;
  g.a_diag = 0;
  g.map_desc = 1;
  g.red_W = c->W;
  g.ld_red_W = c->N;
  g.red_part = c->Xt;
  g.red_q = c->p + 1;
  return gemm_dma(g, s);
}

template <int P>
static void launch_snp_partials_p(Ctx* c, int Mt, int mb, double* b, int64_t ldb, double* s2, double* v, int* st,
                                  hipStream_t s) {
  hipLaunchKernelGGL(snp_partials_solve_kernel<P>, dim3((mb + 255) / 256), dim3(256), 0, s, c->Xt, Mt, mb, c->small,
                     (int)c->n, b, ldb, s2, v, st);
}

static void snp_partials_solve(Ctx* c, int Mt, int mb, double* b, int64_t ldb, double* s2, double* v, int* st,
                               hipStream_t s) {
  switch (c->p) {
#define GLS_P_CASE(P) \
  case P: launch_snp_partials_p<P>(c, Mt, mb, b, ldb, s2, v, st, s); break;
    GLS_P_CASE(1) GLS_P_CASE(2) GLS_P_CASE(3) GLS_P_CASE(4) GLS_P_CASE(5) GLS_P_CASE(6) GLS_P_CASE(7)
    GLS_P_CASE(8) GLS_P_CASE(9) GLS_P_CASE(10) GLS_P_CASE(11) GLS_P_CASE(12) GLS_P_CASE(13) GLS_P_CASE(14)
    GLS_P_CASE(15) GLS_P_CASE(16) GLS_P_CASE(17) GLS_P_CASE(18) GLS_P_CASE(19) GLS_P_CASE(20)
#undef GLS_P_CASE
    default: break;
  }
}

template <int P>
static void launch_snp_p(Ctx* c, const double* Xt, int mb, double* b, int64_t ldb, double* s2, double* v, int* st,
                         hipStream_t s) {
  const int grid = (mb + SNP_PER_WG - 1) / SNP_PER_WG;
  hipLaunchKernelGGL(snp_reduce_solve_kernel<P>, dim3(grid), dim3(64 * SNP_WAVES), 0, s, Xt, (int64_t)c->N, (int)c->N,
                     mb, c->W, c->small, (int)c->n, b, ldb, s2, v, st);
}

void snp_reduce_solve(Ctx* c, const double* Xt, int mb, double* b, int64_t ldb, double* s2, double* v, int* st,
                      hipStream_t s) {
  switch (c->p) {
#define GLS_P_CASE(P) \
  case P: launch_snp_p<P>(c, Xt, mb, b, ldb, s2, v, st, s); break;
    GLS_P_CASE(1) GLS_P_CASE(2) GLS_P_CASE(3) GLS_P_CASE(4) GLS_P_CASE(5) GLS_P_CASE(6) GLS_P_CASE(7)
    GLS_P_CASE(8) GLS_P_CASE(9) GLS_P_CASE(10) GLS_P_CASE(11) GLS_P_CASE(12) GLS_P_CASE(13) GLS_P_CASE(14)
    GLS_P_CASE(15) GLS_P_CASE(16) GLS_P_CASE(17) GLS_P_CASE(18) GLS_P_CASE(19) GLS_P_CASE(20)
#undef GLS_P_CASE
    default: break;
  }
}

}  // namespace gls

// ---------------------------------------------------------------------------
// C-ABI

namespace gls {

// Workspace of gls_solve_noalloc: a file-scope array that each device holds
// from the library's first use on it until the process ends.  Host code must
// not pass `scratch` itself to a kernel (in host code the name is a host-side
// stand-in); it uses the device address that noalloc_workspace() looked up.
static __device__ __align__(256) char scratch[GLS_NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static void* g_scratch_at[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

// Device address of the current device's scratch array, looked up once per
// device with that device current.
static gls_status noalloc_workspace(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "gls_solve_noalloc: hipGetDevice");
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return arg_fail("gls_solve_noalloc: device index above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* at = nullptr;
    e = hipGetSymbolAddress(&at, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "gls_solve_noalloc: hipGetSymbolAddress");
    if (!at) return hip_fail(hipErrorInvalidSymbol, "gls_solve_noalloc: hipGetSymbolAddress");
    g_scratch_at[dev] = at;
  }
  *out = static_cast<char*>(g_scratch_at[dev]);
  return GLS_OK;
}

// Argument checks shared by gls_setup and gls_solve_noalloc; fills the plan.
static gls_status setup_args(const char* fn, int64_t n, int32_t p, const double* Phi, int64_t ld_phi, double h2,
                             const double* XL, int64_t ld_xl, const double* y, const gls_opts* opts, Plan* pl) {
  if (!plan_workspace(n, p, opts, pl)) {
    set_err("%s: invalid n/p/opts (need 1 <= p <= 20, n > p)", fn);
    return GLS_ERR_ARG;
  }
  const char* bad = nullptr;
  if (!Phi || ld_phi < n) bad = "Phi is NULL or ld_phi < n";
  else if (p > 1 && (!XL || ld_xl < n)) bad = "XL is NULL or ld_xl < n";
  else if (!y) bad = "y is NULL";
  else if (!(h2 >= 0.0 && h2 <= 1.0)) bad = "h2 must lie in [0, 1]";
  if (bad) {
    set_err("%s: %s", fn, bad);
    return GLS_ERR_ARG;
  }
  return GLS_OK;
}

// The study setup (Sec. 2.1, Listing 1 before the SNP loop) into a fresh
// handle c whose regions lie in the workspace ws (plan pl).  With a side
// stream the factorization's off-path products overlap there (chol_inv_rec);
// without one every kernel runs on s (the same kernels in the same order per
// output, so the same results).  Synchronizes s, into which the side stream is
// joined: on return nothing enqueued here still runs.
static gls_status setup_into(Ctx* c, const Plan& pl, int64_t n, int32_t p, const double* Phi, int64_t ld_phi,
                             double h2, const double* XL, int64_t ld_xl, const double* y, char* ws,
                             const gls_opts* opts, hipStream_t side_st, hipStream_t s, int64_t* info) {
  c->plan = pl;
  c->opts = *opts;
  c->n = n;
  c->p = p;
  c->N = pl.N;
  c->bc = pl.bc;
  c->h2 = h2;
  c->info = reinterpret_cast<int*>(ws + pl.off_info);
  c->small = reinterpret_cast<double*>(ws + pl.off_small);
  c->gram = reinterpret_cast<double*>(ws + pl.off_gram);
  c->L = reinterpret_cast<double*>(ws + pl.off_L);
  c->Linv = reinterpret_cast<double*>(ws + pl.off_Linv);
  c->W = reinterpret_cast<double*>(ws + pl.off_W);
  c->Xt = reinterpret_cast<double*>(ws + pl.off_Xt);
  c->buf[0] = reinterpret_cast<double*>(ws + pl.off_buf0);
  c->buf[1] = reinterpret_cast<double*>(ws + pl.off_buf1);
  c->ob = reinterpret_cast<double*>(ws + pl.off_ob);
  c->os2 = reinterpret_cast<double*>(ws + pl.off_os2);
  c->ov = reinterpret_cast<double*>(ws + pl.off_ov);
  c->ost = reinterpret_cast<int*>(ws + pl.off_ost);
  const int64_t N = c->N;

  hipError_t e;
  int hinfo[2] = {0, 0};
  auto fail = [&](gls_status st) {   // nothing enqueued here may still run on the caller's workspace
    (void)hipStreamSynchronize(s);
    return st;
  };
  // info[0]: failing pivot of M, info[1]: failing pivot of S_TL
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<double*>(c->info), (int64_t)4, 0.0);
  hipLaunchKernelGGL(form_m_kernel, dim3(grid_for(N * N)), dim3(256), 0, s, c->L, (int)N, (int)n, Phi, ld_phi, h2);
  // L^-1 = 0 but for the identity on rows past the factored leaves
  hipLaunchKernelGGL(identity_tail_kernel, dim3(grid_for(N * N)), dim3(256), 0, s, c->Linv, (int)N,
                     pl.leaves * NB_LEAF);
  {
    SetupSide side;
    if (side_st && (e = side.init(side_st, reinterpret_cast<double*>(ws + pl.off_side))) != hipSuccess)
      return fail(hip_fail(e, "gls_setup: side stream events"));
    chol_inv_rec(c, 0, pl.leaves, 0, &side, s);
    // every side product is joined into s by its node's last product
    if (side.err != hipSuccess) return fail(hip_fail(side.err, "gls_setup: side stream fork/join"));
  }
  c->ub[0] = reinterpret_cast<uint8_t*>(ws + pl.off_ub0);
  c->ub[1] = reinterpret_cast<uint8_t*>(ws + pl.off_ub1);
  if (opts->precision == GLS_INT8_EMU) {
    c->ubp = reinterpret_cast<uint8_t*>(ws + pl.off_ubp);
    c->sl = reinterpret_cast<int8_t*>(ws + pl.off_sl);
    c->ex = reinterpret_cast<int*>(ws + pl.off_ex);
    hipLaunchKernelGGL(row_exponent_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, c->Linv, (int)N, c->ex);
    hipLaunchKernelGGL(slice_factor_kernel, dim3((unsigned)(N / 64), (unsigned)(N / 64)), dim3(256), 0, s, c->Linv,
                       (int)N, (const int*)c->ex, c->sl);
  }
  c->x64 = reinterpret_cast<double*>(ws + pl.off_x64);
  if (pl.lp_bytes) {
    c->Llp = ws + pl.off_Llp;
    c->Blp = ws + pl.off_Blp;
    c->R = reinterpret_cast<double*>(ws + pl.off_R);
    c->cs = reinterpret_cast<double*>(ws + pl.off_cs);
    c->red = reinterpret_cast<double*>(ws + pl.off_red);
    prepare_low_precision(c, s);
  }
  if (opts->flags & GLS_KEEP_FOR_GRAD) {
    c->grad = true;
    c->Phi = reinterpret_cast<double*>(ws + pl.off_Phi);
    c->Lbar = reinterpret_cast<double*>(ws + pl.off_Lbar);
    c->T1 = reinterpret_cast<double*>(ws + pl.off_T1);
    c->T2 = reinterpret_cast<double*>(ws + pl.off_T2);
    c->Xtb = reinterpret_cast<double*>(ws + pl.off_Xtb);
    c->Xb = reinterpret_cast<double*>(ws + pl.off_Xb);
    c->Cb = reinterpret_cast<double*>(ws + pl.off_Cb);
    c->eb = reinterpret_cast<double*>(ws + pl.off_eb);
    c->ct = reinterpret_cast<double*>(ws + pl.off_ct);
    c->Wb = reinterpret_cast<double*>(ws + pl.off_Wb);
    c->W0b = reinterpret_cast<double*>(ws + pl.off_W0b);
    c->acc = reinterpret_cast<double*>(ws + pl.off_acc);
    hipLaunchKernelGGL(keep_phi_kernel, dim3(grid_for(N * N)), dim3(256), 0, s, c->Phi, (int)N, (int)n, Phi, ld_phi);
    reset_adjoint(c, s);
  }
  // [X~_L | y~] = L^-1 [X_L | y]
  double* Wp = c->Xt;
  hipLaunchKernelGGL(pack_covariates_kernel, dim3(grid_for(N * p)), dim3(256), 0, s, Wp, (int)N, (int)n, (int)p, XL,
                     ld_xl, y);
  tri_apply(c, Wp, Wp + N * p, c->W, s);
  hipLaunchKernelGGL(gram_kernel, dim3(p * (p + 1) / 2), dim3(256), 0, s, c->W, (int)N, (int)p, c->gram);
  hipLaunchKernelGGL(small_factor_kernel, dim3(1), dim3(64), 0, s, c->gram, (int)p, c->small, c->info + 1);
  if ((e = hipGetLastError()) != hipSuccess) return fail(hip_fail(e, "gls_setup: launch"));
  if ((e = hipMemcpyAsync(hinfo, c->info, sizeof hinfo, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return fail(hip_fail(e, "gls_setup: info copy"));
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail(hip_fail(e, "gls_setup: synchronize"));
  if (hinfo[0] != 0) {
    if (info) *info = hinfo[0];
    set_err("gls_setup: M is not positive definite (leading minor %d)", hinfo[0]);
    return fail(GLS_ERR_NOT_SPD);
  }
  if (hinfo[1] != 0) {
    if (info) *info = hinfo[1];
    set_err("gls_setup: S_TL = X~_L^T X~_L is not positive definite at covariate %d", hinfo[1]);
    return fail(GLS_ERR_RANK);
  }
  return GLS_OK;
}

// The handle's compute and copy streams.  HIP multiplexes a process's plain
// streams onto a few hardware queues.  On a shared queue a cross-stream wait
// holds up the other stream's work queued behind it, so the copy pipeline
// (copies wait for the solve that last read their buffer, solves for their
// copy) would run copies and solves one after another.  The check: `c` idles
// about 0.4 ms in bounded sleeps, `copy` waits for it, and an empty kernel on
// `comp` must finish while c still runs.  (Kernels of different streams on one
// queue do overlap, so sharing c's queue does not fail the check; a slow host
// can only make its answer a false "shared".)  The copy stream is re-created
// until the check passes, at most four times.
__global__ void idle_kernel(int rounds) {
  for (int r = 0; r < rounds; ++r) __builtin_amdgcn_s_sleep(127);
}
__global__ void empty_kernel() {}

static bool wait_is_isolated(hipStream_t comp, hipStream_t copy, hipStream_t c, hipEvent_t ev) {
  hipLaunchKernelGGL(idle_kernel, dim3(1), dim3(64), 0, c, 100);
  bool ok = hipEventRecord(ev, c) == hipSuccess && hipStreamWaitEvent(copy, ev, 0) == hipSuccess;
  hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, copy);
  hipLaunchKernelGGL(empty_kernel, dim3(1), dim3(64), 0, comp);
  ok = ok && hipGetLastError() == hipSuccess && hipStreamSynchronize(comp) == hipSuccess;
  ok = ok && hipEventQuery(ev) == hipErrorNotReady;
  (void)hipStreamSynchronize(c);
  (void)hipStreamSynchronize(copy);
  (void)hipGetLastError();
  return ok;
}

static hipError_t make_stream_pair(hipStream_t st[2], hipStream_t caller, hipEvent_t ev) {
  hipError_t e = hipStreamCreateWithFlags(&st[0], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&st[1], hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  std::vector<hipStream_t> rejected;
  for (int tries = 0; tries < 4 && !wait_is_isolated(st[0], st[1], caller, ev); ++tries) {
    hipStream_t fresh = nullptr;
    if (hipStreamCreateWithFlags(&fresh, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      break;
    }
    rejected.push_back(st[1]);   // kept until the search ends, so its queue is not handed out again
    st[1] = fresh;
  }
  for (hipStream_t r : rejected) (void)hipStreamDestroy(r);
  return hipSuccess;
}

}  // namespace gls

extern "C" {

const char* gls_status_string(gls_status s) {
  switch (s) {
    case GLS_OK: return "ok";
    case GLS_ERR_ARG: return "invalid argument";
    case GLS_ERR_NOT_SPD: return "M is not positive definite";
    case GLS_ERR_HIP: return "HIP runtime error";
    case GLS_ERR_WORKSPACE: return "workspace too small or misaligned";
    case GLS_ERR_STATE: return "call not valid in this state";
    case GLS_ERR_RANK: return "covariates are rank deficient";
  }
  return "unknown status";
}

const char* gls_last_error(void) { return g_err; }

size_t gls_workspace_bytes(int64_t n, int32_t p, const gls_opts* opts) {
  Plan pl;
  if (!plan_workspace(n, p, opts, &pl)) return 0;
  return pl.total;
}

gls_status gls_setup(gls_handle* out, int64_t n, int32_t p, const double* Phi, int64_t ld_phi, double h2,
                     const double* XL, int64_t ld_xl, const double* y, void* workspace, size_t ws_bytes,
                     const gls_opts* opts, void* stream, int64_t* info) {
  if (info) *info = 0;
  if (!out) return arg_fail("gls_setup: out is NULL");
  *out = nullptr;
  Plan pl;
  gls_status st = setup_args("gls_setup", n, p, Phi, ld_phi, h2, XL, ld_xl, y, opts, &pl);
  if (st != GLS_OK) return st;
  if (!workspace || ((uintptr_t)workspace & 255)) {
    set_err("gls_setup: workspace is NULL or not 256-byte aligned");
    return GLS_ERR_WORKSPACE;
  }
  if (ws_bytes < pl.total) {
    set_err("gls_setup: workspace has %zu bytes, needs %zu", ws_bytes, pl.total);
    return GLS_ERR_WORKSPACE;
  }
  Ctx* c = new (std::nothrow) Ctx();
  if (!c) return arg_fail("gls_setup: out of host memory");
  hipError_t e;
  for (int i = 0; i < 2; ++i) {
    if ((e = hipEventCreateWithFlags(&c->ev_copy[i], hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_comp[i], hipEventDisableTiming)) != hipSuccess) {
      gls_destroy(c);
      return hip_fail(e, "gls_setup: event create");
    }
  }
  if ((e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming)) != hipSuccess) {
    gls_destroy(c);
    return hip_fail(e, "gls_setup: event create");
  }
  hipStream_t side = nullptr;   // the factorization's side products
  if ((e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking)) != hipSuccess) {
    gls_destroy(c);
    return hip_fail(e, "gls_setup: side stream create");
  }
  st = setup_into(c, pl, n, p, Phi, ld_phi, h2, XL, ld_xl, y, static_cast<char*>(workspace), opts, side,
                  static_cast<hipStream_t>(stream), info);
  (void)hipStreamDestroy(side);   // joined into `stream`, which setup_into synchronized
  if (st != GLS_OK) {
    gls_destroy(c);
    return st;
  }
  if ((e = make_stream_pair(c->own_st, static_cast<hipStream_t>(stream), c->ev_join)) != hipSuccess) {
    gls_destroy(c);
    return hip_fail(e, "gls_setup: stream create");
  }
  c->ready = true;
  *out = c;
  return GLS_OK;
}

gls_status gls_block(gls_handle h, int32_t mb, const double* XR, int64_t ld_xr, double* b, int64_t ld_b,
                     double* sigma2, double* v, int32_t* snp_status, void* stream) {
  Ctx* c = h;
  if (!c || !c->ready) {
    set_err("gls_block: handle is not set up");
    return GLS_ERR_STATE;
  }
  if (mb < 0 || mb > c->bc) return arg_fail("gls_block: mb must lie in [0, block_cols]");
  if (mb == 0) return GLS_OK;
  if (!XR || ld_xr < c->n) return arg_fail("gls_block: XR is NULL or ld_xr < n");
  if (!b || ld_b < c->p || !sigma2 || !v || !snp_status) return arg_fail("gls_block: NULL output or ld_b < p");
  hipStream_t s = static_cast<hipStream_t>(stream);
  gls_status st = block_forward(c, mb, XR, ld_xr, b, ld_b, sigma2, v, snp_status, s);
  if (st != GLS_OK) return st;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "gls_block: launch");
  return GLS_OK;
}

gls_status gls_profile_enable(gls_handle h, int32_t on) {
  Ctx* c = h;
  if (!c) return arg_fail("gls_profile_enable: NULL handle");
  c->prof_on = on != 0;
  return GLS_OK;
}

gls_status gls_profile_read(gls_handle h, gls_phase_stats* out, int32_t reset) {
  Ctx* c = h;
  if (!c || !out) return arg_fail("gls_profile_read: NULL argument");
  for (const auto& r : c->prof_pending) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return hip_fail(e, "gls_profile_read");
    c->prof_ms[r.phase] += ms;
    c->prof_n[r.phase] += 1;
    c->prof_free.push_back(r.a);
    c->prof_free.push_back(r.b);
  }
  c->prof_pending.clear();
  for (int i = 0; i < GLS_NUM_PHASES; ++i) {
    out->launches[i] = c->prof_n[i];
    out->ms[i] = c->prof_ms[i];
    if (reset) {
      c->prof_n[i] = 0;
      c->prof_ms[i] = 0.0;
    }
  }
  return GLS_OK;
}

gls_status gls_block_u8(gls_handle h, int32_t mb, const uint8_t* G, int64_t ld_g, double* b, int64_t ld_b,
                        double* sigma2, double* v, int32_t* snp_status, void* stream) {
  Ctx* c = h;
  if (!c || !c->ready) {
    set_err("gls_block_u8: handle is not set up");
    return GLS_ERR_STATE;
  }
  if (mb < 0 || mb > c->bc) return arg_fail("gls_block_u8: mb must lie in [0, block_cols]");
  if (mb == 0) return GLS_OK;
  if (!G || ld_g < c->n) return arg_fail("gls_block_u8: G is NULL or ld_g < n");
  if (!b || ld_b < c->p || !sigma2 || !v || !snp_status) return arg_fail("gls_block_u8: NULL output or ld_b < p");
  hipStream_t s = static_cast<hipStream_t>(stream);
  gls_status st = block_forward_u8(c, mb, G, ld_g, b, ld_b, sigma2, v, snp_status, s);
  if (st != GLS_OK) return st;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "gls_block_u8: launch");
  return GLS_OK;
}

gls_status gls_block_u2(gls_handle h, int32_t mb, const uint8_t* G2, int64_t ld_g2, double* b, int64_t ld_b,
                        double* sigma2, double* v, int32_t* snp_status, void* stream) {
  Ctx* c = h;
  if (!c || !c->ready) {
    set_err("gls_block_u2: handle is not set up");
    return GLS_ERR_STATE;
  }
  if (mb < 0 || mb > c->bc) return arg_fail("gls_block_u2: mb must lie in [0, block_cols]");
  if (mb == 0) return GLS_OK;
  if (!G2 || ld_g2 < (c->n + 3) / 4) return arg_fail("gls_block_u2: G2 is NULL or ld_g2 < ceil(n / 4)");
  if (!b || ld_b < c->p || !sigma2 || !v || !snp_status) return arg_fail("gls_block_u2: NULL output or ld_b < p");
  hipStream_t s = static_cast<hipStream_t>(stream);
  gls_status st = block_forward_u2(c, mb, G2, ld_g2, b, ld_b, sigma2, v, snp_status, s);
  if (st != GLS_OK) return st;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "gls_block_u2: launch");
  return GLS_OK;
}

void gls_destroy(gls_handle h) {
  Ctx* c = h;
  if (!c) return;
  for (const auto& r : c->prof_pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : c->prof_free) (void)hipEventDestroy(e);
  for (int i = 0; i < 2; ++i) {
    if (c->own_st[i]) {
      (void)hipStreamSynchronize(c->own_st[i]);
      (void)hipStreamDestroy(c->own_st[i]);
    }
  }
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  for (int i = 0; i < 2; ++i) {
    if (c->ev_copy[i]) (void)hipEventDestroy(c->ev_copy[i]);
    if (c->ev_comp[i]) (void)hipEventDestroy(c->ev_comp[i]);
  }
  delete c;
}

gls_status gls_solve_noalloc(int64_t n, int32_t p, const double* Phi, int64_t ld_phi, double h2, const double* XL,
                             int64_t ld_xl, const double* y, int64_t m, const double* XR, int64_t ld_xr, double* b,
                             int64_t ld_b, double* sigma2, double* v, int32_t* snp_status, const gls_opts* opts,
                             void* stream, int64_t* info) {
  if (info) *info = 0;
  Plan pl;
  gls_status st = setup_args("gls_solve_noalloc", n, p, Phi, ld_phi, h2, XL, ld_xl, y, opts, &pl);
  if (st != GLS_OK) return st;
  if (opts->flags != 0) return arg_fail("gls_solve_noalloc: opts->flags must be 0");
  if (m < 0) return arg_fail("gls_solve_noalloc: m < 0");
  if (m > 0 && (!XR || ld_xr < n)) return arg_fail("gls_solve_noalloc: XR is NULL or ld_xr < n");
  if (m > 0 && (!b || ld_b < p || !sigma2 || !v || !snp_status))
    return arg_fail("gls_solve_noalloc: NULL output or ld_b < p");
  if (pl.total > GLS_NOALLOC_SCRATCH_BYTES) {
    set_err("gls_solve_noalloc: n = %lld, p = %d, block_cols = %d need %zu bytes of workspace, above the %zu of the "
            "static scratch",
            (long long)n, p, opts->block_cols, pl.total, (size_t)GLS_NOALLOC_SCRATCH_BYTES);
    return GLS_ERR_WORKSPACE;
  }
  char* ws = nullptr;
  if ((st = noalloc_workspace(&ws)) != GLS_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Ctx c;   // the handle lives in this frame: no heap, no events, no side stream
  if ((st = setup_into(&c, pl, n, p, Phi, ld_phi, h2, XL, ld_xl, y, ws, opts, nullptr, s, info)) != GLS_OK) return st;
  c.ready = true;
  for (int64_t j0 = 0; j0 < m && st == GLS_OK; j0 += c.bc) {
    const int mb = (int)std::min<int64_t>(c.bc, m - j0);
    st = block_forward(&c, mb, XR + j0 * ld_xr, ld_xr, b + j0 * ld_b, ld_b, sigma2 + j0, v + j0, snp_status + j0, s);
  }
  const hipError_t e = hipGetLastError();
  const hipError_t es = hipStreamSynchronize(s);   // the scratch is free for the next call on return
  if (st != GLS_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "gls_solve_noalloc: launch");
  if (es != hipSuccess) return hip_fail(es, "gls_solve_noalloc: synchronize");
  return GLS_OK;
}

}  // extern "C"

namespace gls {

static hipEvent_t prof_event(Ctx* c) {
  if (!c->prof_free.empty()) {
    hipEvent_t e = c->prof_free.back();
    c->prof_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

PhaseTimer::PhaseTimer(Ctx* c, int phase, hipStream_t s) : c_(c), phase_(phase), s_(s) {
  if (!c_->prof_on) return;
  a_ = prof_event(c_);
  if (a_ && hipEventRecord(a_, s_) != hipSuccess) {
    c_->prof_free.push_back(a_);
    a_ = nullptr;
  }
}

PhaseTimer::~PhaseTimer() {
  if (!a_) return;
  hipEvent_t b = prof_event(c_);
  if (b && hipEventRecord(b, s_) == hipSuccess) {
    c_->prof_pending.push_back({phase_, a_, b});
  } else {
    c_->prof_free.push_back(a_);
    if (b) c_->prof_free.push_back(b);
  }
}

// Power-of-two target magnitude of the low-precision operands (FP16 has a
// narrow exponent range: fill it; FP32 and BF16 need no range adjustment).
static double lp_target(int precision) { return precision == GLS_FP16_IR ? 16384.0 : 1.0; }

// Setup for the mixed forms: the low-precision copy of L^-1 (row-major,
// scaled by a power of two recorded in red[0]) and zero padding rows of R.
void prepare_low_precision(Ctx* c, hipStream_t s) {
  const int64_t N = c->N;
  double* part = c->red + 8;
  hipLaunchKernelGGL(maxabs_kernel, dim3(1024), dim3(256), 0, s, c->Linv, N * N, part);
  hipLaunchKernelGGL(maxabs_kernel, dim3(1), dim3(256), 0, s, part, (int64_t)1024, part + 1024);
  const double tgt = lp_target(c->opts.precision);
  const int g = grid_for(N * N);
  switch (c->opts.precision) {
    case GLS_FP32_IR:
      hipLaunchKernelGGL(convert_factor_kernel<float>, dim3(g), dim3(256), 0, s, c->Linv, (int)N,
                         static_cast<float*>(c->Llp), part + 1024, tgt, c->red);
      break;
    case GLS_FP16_IR:
      hipLaunchKernelGGL(convert_factor_kernel<_Float16>, dim3(g), dim3(256), 0, s, c->Linv, (int)N,
                         static_cast<_Float16*>(c->Llp), part + 1024, tgt, c->red);
      break;
    default:
      hipLaunchKernelGGL(convert_factor_kernel<__bf16>, dim3(g), dim3(256), 0, s, c->Linv, (int)N,
                         static_cast<__bf16*>(c->Llp), part + 1024, tgt, c->red);
      break;
  }
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(N * c->plan.bcp)), dim3(256), 0, s, c->R, N * c->plan.bcp, 0.0);
}

template <typename T>
static void lp_solve_t(Ctx* c, const double* src, int64_t lds, int mb, double beta, hipStream_t s) {
  const int64_t N = c->N;
  T* Blp = static_cast<T*>(c->Blp);
  hipLaunchKernelGGL(scale_convert_kernel<T>, dim3((mb + 3) / 4), dim3(256), 0, s, src, lds, (int)c->n, (int)N, mb,
                     Blp, N, lp_target(c->opts.precision), (const double*)c->red, c->cs);
  LpArgs a;
  std::memset(&a, 0, sizeof a);
  a.A = c->Llp;
  a.lda = N;
  a.B = Blp;
  a.ldb = N;
  a.Cin = c->Xt;
  a.ldcin = N;
  a.C = c->Xt;
  a.ldc = N;
  a.cscale = c->cs;
  a.M = (int)N;
  a.mvalid = (int)N;
  a.ncols = mb;
  a.K = (int)N;
  a.beta = beta;
  // XCD groups of one row tile x 32 column tiles, heavy row tiles first (measured per 8,192-column launch at
  // n = 10,000: FP32 140 TFLOP/s against 101 with 2 x 8 groups and 75 with 4 x 8, FP16 781 against 678; at
  // n = 4,096 FP32 133 against 74; 1 x 8 and 1 x 16 within 8% of 1 x 32)
  a.map_gm = 1;
  a.map_gn = 32;
  a.map_desc = 1;
  const int Mt = (int)(N / LP_BM), Nt = (mb + LP_BN - 1) / LP_BN;
  GemmArgs m{};
  m.map_gm = a.map_gm;
  m.map_gn = a.map_gn;
  hipLaunchKernelGGL(lp_gemm_kernel<T>, dim3(XcdMap::grid(m, Mt, Nt)), dim3(LP_THREADS), 0, s, a);
}

// Xt (N x mb) = L^-1 src in the handle's low precision with FP32 accumulation;
// beta = 1 adds to the current Xt (a refinement correction).
static void lp_solve(Ctx* c, const double* src, int64_t lds, int mb, double beta, hipStream_t s) {
  switch (c->opts.precision) {
    case GLS_FP32_IR: lp_solve_t<float>(c, src, lds, mb, beta, s); break;
    case GLS_FP16_IR: lp_solve_t<_Float16>(c, src, lds, mb, beta, s); break;
    default: lp_solve_t<__bf16>(c, src, lds, mb, beta, s); break;
  }
}

// R (rows < n) = X - L Xt in FP64 (the refinement residual).
// n rounded up to the product kernel's k step; rows n..N-1 of L, L^-1 and of
// every whitened block are zero off the identity padding, so sums may run to it.
static int k16(const Ctx* c) { return (int)((c->n + DB_BK - 1) / DB_BK * DB_BK); }

// The FP64 block operand of the product with L^-1: X itself when its layout
// feeds the direct-load kernel (n a multiple of 16, 16-byte aligned, even
// ld), else a copy in c->x64 (ld N) whose rows n..K-1 are zero.  Blocks
// already in c->x64 (widened bytes) carry zero rows up to N.  Sets *K, the
// rows the product sums over.
static const double* fp64_operand(Ctx* c, const double* X, int64_t* ldx, int mb, int* K, hipStream_t s) {
  if (X == c->x64) {
    *K = k16(c);
    return X;
  }
  *K = (int)c->n;
  if (dma_b_operand_ok(X, *ldx, c->n)) return X;
  *K = k16(c);
  hipLaunchKernelGGL(pad_copy_kernel, dim3(grid_for((int64_t)*K * mb)), dim3(256), 0, s, c->x64, c->N, X, *ldx,
                     (int)c->n, *K, mb);
  *ldx = c->N;
  return c->x64;
}

static void residual_fp64(Ctx* c, const double* X, int64_t ldx, int mb, hipStream_t s) {
  GemmArgs g = gemm_args(c->L, c->N, c->Xt, c->N, c->R, c->N, (int)c->n, mb, k16(c), -1.0);
  g.Cin = X;
  g.ldcin = ldx;
  g.beta = 1.0;
  g.a_tri = TRI_LOWER;
  g.a_diag = 0;
  g.map_desc = 1;
  gemm(false, false, true, g, s);
}

gls_status block_forward(Ctx* c, int mb, const double* XR, int64_t ld_xr, double* b, int64_t ld_b, double* s2,
                         double* v, int* st, hipStream_t s) {
  if (c->plan.lp_bytes) {
    {
      PhaseTimer t(c, PH_WHITEN, s);
      lp_solve(c, XR, ld_xr, mb, 0.0, s);
    }
    for (int sweep = 0; sweep < c->opts.refine_sweeps; ++sweep) {
      {
        PhaseTimer t(c, PH_RESIDUAL, s);
        residual_fp64(c, XR, ld_xr, mb, s);
      }
      PhaseTimer t(c, PH_WHITEN, s);
      lp_solve(c, c->R, c->N, mb, 1.0, s);
    }
  } else {
    // Plain FP64: the per-SNP sums are fused into the product's epilogue, so
    // X~ is neither stored nor read back; row tiles wholly past the last
    // sample are not computed (their rows would only add zeros).
    const int rows = (int)((c->n + DB_BM - 1) / DB_BM * DB_BM);
    bool fused;
    {
      PhaseTimer t(c, PH_WHITEN, s);
      int K = 0;
      const double* X = fp64_operand(c, XR, &ld_xr, mb, &K, s);
      fused = whiten_fp64_fused(c, X, ld_xr, mb, K, rows, s);
      if (!fused) whiten_fp64(c, X, ld_xr, mb, K, rows, c->Xt, s);
    }
    PhaseTimer t(c, PH_SNP, s);
    if (fused) snp_partials_solve(c, rows / DB_BM, mb, b, ld_b, s2, v, st, s);
    else snp_reduce_solve(c, c->Xt, mb, b, ld_b, s2, v, st, s);
    return GLS_OK;
  }
  {
    PhaseTimer t(c, PH_SNP, s);
    snp_reduce_solve(c, c->Xt, mb, b, ld_b, s2, v, st, s);
  }
  return GLS_OK;
}

}  // namespace gls

namespace gls {

// XCD grouping of the int8-slice product's tiles: 4 row tiles x 4 column tiles
// per group (measured best of 1x16 .. 16x1 at n = 10,000, 8,192 SNPs).
constexpr int OZ_MAP_GM = 4, OZ_MAP_GN = 4;

// The product of L^-1 with the block's dosages in c->ubp (N x mb bytes, rows
// >= n zero) on the integer matrix cores, into c->Xt.
static void ozaki_product(Ctx* c, int mb, hipStream_t s) {
  const int64_t N = c->N;
  OzArgs a;
  a.A = c->sl;
  a.ex = c->ex;
  a.B = c->ubp;
  a.C = c->Xt;
  a.ldc = N;
  a.N = (int)N;
  a.ncols = mb;
  a.map_gm = OZ_MAP_GM;
  a.map_gn = OZ_MAP_GN;
  GemmArgs m{};
  m.map_gm = a.map_gm;
  m.map_gn = a.map_gn;
  hipLaunchKernelGGL(ozaki_i8_kernel, dim3(XcdMap::grid(m, (int)(N / OZ_BM), (mb + OZ_BN - 1) / OZ_BN)),
                     dim3(OZ_THREADS), 0, s, a);
}

// Dosage bytes (or packed 2-bit dosages) of a block widened into the zero-padded FP64 buffer x64 (ld N).
void widen_u8(Ctx* c, const uint8_t* G, int64_t ldg, int mb, hipStream_t s) {
  const int64_t N = c->N;
  hipLaunchKernelGGL(u8_to_f64_kernel, dim3(grid_for(N * mb)), dim3(256), 0, s, G, ldg, (int)c->n, (int)N, mb, c->x64);
}
void widen_u2(Ctx* c, const uint8_t* G2, int64_t ldg, int mb, hipStream_t s) {
  const int64_t N = c->N;
  hipLaunchKernelGGL(unpack_u2_f64_kernel, dim3(grid_for(N / 4 * mb)), dim3(256), 0, s, G2, ldg, (int)c->n, (int)N,
                     mb, c->x64);
}

gls_status block_forward_u8(Ctx* c, int mb, const uint8_t* G, int64_t ldg, double* b, int64_t ld_b, double* s2,
                            double* v, int* st, hipStream_t s) {
  const int64_t N = c->N;
  if (c->opts.precision == GLS_INT8_EMU) {
    {
      PhaseTimer t(c, PH_WHITEN, s);
      hipLaunchKernelGGL(pack_u8_kernel, dim3(grid_for(N * mb)), dim3(256), 0, s, G, ldg, (int)c->n, (int)N, mb, c->ubp);
      ozaki_product(c, mb, s);
    }
    PhaseTimer t(c, PH_SNP, s);
    snp_reduce_solve(c, c->Xt, mb, b, ld_b, s2, v, st, s);
    return GLS_OK;
  }
  widen_u8(c, G, ldg, mb, s);
  return block_forward(c, mb, c->x64, N, b, ld_b, s2, v, st, s);
}

gls_status block_forward_u2(Ctx* c, int mb, const uint8_t* G2, int64_t ldg, double* b, int64_t ld_b, double* s2,
                            double* v, int* st, hipStream_t s) {
  const int64_t N = c->N;
  if (c->opts.precision == GLS_INT8_EMU) {
    {
      PhaseTimer t(c, PH_WHITEN, s);
      hipLaunchKernelGGL(unpack_u2_kernel, dim3(grid_for(N / 4 * mb)), dim3(256), 0, s, G2, ldg, (int)c->n, (int)N,
                         mb, reinterpret_cast<uint32_t*>(c->ubp));
      ozaki_product(c, mb, s);
    }
    PhaseTimer t(c, PH_SNP, s);
    snp_reduce_solve(c, c->Xt, mb, b, ld_b, s2, v, st, s);
    return GLS_OK;
  }
  widen_u2(c, G2, ldg, mb, s);
  return block_forward(c, mb, c->x64, N, b, ld_b, s2, v, st, s);
}

void reset_adjoint(Ctx* c, hipStream_t s) {
  const int64_t N = c->N;
  // T2 holds (L^-1)^T until the Cholesky adjoint of the pass's finish step reuses it: the per-block
  // X_R bar = L^-T X~_R bar then reads an upper-triangular A without a transpose (the direct-load product)
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((N + 31) / 32), (unsigned)((N + 31) / 32)), dim3(256), 0, s,
                     c->T2, N, c->Linv, N, (int)N, (int)N);
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(N * N)), dim3(256), 0, s, c->Lbar, N * N, 0.0);
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(N * c->p)), dim3(256), 0, s, c->Wb, N * c->p, 0.0);
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(256), 0, s, c->acc, (int64_t)adj_nc(c->p), 0.0);
}

template <int P>
static void adjoint_snp_p(Ctx* c, int mb, const double* bbar, const double* s2bar, const double* vbar,
                          hipStream_t s) {
  const int grid = (mb + SNP_PER_WG - 1) / SNP_PER_WG;
  hipLaunchKernelGGL(snp_adjoint_kernel<P>, dim3(grid), dim3(64 * SNP_WAVES), 0, s, c->Xt, (int64_t)c->N, (int)c->N,
                     mb, c->W, c->small, (int)c->n, bbar, (int64_t)P, s2bar, vbar, c->Cb, c->eb, c->ct);
  hipLaunchKernelGGL(reduce_contrib_kernel, dim3(adj_nc(P)), dim3(256), 0, s, c->ct, adj_nc(P), mb, c->acc);
  hipLaunchKernelGGL(xtbar_kernel<P>, dim3(grid_for(c->N * mb)), dim3(256), 0, s, c->W, c->Xt, c->Cb, c->eb,
                     (int)c->N, mb, c->Xtb);
}

template <int P>
static void wbar_shared_p(Ctx* c, hipStream_t s) {
  hipLaunchKernelGGL(wbar_shared_kernel<P>, dim3(grid_for(c->N)), dim3(256), 0, s, c->W, c->acc, (int)c->N, c->Wb);
}

#define GLS_P_SWITCH(p, CALL)                                                                          \
  switch (p) {                                                                                         \
    case 1: CALL(1); break; case 2: CALL(2); break; case 3: CALL(3); break; case 4: CALL(4); break;     \
    case 5: CALL(5); break; case 6: CALL(6); break; case 7: CALL(7); break; case 8: CALL(8); break;     \
    case 9: CALL(9); break; case 10: CALL(10); break; case 11: CALL(11); break; case 12: CALL(12); break; \
    case 13: CALL(13); break; case 14: CALL(14); break; case 15: CALL(15); break; case 16: CALL(16); break; \
    case 17: CALL(17); break; case 18: CALL(18); break; case 19: CALL(19); break; case 20: CALL(20); break; \
    default: break;                                                                                    \
  }

// X~ of a block again (the adjoint recomputes instead of storing X~_R).
static void recompute_whitened(Ctx* c, int mb, const double* XR, int64_t ld_xr, hipStream_t s) {
  if (c->plan.lp_bytes) {
    lp_solve(c, XR, ld_xr, mb, 0.0, s);
    for (int sweep = 0; sweep < c->opts.refine_sweeps; ++sweep) {
      residual_fp64(c, XR, ld_xr, mb, s);
      lp_solve(c, c->R, c->N, mb, 1.0, s);
    }
  } else {
    int K = 0;
    const double* X = fp64_operand(c, XR, &ld_xr, mb, &K, s);
    whiten_fp64(c, X, ld_xr, mb, K, (int)c->N, c->Xt, s);
  }
}

gls_status block_backward(Ctx* c, int mb, const double* XR, int64_t ld_xr, const double* bbar, const double* s2bar,
                          const double* vbar, double* XR_grad, hipStream_t s) {
  const int64_t N = c->N;
  PhaseTimer t(c, PH_BACKWARD, s);
  recompute_whitened(c, mb, XR, ld_xr, s);
#define GLS_ADJ(P) adjoint_snp_p<P>(c, mb, bbar, s2bar, vbar, s)
  GLS_P_SWITCH(c->p, GLS_ADJ)
#undef GLS_ADJ
  {  // Wbar += X~_R Cbar^T in groups of 16 SNPs: group sums into Xb (free until the next product), then added in
     // group order; as many groups per pass as Xb holds (p columns of N per group)
    const int p = c->p;
    const int groups = (mb + ADJ_GROUP - 1) / ADJ_GROUP;
    const int per_pass = (int)std::max<int64_t>(1, c->plan.bcp / p);
    for (int g0 = 0; g0 < groups; g0 += per_pass) {
      const int gn = std::min(per_pass, groups - g0);
#define GLS_WG(P)                                                                                                  \
  hipLaunchKernelGGL(wbar_group_kernel<P>, dim3((unsigned)((N + 255) / 256), (unsigned)gn), dim3(256), 0, s, c->Xt, \
                     (int)N, mb, g0, c->Cb, c->Xb);
      GLS_P_SWITCH(p, GLS_WG)
#undef GLS_WG
      hipLaunchKernelGGL(wbar_add_kernel, dim3(grid_for(N * p)), dim3(256), 0, s, c->Xb, (int)N, p, gn, c->Wb);
    }
  }
  {  // X_R bar = L^-T X~_R bar   (A = (L^-1)^T in T2, upper: non-zero for k >= i; low row tiles hold the most k)
    GemmArgs g = gemm_args(c->T2, N, c->Xtb, N, c->Xb, N, (int)N, mb, (int)N, 1.0);
    g.a_tri = TRI_UPPER;
    g.a_diag = 0;
    g.map_desc = 0;
    gemm(false, false, true, g, s);
  }
  if (XR_grad)
    hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for(c->n * mb)), dim3(256), 0, s, XR_grad, ld_xr, c->Xb, N, (int)c->n,
                       mb);
  // Lbar -= X_R bar X~_R^T (lower tiles; high row tiles hold the most of them) on the direct-load kernel:
  // X~_R^T is formed in Xtb (free once X_R bar is formed), the SNP count is padded to a multiple of 16 with
  // zero SNPs, and the accumulators start from -Lbar, so the 16-SNP stages add onto the running Lbar in SNP
  // order: for block widths that are multiples of 16 Lbar is bitwise independent of the blocking.
  {
    const int K16 = (mb + DB_BK - 1) / DB_BK * DB_BK;
    if (K16 > mb) {
      hipLaunchKernelGGL(fill_kernel, dim3(grid_for(N * (K16 - mb))), dim3(256), 0, s, c->Xt + N * mb,
                         N * (K16 - mb), 0.0);
      hipLaunchKernelGGL(fill_kernel, dim3(grid_for(N * (K16 - mb))), dim3(256), 0, s, c->Xb + N * mb,
                         N * (K16 - mb), 0.0);
    }
    hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)((N + 31) / 32), (unsigned)((K16 + 31) / 32)), dim3(256), 0,
                       s, c->Xtb, (int64_t)K16, c->Xt, N, (int)N, K16);
    GemmArgs g = gemm_args(c->Xb, N, c->Xtb, K16, c->Lbar, N, (int)N, (int)N, K16, -1.0);
    g.beta = 1.0;
    g.acc_cin = 1;
    g.c_lower = 1;
    g.c_diag = 0;
    g.map_desc = 1;
    gemm(false, false, true, g, s);
  }
  return GLS_OK;
}

gls_status finish_backward(Ctx* c, double* y_grad, double* h2_grad, hipStream_t s) {
  const int64_t N = c->N;
  const int p = c->p;
  PhaseTimer t(c, PH_BACKWARD, s);
#define GLS_WB(P) wbar_shared_p<P>(c, s)
  GLS_P_SWITCH(p, GLS_WB)
#undef GLS_WB
  // [X_L | y] bar = L^-T [X~_L | y~] bar
#define GLS_TT(P) \
  hipLaunchKernelGGL(tri_apply_t_kernel<P>, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s, c->Linv, (int)N, c->Wb, c->W0b);
  GLS_P_SWITCH(p, GLS_TT)
#undef GLS_TT
  if (y_grad)
    hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for(c->n)), dim3(256), 0, s, y_grad, c->n, c->W0b + (int64_t)(p - 1) * N,
                       N, (int)c->n, 1);
  {  // Lbar -= [X_L | y]bar [X~_L | y~]^T
    GemmArgs g = gemm_args(c->W0b, N, c->W, N, c->Lbar, N, (int)N, (int)N, p, -1.0);
    g.beta = 1.0;
    g.c_lower = 1;
    g.c_diag = 0;
    gemm(false, true, false, g, s);
  }
  const int gN = grid_for(N * N);
  hipLaunchKernelGGL(lower_part_kernel, dim3(gN), dim3(256), 0, s, c->Lbar, (int)N, 0);
  {  // T1 = lower part of L^T Lbar   (op(A) = L^T upper, op(B) = Lbar lower)
    GemmArgs g = gemm_args(c->L, N, c->Lbar, N, c->T1, N, (int)N, (int)N, (int)N, 1.0);
    g.a_tri = TRI_UPPER;
    g.a_diag = 0;
    g.b_tri = TRI_LOWER;
    g.b_diag = 0;
    g.c_lower = 1;
    g.c_diag = 0;
    gemm(true, false, true, g, s);   // k from the row: low row tiles first
  }
  hipLaunchKernelGGL(lower_part_kernel, dim3(gN), dim3(256), 0, s, c->T1, (int)N, 1);
  {  // T2 = T1 L^-1   (lower x lower = lower)
    GemmArgs g = gemm_args(c->T1, N, c->Linv, N, c->T2, N, (int)N, (int)N, (int)N, 1.0);
    g.a_tri = TRI_LOWER;
    g.a_diag = 0;
    g.b_tri = TRI_LOWER;
    g.b_diag = 0;
    g.c_lower = 1;
    g.c_diag = 0;
    g.map_desc = 1;
    gemm(false, false, true, g, s);   // k in [column, row]: high row tiles first
  }
  {  // T1 = L^-T T2   (the adjoint of M, up to symmetrisation)
    GemmArgs g = gemm_args(c->Linv, N, c->T2, N, c->T1, N, (int)N, (int)N, (int)N, 1.0);
    g.a_tri = TRI_UPPER;
    g.a_diag = 0;
    g.b_tri = TRI_LOWER;
    g.b_diag = 0;
    gemm(true, false, true, g, s);   // k from the row: low row tiles first
  }
  double* part = c->acc + adj_nc(p);
  hipLaunchKernelGGL(h2_contract_kernel, dim3(1024), dim3(256), 0, s, c->T1, c->Phi, (int)N, (int)c->n, part);
  if (h2_grad) hipLaunchKernelGGL(sum_ordered_kernel, dim3(1), dim3(64), 0, s, part, 1024, h2_grad);
  reset_adjoint(c, s);
  return GLS_OK;
}

}  // namespace gls

extern "C" gls_status gls_backward_block(gls_handle h, int32_t mb, const double* XR, int64_t ld_xr,
                                         const double* b_bar, const double* sigma2_bar, const double* v_bar,
                                         double* XR_grad, void* stream) {
  Ctx* c = h;
  if (!c || !c->ready || !c->grad) {
    set_err("gls_backward_block: handle not set up with GLS_KEEP_FOR_GRAD");
    return GLS_ERR_STATE;
  }
  if (mb < 0 || mb > c->bc) return arg_fail("gls_backward_block: mb must lie in [0, block_cols]");
  if (mb == 0) return GLS_OK;
  if (!XR || ld_xr < c->n) return arg_fail("gls_backward_block: XR is NULL or ld_xr < n");
  if (!b_bar || !sigma2_bar || !v_bar) return arg_fail("gls_backward_block: NULL cotangent");
  hipStream_t s = static_cast<hipStream_t>(stream);
  gls_status st = block_backward(c, mb, XR, ld_xr, b_bar, sigma2_bar, v_bar, XR_grad, s);
  if (st != GLS_OK) return st;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "gls_backward_block: launch");
  return GLS_OK;
}

extern "C" gls_status gls_backward_finish(gls_handle h, double* y_grad, double* h2_grad, void* stream) {
  Ctx* c = h;
  if (!c || !c->ready || !c->grad) {
    set_err("gls_backward_finish: handle not set up with GLS_KEEP_FOR_GRAD");
    return GLS_ERR_STATE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  gls_status st = finish_backward(c, y_grad, h2_grad, s);
  if (st != GLS_OK) return st;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "gls_backward_finish: launch");
  return GLS_OK;
}
