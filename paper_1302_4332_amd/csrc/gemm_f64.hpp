// FP64 MFMA matrix-product engine for gfx950.
//
//   C[i, j] = alpha * sum_k op(A)[i, k] * op(B)[k, j] + beta * Cin[i, j]
//
// with optional triangular structure of op(A) / op(B) (the k-range of a tile
// is clipped to where the triangular operand can be non-zero; the operand
// must hold explicit zeros outside its triangle) and an optional
// lower-triangle-only output.  It is the one engine behind every level-3 step
// of the solver: the per-block product with the inverse Cholesky factor, the
// Cholesky trailing updates and panel products, the blocked triangular
// inversion, the refinement residual and the adjoint products.
//
// Tiles are BM x BN per workgroup, staged through LDS in BK-deep slices with
// a register prefetch of the next slice and double-buffered LDS.  Each wave
// owns a (BM/WAVES_M) x (BN/WAVES_N) sub-tile built from 16x16 accumulators
// of v_mfma_f64_16x16x4f64.  Operand layout of that instruction (64 lanes):
//   A fragment: lane l holds A[l % 16][l / 16]  (16 rows x 4 k)
//   B fragment: lane l holds B[l / 16][l % 16]  (4 k x 16 columns)
//   accumulator: lane l, element t holds C[l / 16 + 4 * t][l % 16]
//   (rows interleaved by 4; checked on gfx950 with one-hot operands).
//
// Every output element is summed over the same k order whatever the block
// width or the tile's column position, so results are bitwise independent
// of how SNP columns are grouped into blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gls {

typedef double d4_t __attribute__((ext_vector_type(4)));

enum { TRI_NONE = 0, TRI_LOWER = 1, TRI_UPPER = 2 };
enum { MAP_GRID = 0, MAP_XCD = 1 };

struct GemmArgs {
  const double* A; int64_t lda;     // op(A) = A (TRANS_A false) or A^T
  const double* B; int64_t ldb;     // op(B) = B (TRANS_B false) or B^T
  const double* Cin; int64_t ldcin; // read only when beta != 0
  double* C; int64_t ldc;
  int M;         // rows of the iteration space (multiple of BM)
  int mvalid;    // rows >= mvalid: op(A) reads 0, C is not stored
  int ncols;     // output columns; columns >= ncols: op(B) reads 0, not stored
  int K;         // sum over k < K; op(A)/op(B) read 0 for k >= K
  double alpha, beta;
  int a_tri, a_diag;   // LOWER: op(A)[i,k] = 0 for k > i + a_diag; UPPER: for k < i + a_diag
  int b_tri, b_diag;   // LOWER: op(B)[k,j] = 0 for k < j + b_diag; UPPER: for k > j + b_diag
  int c_lower, c_diag; // skip tiles whose every (i, j) has i < j + c_diag
  // MAP_XCD only: row tiles handled heavy-first (desc = rows with most k first)
  int map_desc;
};

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

// Row/column tile counts and workgroup count of the XCD-aware mapping.
// Row tiles are dealt to the 8 XCDs in a snake order (balanced k-work);
// on each XCD a group of GM local row tiles x GN column tiles runs together
// so both operand strips are shared through that XCD's L2.
struct XcdMap {
  static constexpr int GM = 4;
  static constexpr int GN = 16;
  __host__ __device__ static int rounds(int Mt) { return (Mt + 7) / 8; }
  __host__ __device__ static int slots_per_xcd(int Mt, int Nt) {
    int R = rounds(Mt);
    int rg = (R + GM - 1) / GM;
    int cg = (Nt + GN - 1) / GN;
    return rg * cg * GM * GN;
  }
  __host__ static int grid(int Mt, int Nt) { return 8 * slots_per_xcd(Mt, Nt); }
  // returns false for an idle slot
  __device__ static bool tile(int bid, int Mt, int Nt, int desc, int* ti, int* tj) {
    int x = bid & 7;
    int s = bid >> 3;
    int R = rounds(Mt);
    int cg = (Nt + GN - 1) / GN;
    int per_group = GM * GN;
    int g = s / per_group;
    int w = s - g * per_group;
    int rgi = g / cg;                 // row group (heavy first)
    int cgi = g - rgi * cg;           // column group
    int kl = rgi * GM + (w % GM);     // local row index on this XCD
    int j = cgi * GN + (w / GM);
    if (kl >= R || j >= Nt) return false;
    int pos = (kl & 1) ? (7 - x) : x;
    int ro = kl * 8 + pos;
    if (ro >= Mt) return false;
    *ti = desc ? (Mt - 1 - ro) : ro;
    *tj = j;
    return true;
  }
};

template <int BM, int BN, int BK, int WAVES_M, int WAVES_N, bool TRANS_A, bool TRANS_B, int MAP>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N)
void gemm_f64_kernel(GemmArgs g) {
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int WTM = BM / WAVES_M;
  constexpr int WTN = BN / WAVES_N;
  constexpr int FM = WTM / 16;
  constexpr int FN = WTN / 16;
  constexpr int EA = BM * BK / NT;
  constexpr int EB = BN * BK / NT;
  constexpr int SA = BM + 2;   // LDS row strides (doubles); +2 staggers banks
  constexpr int SB = BN + 2;
  static_assert(BM % (16 * WAVES_M) == 0 && BN % (16 * WAVES_N) == 0, "tile");
  static_assert((BM * BK) % NT == 0 && (BN * BK) % NT == 0, "loader");
  static_assert(BK % 4 == 0, "k step");

  __shared__ double As[2][BK * SA];
  __shared__ double Bs[2][BK * SB];

  int ti, tj;
  if (MAP == MAP_XCD) {
    const int Mt = g.M / BM;
    const int Nt = (g.ncols + BN - 1) / BN;
    if (!XcdMap::tile(blockIdx.x, Mt, Nt, g.map_desc, &ti, &tj)) return;
  } else {
    tj = blockIdx.x;
    ti = blockIdx.y;
  }
  const int i0 = ti * BM;
  const int j0 = tj * BN;
  if (g.c_lower && (i0 + BM - 1) < (j0 + g.c_diag)) return;

  int klo = 0, khi = g.K;
  if (g.a_tri == TRI_LOWER) khi = imin(khi, i0 + BM + g.a_diag);
  if (g.a_tri == TRI_UPPER) klo = imax(klo, i0 + g.a_diag);
  if (g.b_tri == TRI_LOWER) klo = imax(klo, j0 + g.b_diag);
  if (g.b_tri == TRI_UPPER) khi = imin(khi, j0 + BN + g.b_diag);
  klo = (klo / BK) * BK;
  int nk = (khi > klo) ? (khi - klo + BK - 1) / BK : 0;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WAVES_M;
  const int wn = wave / WAVES_M;

  d4_t acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};

  double ra[EA], rb[EB];

  auto load = [&](int kt) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int idx = tid + e * NT;
      int i, k;
      if (!TRANS_A) { i = idx % BM; k = idx / BM; }
      else          { k = idx % BK; i = idx / BK; }
      int gi = i0 + i, gk = kt + k;
      double val = 0.0;
      if (gi < g.mvalid && gk < g.K)
        val = TRANS_A ? g.A[(int64_t)gk + (int64_t)gi * g.lda] : g.A[(int64_t)gi + (int64_t)gk * g.lda];
      ra[e] = val;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int idx = tid + e * NT;
      int j, k;
      if (!TRANS_B) { k = idx % BK; j = idx / BK; }
      else          { j = idx % BN; k = idx / BN; }
      int gj = j0 + j, gk = kt + k;
      double val = 0.0;
      if (gj < g.ncols && gk < g.K)
        val = TRANS_B ? g.B[(int64_t)gj + (int64_t)gk * g.ldb] : g.B[(int64_t)gk + (int64_t)gj * g.ldb];
      rb[e] = val;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int idx = tid + e * NT;
      int i, k;
      if (!TRANS_A) { i = idx % BM; k = idx / BM; }
      else          { k = idx % BK; i = idx / BK; }
      As[buf][k * SA + i] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int idx = tid + e * NT;
      int j, k;
      if (!TRANS_B) { k = idx % BK; j = idx / BK; }
      else          { j = idx % BN; k = idx / BN; }
      Bs[buf][k * SB + j] = rb[e];
    }
  };

  if (nk > 0) {
    load(klo);
    store(0);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int buf = it & 1;
      if (it + 1 < nk) load(klo + (it + 1) * BK);
      const double* as = As[buf];
      const double* bs = Bs[buf];
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double af[FM], bf[FN];
        const int kr = kk + (lane >> 4);
#pragma unroll
        for (int a = 0; a < FM; ++a) af[a] = as[kr * SA + wm * WTM + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < FN; ++b) bf[b] = bs[kr * SB + wn * WTN + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < FM; ++a)
#pragma unroll
          for (int b = 0; b < FN; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
      }
      if (it + 1 < nk) store(buf ^ 1);
      __syncthreads();
    }
  }

  // epilogue: lane holds rows q, q+4, q+8, q+12 (q = lane / 16) of one column
#pragma unroll
  for (int a = 0; a < FM; ++a) {
    const int ib = i0 + wm * WTM + a * 16 + (lane >> 4);
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      const int j = j0 + wn * WTN + b * 16 + (lane & 15);
      if (j >= g.ncols) continue;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = ib + 4 * t;
        if (i >= g.mvalid) continue;
        double val = g.alpha * acc[a][b][t];
        if (g.beta != 0.0) val += g.beta * g.Cin[(int64_t)i + (int64_t)j * g.ldcin];
        g.C[(int64_t)i + (int64_t)j * g.ldc] = val;
      }
    }
  }
}

}  // namespace gls
