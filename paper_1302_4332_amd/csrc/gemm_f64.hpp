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
// owns a (BM/WAVES_M) x (BN/WAVES_N) sub-tile.  Two FP64 matrix instructions
// are supported (operand layouts checked on gfx950 with one-hot operands):
//
//  v_mfma_f64_16x16x4f64 (M4 = false), 16x16 accumulators:
//   A fragment: lane l holds A[l % 16][l / 16]  (16 rows x 4 k)
//   B fragment: lane l holds B[l / 16][l % 16]  (4 k x 16 columns)
//   accumulator: lane l, element t holds C[l / 16 + 4 * t][l % 16]
//
//  v_mfma_f64_4x4x4_4b_f64 (M4 = true): four independent 4x4x4 products,
//   block b = (l >> 2) & 3 of lane l; A[b][l & 3][l >> 4], B[b][l >> 4][l & 3],
//   D[b][l >> 4][l & 3].  Taking the four blocks as four consecutive 4-row
//   blocks of a 16-row strip makes the A fragment identical to the one above
//   (A[l % 16][l / 16]); the B fragment is a 4-column slice B[l / 16][l % 4]
//   shared by the four blocks, and the lane's one accumulator holds
//   C[4 * ((l >> 2) & 3) + (l >> 4)][l & 3].  On gfx950 this form sustains
//   close to the FP64 peak, about 1.6x the 16x16x4 form.
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
  // MAP_XCD only: row tiles handled heavy-first (desc = rows with most k first);
  // map_gm x map_gn tiles per co-resident group on one XCD (0 = defaults)
  int map_desc;
  int map_gm, map_gn;
  int map_slab;   // 1: column groups outer (a slab of GN column tiles meets every row tile in turn)
  // trmm_f64_dma_kernel only: with red_q > 0, C is not stored; instead each
  // row tile ti writes, for every column j, the red_q sums over its rows
  // sum_i C[i,j] red_W[i + q ld_red_W] (q < red_q - 1) and sum_i C[i,j]^2
  // (q = red_q - 1) to red_part[(ti red_q + q) ncols + j]
  const double* red_W; int64_t ld_red_W;
  double* red_part;
  int red_q;
  // trmm_f64_dma_kernel only: with acc_cin (alpha = +-1, beta = 1) the
  // accumulators start at alpha Cin and C = alpha acc: the k stages add onto
  // the running value in order, so a sum split over launches at stage
  // boundaries gives bitwise the result of one launch
  int acc_cin;
};

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

// XCD-aware workgroup -> tile mapping.  Workgroups are dispatched to the 8
// XCDs round-robin (workgroup id % 8), so row tiles are dealt to the XCDs in
// a snake order (balanced k-work) and, on each XCD, groups of GM local row
// tiles x GN column tiles run together so the operand strips they share stay
// in that XCD's L2.  Row groups are issued heavy-first.
struct XcdMap {
  static constexpr int GM_DEFAULT = 1;   // measured best on gfx950 for the
  static constexpr int GN_DEFAULT = 16;  // n = 10,000 per-block product
  __host__ __device__ static int gm(const GemmArgs& g) { return g.map_gm > 0 ? g.map_gm : GM_DEFAULT; }
  __host__ __device__ static int gn(const GemmArgs& g) { return g.map_gn > 0 ? g.map_gn : GN_DEFAULT; }
  __host__ __device__ static int rounds(int Mt) { return (Mt + 7) / 8; }
  __host__ __device__ static int slots_per_xcd(int Mt, int Nt, int GM, int GN) {
    int R = rounds(Mt);
    int rg = (R + GM - 1) / GM;
    int cg = (Nt + GN - 1) / GN;
    return rg * cg * GM * GN;
  }
  __host__ static int grid(const GemmArgs& g, int Mt, int Nt) { return 8 * slots_per_xcd(Mt, Nt, gm(g), gn(g)); }
  // returns false for an idle slot
  __device__ static bool tile(const GemmArgs& ga, int bid, int Mt, int Nt, int* ti, int* tj) {
    const int GM = gm(ga), GN = gn(ga);
    int x = bid & 7;
    int s = bid >> 3;
    int R = rounds(Mt);
    int cg = (Nt + GN - 1) / GN;
    int per_group = GM * GN;
    int g = s / per_group;
    int w = s - g * per_group;
    const int rg = (R + GM - 1) / GM;
    int rgi, cgi;
    if (ga.map_slab) {                // column group outer, row groups heavy first inside
      cgi = g / rg;
      rgi = g - cgi * rg;
    } else {                          // row group (heavy first) outer
      rgi = g / cg;
      cgi = g - rgi * cg;
    }
    int kl = rgi * GM + (w % GM);     // local row index on this XCD
    int j = cgi * GN + (w / GM);
    if (kl >= R || j >= Nt) return false;
    int pos = (kl & 1) ? (7 - x) : x;
    int ro = kl * 8 + pos;
    if (ro >= Mt) return false;
    *ti = ga.map_desc ? (Mt - 1 - ro) : ro;
    *tj = j;
    return true;
  }
};

template <int BM, int BN, int BK, int NT, bool TRANS_A, bool TRANS_B, bool VEC>
struct Stager {
  static constexpr int SA = BM + 16;   // row strides (doubles): +16 puts k and k+1 on
  static constexpr int SB = BN + 16;   // opposite halves of the LDS banks
  static constexpr int W = VEC ? 8 : 1;
  static constexpr int TA = BM * BK / W;   // chunks (or doubles) per slice
  static constexpr int TB = BN * BK / W;
  static constexpr int CA = (TA + NT - 1) / NT;   // per thread (the last round may be partial)
  static constexpr int CB = (TB + NT - 1) / NT;
  static_assert(TA % NT == 0 || NT % TA == 0, "loader split");
  static_assert(TB % NT == 0 || NT % TB == 0, "loader split");
  double ra[CA * W], rb[CB * W];

  __device__ __forceinline__ static void vload8(double* dst, const double* src) {
    const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double2 v = s2[q];
      dst[2 * q] = v.x;
      dst[2 * q + 1] = v.y;
    }
  }

  __device__ __forceinline__ void load(const GemmArgs& g, int i0, int j0, int kt, int tid) {
#pragma unroll
    for (int e = 0; e < CA; ++e) {
      const int c = tid + e * NT;
      if (TA < NT && c >= TA) break;
      int i, k;
      if (!TRANS_A) { i = (c % (BM / W)) * W; k = c / (BM / W); }
      else          { k = (c % (BK / W)) * W; i = c / (BK / W); }
      const int gi = i0 + i, gk = kt + k;
      if (VEC) {
        if (gi < g.mvalid && gk < g.K) {
          vload8(&ra[e * 8], TRANS_A ? g.A + (int64_t)gk + (int64_t)gi * g.lda : g.A + (int64_t)gi + (int64_t)gk * g.lda);
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) ra[e * 8 + q] = 0.0;
        }
      } else {
        ra[e] = (gi < g.mvalid && gk < g.K)
                    ? (TRANS_A ? g.A[(int64_t)gk + (int64_t)gi * g.lda] : g.A[(int64_t)gi + (int64_t)gk * g.lda])
                    : 0.0;
      }
    }
#pragma unroll
    for (int e = 0; e < CB; ++e) {
      const int c = tid + e * NT;
      if (TB < NT && c >= TB) break;
      int j, k;
      if (!TRANS_B) { k = (c % (BK / W)) * W; j = c / (BK / W); }
      else          { j = (c % (BN / W)) * W; k = c / (BN / W); }
      const int gj = j0 + j, gk = kt + k;
      if (VEC) {
        if (gj < g.ncols && gk < g.K) {
          vload8(&rb[e * 8], TRANS_B ? g.B + (int64_t)gj + (int64_t)gk * g.ldb : g.B + (int64_t)gk + (int64_t)gj * g.ldb);
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) rb[e * 8 + q] = 0.0;
        }
      } else {
        rb[e] = (gj < g.ncols && gk < g.K)
                    ? (TRANS_B ? g.B[(int64_t)gj + (int64_t)gk * g.ldb] : g.B[(int64_t)gk + (int64_t)gj * g.ldb])
                    : 0.0;
      }
    }
  }

  __device__ __forceinline__ void store(double* As, double* Bs, int tid) const {
#pragma unroll
    for (int e = 0; e < CA; ++e) {
      const int c = tid + e * NT;
      if (TA < NT && c >= TA) break;
      int i, k;
      if (!TRANS_A) { i = (c % (BM / W)) * W; k = c / (BM / W); }
      else          { k = (c % (BK / W)) * W; i = c / (BK / W); }
      if (VEC && !TRANS_A) {
        double2* d = reinterpret_cast<double2*>(As + k * SA + i);
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = double2{ra[e * 8 + 2 * q], ra[e * 8 + 2 * q + 1]};
      } else {
#pragma unroll
        for (int q = 0; q < W; ++q) As[(k + (TRANS_A ? q : 0)) * SA + i + (TRANS_A ? 0 : q)] = ra[e * W + q];
      }
    }
#pragma unroll
    for (int e = 0; e < CB; ++e) {
      const int c = tid + e * NT;
      if (TB < NT && c >= TB) break;
      int j, k;
      if (!TRANS_B) { k = (c % (BK / W)) * W; j = c / (BK / W); }
      else          { j = (c % (BN / W)) * W; k = c / (BN / W); }
      if (VEC && TRANS_B) {
        double2* d = reinterpret_cast<double2*>(Bs + k * SB + j);
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = double2{rb[e * 8 + 2 * q], rb[e * 8 + 2 * q + 1]};
      } else {
#pragma unroll
        for (int q = 0; q < W; ++q) Bs[(k + (TRANS_B ? 0 : q)) * SB + j + (TRANS_B ? q : 0)] = rb[e * W + q];
      }
    }
  }
};

template <int BM, int BN, int BK, int WAVES_M, int WAVES_N, bool TRANS_A, bool TRANS_B, int MAP, bool VEC,
          bool M4 = true>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N)
void gemm_f64_kernel(GemmArgs g) {
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int WTM = BM / WAVES_M;
  constexpr int WTN = BN / WAVES_N;
  constexpr int FM = WTM / 16;
  constexpr int FN = WTN / 16;
  using St = Stager<BM, BN, BK, NT, TRANS_A, TRANS_B, VEC>;
  constexpr int SA = St::SA;
  constexpr int SB = St::SB;
  static_assert(BM % (16 * WAVES_M) == 0 && BN % (16 * WAVES_N) == 0, "tile");
  static_assert(BK % 8 == 0, "k step");

  __shared__ double As[2][BK * SA];
  __shared__ double Bs[2][BK * SB];

  int ti, tj;
  if (MAP == MAP_XCD) {
    const int Mt = g.M / BM;
    const int Nt = (g.ncols + BN - 1) / BN;
    if (!XcdMap::tile(g, blockIdx.x, Mt, Nt, &ti, &tj)) return;
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

  constexpr int FC = WTN / 4;   // 4-column slices per wave (M4)
  d4_t acc[M4 ? 1 : FM][M4 ? 1 : FN];
  double acc4[M4 ? FM : 1][M4 ? FC : 1];
  if (M4) {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int c = 0; c < FC; ++c) acc4[a][c] = 0.0;
  } else {
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) acc[a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
  }

  St st;
  if (nk > 0) {
    st.load(g, i0, j0, klo, tid);
    st.store(As[0], Bs[0], tid);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int buf = it & 1;
      if (it + 1 < nk) st.load(g, i0, j0, klo + (it + 1) * BK, tid);
      const double* as = As[buf];
      const double* bs = Bs[buf];
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const int kr = kk + (lane >> 4);
        double af[FM];
#pragma unroll
        for (int a = 0; a < FM; ++a) af[a] = as[kr * SA + wm * WTM + a * 16 + (lane & 15)];
        if (M4) {
#pragma unroll
          for (int c = 0; c < FC; ++c) {
            const double bf = bs[kr * SB + wn * WTN + c * 4 + (lane & 3)];
#pragma unroll
            for (int a = 0; a < FM; ++a) acc4[a][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[a], bf, acc4[a][c], 0, 0, 0);
          }
        } else {
          double bf[FN];
#pragma unroll
          for (int b = 0; b < FN; ++b) bf[b] = bs[kr * SB + wn * WTN + b * 16 + (lane & 15)];
#pragma unroll
          for (int a = 0; a < FM; ++a)
#pragma unroll
            for (int b = 0; b < FN; ++b)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
      }
      if (it + 1 < nk) st.store(As[buf ^ 1], Bs[buf ^ 1], tid);
      __syncthreads();
    }
  }

  if (M4) {
    // lane holds C[4 * ((lane >> 2) & 3) + (lane >> 4)][lane & 3] of each 16 x 4 slice
#pragma unroll
    for (int a = 0; a < FM; ++a) {
      const int i = i0 + wm * WTM + a * 16 + 4 * ((lane >> 2) & 3) + (lane >> 4);
      if (i >= g.mvalid) continue;
#pragma unroll
      for (int c = 0; c < FC; ++c) {
        const int j = j0 + wn * WTN + c * 4 + (lane & 3);
        if (j >= g.ncols) continue;
        double val = g.alpha * acc4[a][c];
        if (g.beta != 0.0) val += g.beta * g.Cin[(int64_t)i + (int64_t)j * g.ldcin];
        g.C[(int64_t)i + (int64_t)j * g.ldc] = val;
      }
    }
    return;
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

// Whether the chunked (VEC) loader may be used for these arguments.
inline bool gemm_vec_ok(const GemmArgs& g, bool ta, bool tb) {
  auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  if (!al16(g.A) || !al16(g.B) || (g.lda & 1) || (g.ldb & 1)) return false;
  // chunks run along i for A (no transpose) or k (transpose); along k for B
  // (no transpose) or j (transpose): the run's bound must be a multiple of 8
  if (!ta && (g.mvalid % 8)) return false;
  if ((ta || !tb) && (g.K % 8)) return false;
  if (tb && (g.ncols % 8)) return false;
  return true;
}

}  // namespace gls
