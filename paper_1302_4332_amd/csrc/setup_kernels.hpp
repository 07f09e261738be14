// Setup-phase kernels: forming M, the in-LDS factorization and inversion of
// the diagonal blocks, packing, and the small Gram matrix of [X~_L | y~].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gls {

// Leaf (diagonal block) size of the blocked Cholesky / inversion.
constexpr int NB_LEAF = 64;

// L <- M = h2 * Phi + (1 - h2) * I in the lower triangle of the leading n x n
// block (read from Phi's lower triangle), identity on the padding rows
// n..N-1, zeros above the diagonal.  N x N column-major, ld = N.
__global__ void form_m_kernel(double* __restrict__ L, int N, int n,
                              const double* __restrict__ Phi, int64_t ld_phi, double h2) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)N * N;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(idx % N);
    int j = (int)(idx / N);
    double v = 0.0;
    if (i >= j) {
      if (i < n) v = h2 * Phi[(int64_t)i + (int64_t)j * ld_phi] + (i == j ? (1.0 - h2) : 0.0);
      else if (i == j) v = 1.0;
    }
    L[idx] = v;
  }
}

__global__ void fill_kernel(double* __restrict__ p, int64_t count, double v) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; idx < count; idx += (int64_t)gridDim.x * blockDim.x) p[idx] = v;
}

// dst (rows x cols, ld_dst) <- src (rows x cols, ld_src)
__global__ void copy2d_kernel(double* __restrict__ dst, int64_t ld_dst,
                              const double* __restrict__ src, int64_t ld_src, int rows, int cols) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)rows * cols;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(idx % rows);
    int j = (int)(idx / rows);
    dst[(int64_t)i + (int64_t)j * ld_dst] = src[(int64_t)i + (int64_t)j * ld_src];
  }
}

// Wpack (N x p, ld N) <- [X_L | y] with zero rows n..N-1.
__global__ void pack_covariates_kernel(double* __restrict__ Wp, int N, int n, int p,
                                       const double* __restrict__ XL, int64_t ld_xl,
                                       const double* __restrict__ y) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)N * p;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(idx % N);
    int j = (int)(idx / N);
    double v = 0.0;
    if (i < n) v = (j < p - 1) ? XL[(int64_t)i + (int64_t)j * ld_xl] : y[i];
    Wp[idx] = v;
  }
}

// 1/p to full double precision: hardware reciprocal estimate plus two
// Newton steps (off the IEEE division's long sequence; used where the last
// bit is immaterial, the pivots of the right-looking update).
__device__ __forceinline__ double fast_rcp(double p) {
  double r = __builtin_amdgcn_rcp(p);
  double e = __builtin_fma(-p, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-p, r, 1.0);
  return __builtin_fma(r, e, r);
}

// One diagonal block of the blocked factorization, entirely on chip:
//   Cholesky of the NB_LEAF x NB_LEAF lower block at A (ld), right-looking.
//   Each thread keeps its share of the trailing matrix in registers (column
//   kc = t % 64, rows kc + t/64 + 4q, q < 16; entries past the block are
//   dummies, so no per-entry branches).  At step j the owners of column j
//   publish it (unscaled) into its own LDS column, one barrier per step, and
//   every later column is updated with that column times 1/pivot.  The
//   columns are scaled by 1/sqrt(pivot) after the loop, in parallel.
//   Then the inverse of the factor, right-looking as well: lane jj holds
//   column jj of the inverse in registers; at step k its entry k is scaled by
//   1/L[k][k] and subtracted, times L[i][k], from every later entry i (the
//   same terms, in the same order, as forward substitution).
//   Writes the factor (zero upper part) back to A and the inverse (zero upper
//   part) to Ainv (ld).  A non-positive or NaN pivot sets *info = row0 + j + 1
//   if *info is still 0 (the 1-based global pivot; blocks run in order, so the
//   first failure wins).
__global__ __launch_bounds__(256) void leaf_potrf_trtri_kernel(double* __restrict__ A, double* __restrict__ Ainv,
                                                               int64_t ld, int row0, int* __restrict__ info) {
  constexpr int B = NB_LEAF;
  constexpr int SC = 2 * B;   // column stride of lt (room for the dummy rows)
  constexpr int S = B + 1;
  constexpr int QR = B / 4;   // register rows per thread
  static_assert(B == 64, "one lane per column of the block");
  __shared__ double lt[B * SC];   // column j of the factor: lt[j * SC + i] = L[i][j]
  __shared__ double rs[B];        // 1 / sqrt(pivot j) = 1 / L[j][j]
  __shared__ double xo[B * S];    // inverse, column-major staging for the store
  const int t = threadIdx.x;
  const int kc = t & (B - 1);
  const int r0 = t >> 6;
  double a[QR];
#pragma unroll
  for (int q = 0; q < QR; ++q) {
    const int i = kc + r0 + 4 * q;
    a[q] = (i < B) ? A[(int64_t)i + (int64_t)kc * ld] : 0.0;
  }
  for (int j = 0; j < B; ++j) {
    double* cj = lt + j * SC;
    if (kc == j) {
#pragma unroll
      for (int q = 0; q < QR; ++q) cj[kc + r0 + 4 * q] = a[q];
    }
    __syncthreads();
    const double lk = (kc > j) ? cj[kc] * fast_rcp(cj[j]) : 0.0;
#pragma unroll
    for (int q = 0; q < QR; ++q) a[q] -= cj[kc + r0 + 4 * q] * lk;
  }
  if (t == 0) {
    for (int j = 0; j < B; ++j) {
      if (!(lt[j * SC + j] > 0.0)) {
        if (*info == 0) *info = row0 + j + 1;
        break;
      }
    }
  }
  if (t < B) rs[t] = 1.0 / sqrt(lt[t * SC + t]);
  __syncthreads();
  for (int idx = t; idx < B * B; idx += blockDim.x) {
    const int i = idx % B, j = idx / B;
    if (i > j) lt[j * SC + i] *= rs[j];
    else if (i == j) lt[j * SC + i] = sqrt(lt[j * SC + i]);
  }
  __syncthreads();
  for (int idx = t; idx < B * B; idx += blockDim.x) {
    const int i = idx % B, k = idx / B;
    A[(int64_t)i + (int64_t)k * ld] = (i >= k) ? lt[k * SC + i] : 0.0;
  }
  if (t < B) {
    // Sliding window: before step k, w[d] holds entry k + d of the lane's
    // column (entries past the block are dummies, never stored).  A runtime
    // loop over k keeps the code small: straight-line code run once would be
    // bound by instruction fetch.
    const int jj = t;
    double w[B];
#pragma unroll
    for (int d = 0; d < B; ++d) w[d] = (d == jj) ? 1.0 : 0.0;
    for (int k = 0; k < B; ++k) {
      const double xk = w[0] * rs[k];
      xo[k + jj * S] = xk;
      const double* lk = lt + k * SC + k;   // L[k + d][k] for d >= 1 (rows past the block: dummies)
#pragma unroll
      for (int d = 1; d < B; ++d) w[d - 1] = w[d] - lk[d] * xk;
      w[B - 1] = 0.0;
    }
  }
  __syncthreads();
  for (int idx = t; idx < B * B; idx += blockDim.x) {
    const int i = idx % B, k = idx / B;
    Ainv[(int64_t)i + (int64_t)k * ld] = xo[i + k * S];
  }
}

// G[j][k] = sum_r W[r][j] * W[r][k] for j >= k (p x p, both triangles written);
// one workgroup per (j, k) pair, fixed-order tree reduction.
__global__ __launch_bounds__(256) void gram_kernel(const double* __restrict__ W, int N, int p, double* __restrict__ G) {
  __shared__ double red[256];
  int pair = blockIdx.x;
  int j = 0;
  while ((j + 1) * (j + 2) / 2 <= pair) ++j;
  int k = pair - j * (j + 1) / 2;
  double s = 0.0;
  const double* wj = W + (int64_t)j * N;
  const double* wk = W + (int64_t)k * N;
  for (int r = threadIdx.x; r < N; r += 256) s += wj[r] * wk[r];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    G[j + k * p] = red[0];
    G[k + j * p] = red[0];
  }
}

// Layout of the small per-study constants used by the per-SNP solve.
//   Lt  : q x q lower Cholesky factor of S_TL (q = p - 1), column-major
//   zT  : q      Lt^-1 r~_T
//   c   : 1      y~^T y~
//   qres: 1      c - zT^T zT   (residual of y~ on X~_L)
struct SmallLayout {
  static __host__ __device__ int Lt(int) { return 0; }
  static __host__ __device__ int zT(int p) { return (p - 1) * (p - 1); }
  static __host__ __device__ int c(int p) { return (p - 1) * (p - 1) + (p - 1); }
  static __host__ __device__ int qres(int p) { return c(p) + 1; }
  static __host__ __device__ int size(int p) { return qres(p) + 1; }
};

// Single-thread factorization of S_TL = G[0:q, 0:q] and the hoisted
// right-hand side.  Sets *info_rank = j + 1 for the first non-positive pivot.
__global__ void small_factor_kernel(const double* __restrict__ G, int p, double* __restrict__ small,
                                    int* __restrict__ info_rank) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int q = p - 1;
  double* Lt = small + SmallLayout::Lt(p);
  double* zT = small + SmallLayout::zT(p);
  for (int j = 0; j < q; ++j) {
    double d = G[j + j * p];
    for (int k = 0; k < j; ++k) d -= Lt[j + k * q] * Lt[j + k * q];
    if (!(d > 0.0) && *info_rank == 0) *info_rank = j + 1;
    d = sqrt(d);
    Lt[j + j * q] = d;
    for (int i = j + 1; i < q; ++i) {
      double s = G[i + j * p];
      for (int k = 0; k < j; ++k) s -= Lt[i + k * q] * Lt[j + k * q];
      Lt[i + j * q] = s / d;
    }
    for (int i = 0; i < j; ++i) Lt[i + j * q] = 0.0;
  }
  double zz = 0.0;
  for (int j = 0; j < q; ++j) {
    double s = G[j + q * p];
    for (int k = 0; k < j; ++k) s -= Lt[j + k * q] * zT[k];
    zT[j] = s / Lt[j + j * q];
    zz += zT[j] * zT[j];
  }
  const double c = G[q + q * p];
  small[SmallLayout::c(p)] = c;
  small[SmallLayout::qres(p)] = c - zz;
}

}  // namespace gls
