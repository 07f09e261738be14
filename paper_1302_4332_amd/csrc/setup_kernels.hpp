// Setup-phase kernels: forming M, the in-LDS factorization and inversion of
// the diagonal blocks, packing, and the small Gram matrix of [X~_L | y~].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gls {

// Leaf (diagonal block) size of the blocked Cholesky / inversion.
constexpr int NB_LEAF = 128;

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

// N x N zeros with ones on the diagonal from row r0 on.
__global__ void identity_tail_kernel(double* __restrict__ p, int N, int r0) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * N;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % N), j = (int)(idx / N);
    p[idx] = (i == j && i >= r0) ? 1.0 : 0.0;
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

// dst[k + j ld_dst] = src[k + j ld_src] for k < n, 0 for n <= k < rows, over
// cols columns: a block copied into a buffer whose rows past n are zero.
__global__ void pad_copy_kernel(double* __restrict__ dst, int64_t ld_dst, const double* __restrict__ src,
                                int64_t ld_src, int n, int rows, int cols) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)rows * cols;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % rows);
    const int j = (int)(idx / rows);
    dst[(int64_t)i + (int64_t)j * ld_dst] = (i < n) ? src[(int64_t)i + (int64_t)j * ld_src] : 0.0;
  }
}

// dst (cols x rows, ld_dst) <- src^T for src (rows x cols, ld_src), through
// 32 x 32 LDS tiles so that both the reads and the writes are column runs.
__global__ __launch_bounds__(256) void transpose_kernel(double* __restrict__ dst, int64_t ld_dst,
                                                        const double* __restrict__ src, int64_t ld_src, int rows,
                                                        int cols) {
  __shared__ double tile[32][33];
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  double v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + tx, c = c0 + ty + 8 * q;
    v[q] = (r < rows && c < cols) ? src[(int64_t)r + (int64_t)c * ld_src] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) tile[ty + 8 * q][tx] = v[q];   // tile[c - c0][r - r0]
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = c0 + tx, r = r0 + ty + 8 * q;               // dst row c, column r
    if (r < rows && c < cols) dst[(int64_t)c + (int64_t)r * ld_dst] = tile[tx][ty + 8 * q];
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

// W = L^-1 V for the thin covariate block V = [X_L | y] (N x P, ld N) and the
// lower-triangular inverse factor (N x N, ld N): a matrix-vector-shaped
// product bound by reading L^-1's lower triangle once, so it runs split over
// k on the vector units.  Workgroup (r, s) takes rows 64 r .. 64 r + 63 and
// k in [TA_KC s, TA_KC s + TA_KC), clipped to k <= row; each wave walks every
// fourth k, so a wave's loads are one 512-byte column segment.  Partial sums
// go to part[s] (N x P, ld N); chunks entirely above a row tile are skipped,
// and tri_apply_sum_kernel adds, in chunk order, exactly the chunks that
// reach each row tile.
constexpr int TA_KC = 256;

template <int P>
__global__ __launch_bounds__(256) void tri_apply_partial_kernel(const double* __restrict__ Li, int N,
                                                                const double* __restrict__ V,
                                                                double* __restrict__ part) {
  __shared__ double v[TA_KC * P];       // v[kk * P + j] = V[k0 + kk][j]; then the group sums
  const int i0 = blockIdx.x * 64, s = blockIdx.y, k0 = s * TA_KC;
  if (k0 > i0 + 63) return;
  const int t = threadIdx.x, r = t & 63, g = t >> 6;
  static_assert(TA_KC == 256, "one staged k per thread and column");
  {
    double x[P];
#pragma unroll
    for (int j = 0; j < P; ++j) x[j] = (k0 + t < N) ? V[(int64_t)(k0 + t) + (int64_t)j * N] : 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) v[t * P + j] = x[j];
  }
  __syncthreads();
  const int i = i0 + r;
  const int kend = min(min(k0 + TA_KC, i0 + 64), N);
  double acc[P];
#pragma unroll
  for (int j = 0; j < P; ++j) acc[j] = 0.0;
  // eight loads in flight per thread, then their products
  for (int kb = k0 + g; kb < kend; kb += 32) {
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = kb + 4 * u;
      a[u] = (k < kend && k <= i) ? Li[(int64_t)i + (int64_t)k * N] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int kk = kb + 4 * u - k0;
      if (kb + 4 * u < kend) {
#pragma unroll
        for (int j = 0; j < P; ++j) acc[j] = fma(a[u], v[kk * P + j], acc[j]);
      }
    }
  }
  __syncthreads();   // v is reused for the four groups' sums
#pragma unroll
  for (int j = 0; j < P; ++j) v[(g * 64 + r) * P + j] = acc[j];
  __syncthreads();
  if (g == 0) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const double x = ((acc[j] + v[(64 + r) * P + j]) + v[(128 + r) * P + j]) + v[(192 + r) * P + j];
      part[(int64_t)s * N * P + (int64_t)j * N + i] = x;
    }
  }
}

__global__ void tri_apply_sum_kernel(const double* __restrict__ part, int N, int P, double* __restrict__ W) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * P;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % N);
    const int last = (i / 64 * 64 + 63) / TA_KC;   // chunks s <= last reach row tile i / 64
    double x = 0.0;
    for (int s = 0; s <= last; ++s) x += part[(int64_t)s * total + idx];
    W[idx] = x;
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

// One diagonal block of the blocked factorization, entirely on chip.
//
// The NB_LEAF x NB_LEAF block (128 x 128 doubles, 129 KB with the padded
// column stride) sits in LDS and is processed as 8 x 8 blocks of 16 x 16:
//   Cholesky, panel by panel (16 columns at a time):
//     - one wave factors the 16 x 16 diagonal block (lane i owns row i; the
//       column of each step is exchanged through LDS within the wave);
//     - every row below solves against it (one thread per row, forward
//       substitution with the stored 1 / L[k][k]);
//     - the trailing lower blocks take the rank-16 update on
//       v_mfma_f64_16x16x4f64; wave 0 updates the next diagonal block first
//       and factors it while the other waves finish the update.
//   Inverse, in place: the 16 x 16 diagonal inverses (one per wave), then
//   block columns from right to left,
//     X[i][j] = -(sum_{k=j+1..i} X[i][k] L[k][j]) X[j][j]   (i > j),
//   again on 16 x 16 matrix-core products.
// Block columns of the factor and of the inverse are written to A and Ainv
// (ld, zeros above the diagonal) as soon as they are final.  A non-positive or
// NaN pivot sets *info = row0 + j + 1 if *info is still 0 (the 1-based global
// pivot; blocks run in order, so the first failure wins).

typedef double l4_t __attribute__((ext_vector_type(4)));

constexpr int LT = 16;                 // inner block size
constexpr int LNB = NB_LEAF / LT;      // inner blocks per side
constexpr int LD = NB_LEAF + 1;        // LDS column stride: odd, so 16 lanes reading along a row hit 16 banks
static_assert(NB_LEAF % LT == 0 && LNB == 8, "the inverse's scratch blocks assume 8 x 8 inner blocks");

__device__ __forceinline__ double* leaf_blk(double* S, int bi, int bj) { return S + (LT * bj) * LD + LT * bi; }

// acc += op(A) op(B) for 16 x 16 blocks on v_mfma_f64_16x16x4f64.  A element
// (r, k) at pa[r * ars + k * aks], B element (k, c) at pb[k * bks + c * bcs];
// neg negates A.  Lane l supplies A[l % 16][4 s + l / 16] and
// B[4 s + l / 16][l % 16]; the accumulator holds D[l / 16 + 4 t][l % 16].
__device__ __forceinline__ void leaf_mma16(l4_t& acc, const double* pa, int ars, int aks, const double* pb, int bks,
                                           int bcs, bool neg, int lane) {
  const int r = lane & 15, q = lane >> 4;
  double a[4], b[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    a[s] = pa[r * ars + (4 * s + q) * aks];
    b[s] = pb[(4 * s + q) * bks + r * bcs];
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(neg ? -a[s] : a[s], b[s], acc, 0, 0, 0);
}
__device__ __forceinline__ l4_t leaf_ld_acc(const double* p, int lane) {
  const int c = lane & 15, q = lane >> 4;
  return l4_t{p[q + c * LD], p[q + 4 + c * LD], p[q + 8 + c * LD], p[q + 12 + c * LD]};
}
__device__ __forceinline__ void leaf_st_acc(double* p, l4_t v, int lane) {
  const int c = lane & 15, q = lane >> 4;
  p[q + c * LD] = v[0];
  p[q + 4 + c * LD] = v[1];
  p[q + 8 + c * LD] = v[2];
  p[q + 12 + c * LD] = v[3];
}

// One wave factors the 16 x 16 diagonal block of panel p in place.  Lane i
// (< 16) owns row i; at step j the column goes through LDS (the operations of
// one wave on LDS complete in order; the empty asm statements with a memory
// clobber stop the compiler from carrying values across the exchange).
// Stores 1 / L[k][k] in rd[16 p + k]; returns the first non-positive pivot
// (1-based within the leaf) or 0.
__device__ __forceinline__ int leaf_factor16(double* S, int p, double* col, double* rd, int lane) {
  const int i = lane & 15;
  double* D = leaf_blk(S, p, p);
  double w[LT];
#pragma unroll
  for (int k = 0; k < LT; ++k) w[k] = D[i + k * LD];
  int bad = 0;
#pragma unroll
  for (int j = 0; j < LT; ++j) {
    if (lane < LT) col[i] = w[j];
    asm volatile("" ::: "memory");
    double c[LT];
#pragma unroll
    for (int k = j; k < LT; ++k) c[k] = col[k];
    asm volatile("" ::: "memory");
    const double d = c[j];
    if (bad == 0 && !(d > 0.0)) bad = LT * p + j + 1;
    const double sd = sqrt(d);
    const double r = fast_rcp(sd);
    const double lr = (i < j) ? 0.0 : w[j] * r * r;   // L[i][j] / L[j][j]
    w[j] = (i < j) ? 0.0 : ((i == j) ? sd : w[j] * r);
#pragma unroll
    for (int k = j + 1; k < LT; ++k) w[k] -= lr * c[k];
    if (lane == 0) rd[LT * p + j] = r;
  }
  if (lane < LT) {
#pragma unroll
    for (int k = 0; k < LT; ++k) D[i + k * LD] = w[k];
  }
  return bad;
}

// Block column q (columns 16 q .. 16 q + 15) of the lower triangle of S to G (ld), zeros above the diagonal.
__device__ __forceinline__ void leaf_store_col(const double* S, double* G, int64_t ld, int q, int t) {
  for (int idx = t; idx < NB_LEAF * LT; idx += 512) {
    const int r = idx % NB_LEAF, c = LT * q + idx / NB_LEAF;
    G[(int64_t)r + (int64_t)c * ld] = (r >= c) ? S[r + c * LD] : 0.0;
  }
}

__global__ __launch_bounds__(512) void leaf_potrf_trtri_kernel(double* __restrict__ A, double* __restrict__ Ainv,
                                                               int64_t ld, int row0, int* __restrict__ info) {
  __shared__ __align__(16) double S[NB_LEAF * LD];
  __shared__ double rd[NB_LEAF];   // 1 / L[k][k]
  __shared__ double colw[LT];      // wave 0's column exchange
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  {  // all loads first, then the LDS stores: one memory latency instead of one per element
    constexpr int PER = NB_LEAF * NB_LEAF / 512;
    static_assert(512 % NB_LEAF == 0, "a thread keeps its row");
    const int r = t % NB_LEAF, c0 = t / NB_LEAF;
    double v[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) v[q] = A[(int64_t)r + (int64_t)(c0 + q * (512 / NB_LEAF)) * ld];
#pragma unroll
    for (int q = 0; q < PER; ++q) S[r + (c0 + q * (512 / NB_LEAF)) * LD] = v[q];
  }
  __syncthreads();
  int bad = 0;   // meaningful in wave 0
  if (wave == 0) bad = leaf_factor16(S, 0, colw, rd, lane);
  __syncthreads();
  for (int p = 0; p < LNB; ++p) {
    // rows below the diagonal block, one thread each:
    //   L[r][16p + k] = (A[r][16p + k] - sum_{m<k} L[r][16p + m] L[16p + k][16p + m]) / L[16p + k][16p + k]
    {
      const int r = LT * (p + 1) + t;
      if (r < NB_LEAF) {
        const double* D = leaf_blk(S, p, p);
        double* Pr = S + (LT * p) * LD + r;
        double x[LT];
#pragma unroll
        for (int k = 0; k < LT; ++k) x[k] = Pr[k * LD];
#pragma unroll
        for (int k = 0; k < LT; ++k) {
          x[k] *= rd[LT * p + k];
#pragma unroll
          for (int m = k + 1; m < LT; ++m) x[m] -= x[k] * D[m + k * LD];
        }
#pragma unroll
        for (int k = 0; k < LT; ++k) Pr[k * LD] = x[k];
      }
    }
    __syncthreads();
    leaf_store_col(S, A, ld, p, t);   // block column p of the factor is final
    if (p == LNB - 1) break;
    // trailing update A[i][c] -= L[i][p] L[c][p]^T for p < c <= i.  Task 0 is
    // the next diagonal block: wave 0 updates it and factors it at once; waves
    // 1..7 share the other tasks.
    {
      const int nb = LNB - 1 - p;
      const int tasks = nb * (nb + 1) / 2;
      for (int task = wave; task < tasks; task += (wave == 0) ? tasks : LNB - 1) {
        int c = 0, rem = task;
        while (rem >= nb - c) {
          rem -= nb - c;
          ++c;
        }
        const int bc = p + 1 + c, bi = bc + rem;
        double* C = leaf_blk(S, bi, bc);
        l4_t acc = leaf_ld_acc(C, lane);
        leaf_mma16(acc, leaf_blk(S, bi, p), 1, LD, leaf_blk(S, bc, p), LD, 1, true, lane);
        leaf_st_acc(C, acc, lane);
      }
      if (wave == 0) {
        const int b = leaf_factor16(S, p + 1, colw, rd, lane);
        if (bad == 0) bad = b;
      }
    }
    __syncthreads();
  }
  if (wave == 0 && lane == 0 && bad != 0 && *info == 0) *info = row0 + bad;
  __syncthreads();
  // the 16 x 16 diagonal inverses, in place: wave w takes block w, lane c < 16 forms column c
  {
    const int c = lane & 15;
    double* D = leaf_blk(S, wave, wave);
    double x[LT];
#pragma unroll
    for (int k = 0; k < LT; ++k) x[k] = (k == c) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < LT; ++k) {
      x[k] *= rd[LT * wave + k];
#pragma unroll
      for (int m = k + 1; m < LT; ++m) x[m] -= D[m + k * LD] * x[k];
    }
    if (lane < LT) {
#pragma unroll
      for (int k = 0; k < LT; ++k) D[k + c * LD] = x[k];
    }
  }
  __syncthreads();
  leaf_store_col(S, Ainv, ld, LNB - 1, t);
  // block columns of the inverse, right to left; T goes to a scratch block of
  // the strictly upper triangle (never read as data)
  for (int j = LNB - 2; j >= 0; --j) {
    const int bi = j + 1 + wave;
    double* T = (wave < LNB - 1) ? leaf_blk(S, wave, LNB - 1) : leaf_blk(S, 0, LNB - 2);
    l4_t acc = {0.0, 0.0, 0.0, 0.0};
    if (bi < LNB) {
      for (int k = j + 1; k <= bi; ++k) leaf_mma16(acc, leaf_blk(S, bi, k), 1, LD, leaf_blk(S, k, j), 1, LD, false, lane);
      leaf_st_acc(T, acc, lane);
    }
    __syncthreads();
    if (bi < LNB) {
      acc = l4_t{0.0, 0.0, 0.0, 0.0};
      leaf_mma16(acc, T, 1, LD, leaf_blk(S, j, j), 1, LD, true, lane);
      leaf_st_acc(leaf_blk(S, bi, j), acc, lane);
    }
    __syncthreads();
    leaf_store_col(S, Ainv, ld, j, t);   // block column j of the inverse is final
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

// Relative pivot floor of the covariate factorization: X_L counts as rank
// deficient when a squared pivot of S_TL falls to 2^-40 of its diagonal entry
// or below (exactly collinear covariates leave a rounding residual of either
// sign, about 1e-16 of it).
constexpr double RANK_REL = 9.094947017729282e-13;  // 2^-40

// Single-thread factorization of S_TL = G[0:q, 0:q] and the hoisted
// right-hand side.  Sets *info_rank = j + 1 for the first pivot at or below
// the floor.
__global__ void small_factor_kernel(const double* __restrict__ G, int p, double* __restrict__ small,
                                    int* __restrict__ info_rank) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int q = p - 1;
  double* Lt = small + SmallLayout::Lt(p);
  double* zT = small + SmallLayout::zT(p);
  for (int j = 0; j < q; ++j) {
    double d = G[j + j * p];
    for (int k = 0; k < j; ++k) d -= Lt[j + k * q] * Lt[j + k * q];
    if (!(d > RANK_REL * G[j + j * p]) && *info_rank == 0) *info_rank = j + 1;
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
