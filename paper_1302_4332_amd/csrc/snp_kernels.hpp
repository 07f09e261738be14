// Per-SNP kernels: the products S_BL,i = x~_i^T X~_L, r~_B,i = x~_i^T y~,
// S_BR,i = x~_i^T x~_i (Sec. 2.1, the S-loop of the structured algorithm) and
// the p x p SPD solve b_i = S_i^-1 r~_i (posv), done as a Cholesky of S_i
// whose leading (p-1) x (p-1) block, the factor of S_TL, is shared by every
// SNP and was factored once at setup.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "setup_kernels.hpp"

namespace gls {

// S_i is singular when its last squared pivot is not above this fraction of S_BR,i.
constexpr double SINGULAR_REL = 9.094947017729282e-13;  // 2^-40

constexpr int SNP_PER_WAVE = 4;
constexpr int SNP_WAVES = 4;
constexpr int SNP_PER_WG = SNP_PER_WAVE * SNP_WAVES;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The p x p Cholesky solve of one SNP from its reduced products.
//   s[0..q-1] = S_BL,i,  rB = r~_B,i,  sbr = S_BR,i
template <int P>
__device__ __forceinline__ void snp_solve(const double* __restrict__ small, const double* s, double rB, double sbr,
                                          int n, double* __restrict__ bout, double* sigma2, double* v, int* status) {
  constexpr int Q = P - 1;
  const double* Lt = small + SmallLayout::Lt(P);
  const double* zT = small + SmallLayout::zT(P);
  const double qres = small[SmallLayout::qres(P)];
  double l[Q > 0 ? Q : 1];
  double d2 = sbr;
  double lz = 0.0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    double t = s[j];
#pragma unroll
    for (int k = 0; k < j; ++k) t -= Lt[j + k * Q] * l[k];
    l[j] = t / Lt[j + j * Q];
    d2 -= l[j] * l[j];
    lz += l[j] * zT[j];
  }
  if (!(d2 > SINGULAR_REL * sbr)) {
    const double nan = __builtin_nan("");
#pragma unroll
    for (int j = 0; j < P; ++j) bout[j] = nan;
    *sigma2 = nan;
    *v = nan;
    *status = 1;
    return;
  }
  const double d = sqrt(d2);
  const double zp = (rB - lz) / d;
  const double bp = zp / d;
  double bt[Q > 0 ? Q : 1];
#pragma unroll
  for (int j = Q - 1; j >= 0; --j) {
    double t = zT[j] - l[j] * bp;
#pragma unroll
    for (int k = j + 1; k < Q; ++k) t -= Lt[k + j * Q] * bt[k];
    bt[j] = t / Lt[j + j * Q];
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) bout[j] = bt[j];
  bout[Q] = bp;
  *sigma2 = (qres - zp * zp) / (double)(n - P);
  *v = 1.0 / d2;
  *status = 0;
}

// One wave per SNP_PER_WAVE SNP columns of Xt (rows 0..n-1 read, ld ldx).
// W = [X~_L | y~] (N x P, ld N).  Lane-strided row sums over the n sample
// rows (the padding rows of W are zero, those of Xt need not be written),
// then a fixed butterfly reduction: every SNP's arithmetic depends only on
// its own column.
template <int P>
__global__ __launch_bounds__(64 * SNP_WAVES)
void snp_reduce_solve_kernel(const double* __restrict__ Xt, int64_t ldx, int N, int mb,
                             const double* __restrict__ W, const double* __restrict__ small, int n,
                             double* __restrict__ b, int64_t ldb, double* __restrict__ sigma2,
                             double* __restrict__ v, int* __restrict__ status) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int c0 = (blockIdx.x * SNP_WAVES + wave) * SNP_PER_WAVE;
  if (c0 >= mb) return;
  double acc[SNP_PER_WAVE][P + 1];
#pragma unroll
  for (int s = 0; s < SNP_PER_WAVE; ++s)
#pragma unroll
    for (int j = 0; j <= P; ++j) acc[s][j] = 0.0;
  const double* xs[SNP_PER_WAVE];
#pragma unroll
  for (int s = 0; s < SNP_PER_WAVE; ++s) {
    int c = c0 + s < mb ? c0 + s : c0;   // clamp: a repeated column, result discarded
    xs[s] = Xt + (int64_t)c * ldx;
  }
  for (int r = lane; r < n; r += 64) {
    double w[P];
#pragma unroll
    for (int j = 0; j < P; ++j) w[j] = W[r + (int64_t)j * N];
#pragma unroll
    for (int s = 0; s < SNP_PER_WAVE; ++s) {
      const double x = xs[s][r];
#pragma unroll
      for (int j = 0; j < P; ++j) acc[s][j] += x * w[j];
      acc[s][P] += x * x;
    }
  }
#pragma unroll
  for (int s = 0; s < SNP_PER_WAVE; ++s)
#pragma unroll
    for (int j = 0; j <= P; ++j) acc[s][j] = wave_sum(acc[s][j]);
  if (lane < SNP_PER_WAVE && c0 + lane < mb) {
    const int c = c0 + lane;
    double sv[P + 1];
    // select this lane's SNP without dynamic register indexing
#pragma unroll
    for (int j = 0; j <= P; ++j) {
      double t = acc[0][j];
#pragma unroll
      for (int s = 1; s < SNP_PER_WAVE; ++s) t = (lane == s) ? acc[s][j] : t;
      sv[j] = t;
    }
    double bo[P];
    double s2, vv;
    int st;
    snp_solve<P>(small, sv, sv[P - 1], sv[P], n, bo, &s2, &vv, &st);
#pragma unroll
    for (int j = 0; j < P; ++j) b[(int64_t)c * ldb + j] = bo[j];
    sigma2[c] = s2;
    v[c] = vv;
    status[c] = st;
  }
}

// The per-SNP solve from row-tile partial sums (the product's fused epilogue):
// part[(t (P + 1) + q) mb + j] for row tiles t < Mt holds SNP j's sums over
// tile t of x~ times [X~_L | y~] column q (q < P) and of x~^2 (q = P).  One
// thread per SNP adds the tiles in order, then solves as snp_reduce_solve_kernel.
template <int P>
__global__ __launch_bounds__(256) void snp_partials_solve_kernel(const double* __restrict__ part, int Mt, int mb,
                                                                  const double* __restrict__ small, int n,
                                                                  double* __restrict__ b, int64_t ldb,
                                                                  double* __restrict__ sigma2, double* __restrict__ v,
                                                                  int* __restrict__ status) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= mb) return;
  double sv[P + 1];
#pragma unroll
  for (int q = 0; q <= P; ++q) sv[q] = 0.0;
  for (int t = 0; t < Mt; ++t) {
    const double* pt = part + (int64_t)t * (P + 1) * mb + j;
#pragma unroll
    for (int q = 0; q <= P; ++q) sv[q] += pt[(int64_t)q * mb];
  }
  double bo[P];
  double s2, vv;
  int st;
  snp_solve<P>(small, sv, sv[P - 1], sv[P], n, bo, &s2, &vv, &st);
#pragma unroll
  for (int q = 0; q < P; ++q) b[(int64_t)j * ldb + q] = bo[q];
  sigma2[j] = s2;
  v[j] = vv;
  status[j] = st;
}

}  // namespace gls
