// Kernels of the hand-written adjoint (reverse mode) of the GLS sequence.
//
// Per SNP, with S = S_i, r = r~_i, b = S^-1 r, sigma2 = (c - b^T r)/(n - p),
// v = (S^-1)_pp and cotangents (bbar, s2bar, vbar):
//     lambda = S^-1 bbar,   u = S^-1 e_p,   kappa = s2bar / (n - p)
//     rbar = lambda - 2 kappa b,            cbar = kappa
//     Sbar = -(lambda b^T + b lambda^T)/2 + kappa b b^T - vbar u u^T
// S_i = [[S_TL, s], [s^T, S_BR]] with s = X~_L^T x~, S_BR = x~^T x~ and
// r~_B = y~^T x~, so
//     x~bar = X~_L (2 Sbar[p, 0:q]) + y~ rbar[p] + 2 Sbar[p, p] x~,
// while Sbar[0:q, 0:q], rbar[0:q] and cbar accumulate into the adjoints of
// the study-wide S_TL, r~_T and y~^T y~.  S_i^-1 is applied with the same
// blocked Cholesky the forward solve uses (leading factor of S_TL shared).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "setup_kernels.hpp"
#include "snp_kernels.hpp"

namespace gls {

// Shared-term contributions per SNP: lower triangle of Sbar[0:q,0:q]
// (row-major, (i, j) with j <= i), then rbar[0:q], then cbar.
__host__ __device__ constexpr int adj_nc(int p) { return (p - 1) * p / 2 + (p - 1) + 1; }

template <int P>
__global__ __launch_bounds__(64 * SNP_WAVES)
void snp_adjoint_kernel(double* __restrict__ Xt, int64_t ldx, int N, int mb, const double* __restrict__ W,
                        const double* __restrict__ small, int n, const double* __restrict__ bbar, int64_t ldbb,
                        const double* __restrict__ s2bar, const double* __restrict__ vbar,
                        double* __restrict__ Cbar, double* __restrict__ ebar, double* __restrict__ contrib) {
  constexpr int Q = P - 1;
  constexpr int NC = adj_nc(P);
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
    int c = c0 + s < mb ? c0 + s : c0;
    xs[s] = Xt + (int64_t)c * ldx;
  }
  for (int r = lane; r < N; r += 64) {
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
  if (lane >= SNP_PER_WAVE || c0 + lane >= mb) return;
  const int c = c0 + lane;
  double sv[P + 1];
#pragma unroll
  for (int j = 0; j <= P; ++j) {
    double t = acc[0][j];
#pragma unroll
    for (int s = 1; s < SNP_PER_WAVE; ++s) t = (lane == s) ? acc[s][j] : t;
    sv[j] = t;
  }
  const double* Lt = small + SmallLayout::Lt(P);
  const double* zT = small + SmallLayout::zT(P);
  const double qres = small[SmallLayout::qres(P)];
  const double sbr = sv[P], rB = sv[P - 1];
  double* cb = Cbar + (int64_t)c * P;
  double* ct = contrib + (int64_t)c * NC;
  // forward quantities
  double l[Q > 0 ? Q : 1];
  double d2 = sbr, lz = 0.0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    double t = sv[j];
#pragma unroll
    for (int k = 0; k < j; ++k) t -= Lt[j + k * Q] * l[k];
    l[j] = t / Lt[j + j * Q];
    d2 -= l[j] * l[j];
    lz += l[j] * zT[j];
  }
  const double bb_p = bbar[(int64_t)c * ldbb + (P - 1)];
  if (!(d2 > SINGULAR_REL * sbr)) {
    // singular S_i (status 1, NaN outputs): no contribution.  Its whitened
    // column may hold NaN (a NaN sample), and 0 * NaN would reach the
    // study-wide sums through the later products with X~, so the column is
    // zeroed; the wave's reads of it are complete (they fed the sums above).
#pragma unroll
    for (int j = 0; j < P; ++j) cb[j] = 0.0;
    ebar[c] = 0.0;
    for (int t = 0; t < NC; ++t) ct[t] = 0.0;
    double* col = Xt + (int64_t)c * ldx;
    for (int r = 0; r < N; ++r) col[r] = 0.0;
    return;
  }
  const double d = sqrt(d2);
  const double zp = (rB - lz) / d;
  double b[P];
  b[Q] = zp / d;
#pragma unroll
  for (int j = Q - 1; j >= 0; --j) {
    double t = zT[j] - l[j] * b[Q];
#pragma unroll
    for (int k = j + 1; k < Q; ++k) t -= Lt[k + j * Q] * b[k];
    b[j] = t / Lt[j + j * Q];
  }
  const double vv = 1.0 / d2;
  // lambda = S^-1 bbar
  double lam[P];
  {
    double zt[Q > 0 ? Q : 1];
    double lzt = 0.0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      double t = bbar[(int64_t)c * ldbb + j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= Lt[j + k * Q] * zt[k];
      zt[j] = t / Lt[j + j * Q];
      lzt += l[j] * zt[j];
    }
    lam[Q] = (bb_p - lzt) / d2;
#pragma unroll
    for (int j = Q - 1; j >= 0; --j) {
      double t = zt[j] - l[j] * lam[Q];
#pragma unroll
      for (int k = j + 1; k < Q; ++k) t -= Lt[k + j * Q] * lam[k];
      lam[j] = t / Lt[j + j * Q];
    }
  }
  // u = S^-1 e_p:  u_p = v,  u_T = -Lt^-T l v
  double u[P];
  u[Q] = vv;
#pragma unroll
  for (int j = Q - 1; j >= 0; --j) {
    double t = -l[j] * vv;
#pragma unroll
    for (int k = j + 1; k < Q; ++k) t -= Lt[k + j * Q] * u[k];
    u[j] = t / Lt[j + j * Q];
  }
  (void)qres;
  const double kappa = s2bar[c] / (double)(n - P);
  const double vb = vbar[c];
  auto sbar = [&](int j, int k) {
    return -0.5 * (lam[j] * b[k] + b[j] * lam[k]) + kappa * b[j] * b[k] - vb * u[j] * u[k];
  };
#pragma unroll
  for (int j = 0; j < Q; ++j) cb[j] = 2.0 * sbar(Q, j);
  cb[Q] = lam[Q] - 2.0 * kappa * b[Q];
  ebar[c] = 2.0 * sbar(Q, Q);
  int t = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) ct[t++] = sbar(i, j);
#pragma unroll
  for (int j = 0; j < Q; ++j) ct[t++] = lam[j] - 2.0 * kappa * b[j];
  ct[t] = kappa;
}

// Study-wide adjoint sums add the block's SNPs in groups of 16 consecutive
// SNPs: each group is summed in SNP order, and the group sums are added to the
// running value in group order.  With blocks that start at multiples of 16
// the groups and their order are the same whatever the block widths, so these
// sums are bitwise independent of how SNPs are grouped into blocks.
constexpr int ADJ_GROUP = 16;
constexpr int ADJ_GROUPS_PER_PASS = 1024;   // group sums held in LDS per pass of reduce_contrib_kernel

// acc[t] += the block's contributions contrib[t + j nc], j < mb, one
// workgroup per term: the group sums in parallel, then one thread adds them.
__global__ __launch_bounds__(256) void reduce_contrib_kernel(const double* __restrict__ contrib, int nc, int mb,
                                                             double* __restrict__ acc) {
  __shared__ double gs[ADJ_GROUPS_PER_PASS];
  const int t = blockIdx.x;
  const int groups = (mb + ADJ_GROUP - 1) / ADJ_GROUP;
  double run = acc[t];   // meaningful in thread 0
  for (int g0 = 0; g0 < groups; g0 += ADJ_GROUPS_PER_PASS) {
    const int gn = min(ADJ_GROUPS_PER_PASS, groups - g0);
    for (int g = threadIdx.x; g < gn; g += 256) {
      const int j0 = (g0 + g) * ADJ_GROUP, j1 = min(mb, j0 + ADJ_GROUP);
      double s = 0.0;
      for (int j = j0; j < j1; ++j) s += contrib[t + (int64_t)j * nc];
      gs[g] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0)
      for (int g = 0; g < gn; ++g) run += gs[g];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[t] = run;
}

// Wbar += X~ Cbar^T (N x P; X~ N x mb, ld N; Cbar P x mb) in groups of 16
// SNPs as above, in two steps.  wbar_group_kernel forms the sums of groups
// g0 .. g0 + gn - 1, one thread per (row r, group):
//   part[(g P + t) N + r] = sum over the group's SNPs j, in order, of X~[r, j] Cbar[t, j]
// (rows coalesced, Cbar broadcast); wbar_add_kernel then adds them to Wbar in
// group order, one thread per entry of Wbar.
template <int P>
__global__ __launch_bounds__(256) void wbar_group_kernel(const double* __restrict__ Xt, int N, int mb, int g0,
                                                         const double* __restrict__ Cbar, double* __restrict__ part) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int g = blockIdx.y;
  if (r >= N) return;
  const int j0 = (g0 + g) * ADJ_GROUP, j1 = min(mb, j0 + ADJ_GROUP);
  double s[P];
#pragma unroll
  for (int t = 0; t < P; ++t) s[t] = 0.0;
  for (int j = j0; j < j1; ++j) {
    const double x = Xt[r + (int64_t)j * N];
#pragma unroll
    for (int t = 0; t < P; ++t) s[t] += x * Cbar[t + (int64_t)j * P];
  }
#pragma unroll
  for (int t = 0; t < P; ++t) part[((int64_t)g * P + t) * N + r] = s[t];
}

__global__ void wbar_add_kernel(const double* __restrict__ part, int N, int P, int gn, double* __restrict__ Wbar) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)N * P) return;
  const int r = (int)(idx % N), t = (int)(idx / N);
  double run = Wbar[idx];
#pragma unroll 8
  for (int g = 0; g < gn; ++g) run += part[((int64_t)g * P + t) * N + r];
  Wbar[idx] = run;
}

// Xtbar[r, j] = sum_t W[r, t] Cbar[t, j] + ebar[j] Xt[r, j]   (N x mb, ld N)
template <int P>
__global__ void xtbar_kernel(const double* __restrict__ W, const double* __restrict__ Xt, const double* __restrict__ Cbar,
                             const double* __restrict__ ebar, int N, int mb, double* __restrict__ Xtbar) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * mb;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % N);
    const int j = (int)(idx / N);
    double s = ebar[j] * Xt[idx];
#pragma unroll
    for (int t = 0; t < P; ++t) s += W[r + (int64_t)t * N] * Cbar[t + (int64_t)j * P];
    Xtbar[idx] = s;
  }
}

// Wbar[r, t] += sum_u W[r, u] Ghat[u, t],  Ghat = [[2 S_TLbar, r~_Tbar], [r~_Tbar^T, 2 cbar]]
// built from the accumulated shared adjoints acc (layout as contrib).
template <int P>
__global__ void wbar_shared_kernel(const double* __restrict__ W, const double* __restrict__ acc, int N,
                                   double* __restrict__ Wbar) {
  constexpr int Q = P - 1;
  __shared__ double G[P * P];
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < Q; ++i)
      for (int j = 0; j <= i; ++j) {
        G[i + j * P] = 2.0 * acc[t];
        G[j + i * P] = 2.0 * acc[t];
        ++t;
      }
    for (int j = 0; j < Q; ++j) {
      G[j + Q * P] = acc[t];
      G[Q + j * P] = acc[t];
      ++t;
    }
    G[Q + Q * P] = 2.0 * acc[t];
  }
  __syncthreads();
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  for (; r < N; r += gridDim.x * blockDim.x) {
    double w[P];
#pragma unroll
    for (int u = 0; u < P; ++u) w[u] = W[r + (int64_t)u * N];
#pragma unroll
    for (int c = 0; c < P; ++c) {
      double s = Wbar[r + (int64_t)c * N];
#pragma unroll
      for (int u = 0; u < P; ++u) s += w[u] * G[u + c * P];
      Wbar[r + (int64_t)c * N] = s;
    }
  }
}

// A (N x N): zero above the diagonal; with halve_diag also halve the diagonal
// (the operator that keeps the lower triangle and half the diagonal).
// W (N x P, ld N) = L^-T V for V (N x P, ld N) and the lower-triangular
// inverse factor Li (N x N, ld N): row i of the result needs column i of Li
// from row i down, a contiguous run.  One wave per output row, lanes over k
// (four loads in flight per lane), then a fixed-order wave reduction per
// column of V.
template <int P>
__global__ __launch_bounds__(256) void tri_apply_t_kernel(const double* __restrict__ Li, int N,
                                                          const double* __restrict__ V, double* __restrict__ W) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= N) return;
  const double* col = Li + (int64_t)i * N;
  double acc[P];
#pragma unroll
  for (int j = 0; j < P; ++j) acc[j] = 0.0;
  for (int kb = i + lane; kb < N; kb += 256) {
    double a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = (kb + 64 * u < N) ? col[kb + 64 * u] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = kb + 64 * u;
      if (k < N) {
#pragma unroll
        for (int j = 0; j < P; ++j) acc[j] = fma(a[u], V[k + (int64_t)j * N], acc[j]);
      }
    }
  }
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const double t = wave_sum(acc[j]);
    if (lane == 0) W[i + (int64_t)j * N] = t;
  }
}

__global__ void lower_part_kernel(double* __restrict__ A, int N, int halve_diag) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * N;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % N), j = (int)(idx / N);
    if (i < j) A[idx] = 0.0;
    else if (i == j && halve_diag) A[idx] *= 0.5;
  }
}

// Partial sums of <Q, Phi - I> over the leading n x n block, reading only the
// lower triangle of Phi:  sum_i Q_ii (Phi_ii - 1) + sum_{i>j} (Q_ij + Q_ji) Phi_ij.
__global__ __launch_bounds__(256) void h2_contract_kernel(const double* __restrict__ Qm, const double* __restrict__ Phi,
                                                          int N, int n, double* __restrict__ part) {
  __shared__ double red[256];
  double s = 0.0;
  const int64_t total = (int64_t)N * N;
  for (int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx % N), j = (int)(idx / N);
    if (i >= n || j >= n || i < j) continue;
    if (i == j) s += Qm[idx] * (Phi[idx] - 1.0);
    else s += (Qm[idx] + Qm[(int64_t)j + (int64_t)i * N]) * Phi[idx];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[0] = sum of part[0..count) in index order (one thread: fixed order).
__global__ void sum_ordered_kernel(const double* __restrict__ part, int count, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < count; ++i) s += part[i];
  out[0] = s;
}

// Phi copy for the h2 adjoint: P (N x N, ld N) = lower triangle of Phi (n x n), zeros elsewhere.
__global__ void keep_phi_kernel(double* __restrict__ Pk, int N, int n, const double* __restrict__ Phi, int64_t ld_phi) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * N;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx % N), j = (int)(idx / N);
    Pk[idx] = (i < n && j < n && i >= j) ? Phi[(int64_t)i + (int64_t)j * ld_phi] : 0.0;
  }
}

}  // namespace gls
