// FP64-accurate per-block product on the integer matrix cores, for genotype
// dosages held as bytes.
//
// Each row i of L^-1 is split exactly into S int8 slices (Ozaki-style):
//     L^-1[i, k] = 2^e_i * sum_{s<S} a_s[i, k] * 2^(-7 (s+1))  +  r_ik,
//     |a_s| <= 127,  |r_ik| < 2^(e_i - 7 S),  max_k |L^-1[i, k]| < 2^e_i,
// obtained by repeatedly scaling by 2^7 and taking the integer part (every
// step exact in FP64).  Dosages x are small integers, exact in int8, so
//     (L^-1 X)[i, j] = sum_s 2^(e_i - 7(s+1)) * (a_s X)[i, j]   (+ truncation)
// where each a_s X is an exact int32 product (|a_s x| sums stay below 2^31
// for n * 127 * max|x| < 2^31).  With S = 8 the truncation is below 2^-56 of
// the row's largest entry, under FP64 rounding of the result.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_f64.hpp"

namespace gls {

constexpr int OZ_SLICES = 8;

typedef int i4_t __attribute__((ext_vector_type(4)));

// Per-row exponent: ex[i] with max_k |Li[i, k]| < 2^ex[i] (0 for a zero row).
// One thread per row; threads of a wave read consecutive rows (coalesced).
__global__ void row_exponent_kernel(const double* __restrict__ Li, int N, int* __restrict__ ex) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double m = 0.0;
  for (int k = 0; k <= i; ++k) m = fmax(m, fabs(Li[(int64_t)i + (int64_t)k * N]));
  int e = 0;
  if (m > 0.0) frexp(m, &e);
  ex[i] = e;
}

// Slices: out[s][i * N + k] = a_s[i, k] (row-major, k contiguous) for a 64 x 64
// tile per workgroup; reads Li column-major through LDS.
__global__ __launch_bounds__(256) void slice_factor_kernel(const double* __restrict__ Li, int N,
                                                           const int* __restrict__ ex, int8_t* __restrict__ out) {
  __shared__ double tile[64][65];
  const int i0 = blockIdx.y * 64, k0 = blockIdx.x * 64;
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int ii = idx % 64, kk = idx / 64;
    tile[ii][kk] = Li[(int64_t)(i0 + ii) + (int64_t)(k0 + kk) * N];
  }
  __syncthreads();
  const int64_t plane = (int64_t)N * N;
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    const int kk = idx % 64, ii = idx / 64;
    double v = ldexp(tile[ii][kk], -ex[i0 + ii]);   // |v| < 1, exact
    const int64_t o = (int64_t)(i0 + ii) * N + (k0 + kk);
#pragma unroll
    for (int s = 0; s < OZ_SLICES; ++s) {
      v *= 128.0;                   // exact
      const double d = trunc(v);    // |d| <= 127
      v -= d;                       // exact
      out[s * plane + o] = (int8_t)d;
    }
  }
}

// Bytes of a block into an N-row, zero-padded column-major buffer.
__global__ void pack_u8_kernel(const uint8_t* __restrict__ G, int64_t ldg, int n, int N, int mb,
                               uint8_t* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * mb;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx % N), j = (int)(idx / N);
    out[idx] = (k < n) ? G[(int64_t)k + (int64_t)j * ldg] : (uint8_t)0;
  }
}

// Bytes of a block as FP64 (exact), N-row zero-padded, ld N.
__global__ void u8_to_f64_kernel(const uint8_t* __restrict__ G, int64_t ldg, int n, int N, int mb,
                                 double* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)N * mb;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(idx % N), j = (int)(idx / N);
    out[idx] = (k < n) ? (double)G[(int64_t)k + (int64_t)j * ldg] : 0.0;
  }
}

struct OzArgs {
  const int8_t* A;        // OZ_SLICES planes of N x N, row-major
  const int* ex;          // row exponents
  const uint8_t* B;       // N x ncols bytes, column-major, ld N (rows >= n are zero)
  double* C; int64_t ldc; // N x ncols FP64
  int N, ncols;
  int map_gm, map_gn;
};

// v_mfma_i32_16x16x64_i8 operand layout (checked on gfx950 with known
// operands): lane l holds A[l % 16][16 (l / 16) + e] and B[16 (l / 16) + e][l % 16]
// for bytes e = 0..15; accumulator element t is C[4 (l / 16) + t][l % 16].
//
// 64 x 64 output tiles, k in slices of 64; four waves, each a 64 x 16 strip
// (four 16x16 int32 accumulators per slice).  The byte block is staged once
// per k-slice and shared by all S factor slices.
__global__ __launch_bounds__(256) void ozaki_i8_kernel(OzArgs g) {
  constexpr int BM = 64, BN = 64, BK = 64, S = OZ_SLICES;
  constexpr int SK = BK + 16;   // LDS row stride in bytes (16-byte aligned, staggered)
  __shared__ int8_t As[2][S][BM * SK];
  __shared__ uint8_t Bs[2][BN * SK];

  int ti, tj;
  {
    GemmArgs m{};
    m.map_gm = g.map_gm;
    m.map_gn = g.map_gn;
    m.map_desc = 1;
    const int Mt = g.N / BM, Nt = (g.ncols + BN - 1) / BN;
    if (!XcdMap::tile(m, blockIdx.x, Mt, Nt, &ti, &tj)) return;
  }
  const int i0 = ti * BM, j0 = tj * BN;
  const int nk = (i0 + BM + BK - 1) / BK;   // lower triangular factor: k < i0 + BM
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t plane = (int64_t)g.N * g.N;

  i4_t acc[S][4];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[s][a] = i4_t{0, 0, 0, 0};

  // loader: 16-byte chunks; a 64 x 64 byte tile is 256 chunks, one per thread
  const int lr = tid / 4, lc = (tid % 4) * 16;
  uint4 ra[S], rb;
  auto load = [&](int kt) {
#pragma unroll
    for (int s = 0; s < S; ++s)
      ra[s] = *reinterpret_cast<const uint4*>(g.A + s * plane + (int64_t)(i0 + lr) * g.N + kt + lc);
    rb = *reinterpret_cast<const uint4*>(g.B + (int64_t)(kt + lc) + (int64_t)(j0 + lr) * g.N);
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int s = 0; s < S; ++s) *reinterpret_cast<uint4*>(&As[buf][s][lr * SK + lc]) = ra[s];
    *reinterpret_cast<uint4*>(&Bs[buf][lr * SK + lc]) = rb;
  };
  load(0);
  store(0);
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    if (it + 1 < nk) load((it + 1) * BK);
    const int ko = (lane >> 4) * 16;
    const i4_t bf = *reinterpret_cast<const i4_t*>(&Bs[buf][(wave * 16 + (lane & 15)) * SK + ko]);
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const i4_t af = *reinterpret_cast<const i4_t*>(&As[buf][s][(a * 16 + (lane & 15)) * SK + ko]);
        acc[s][a] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af, bf, acc[s][a], 0, 0, 0);
      }
    }
    if (it + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }
  const int j = j0 + wave * 16 + (lane & 15);
  if (j >= g.ncols) return;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = i0 + a * 16 + 4 * (lane >> 4) + t;
      const int e = g.ex[i];
      double v = 0.0;
#pragma unroll
      for (int s = S - 1; s >= 0; --s) v += ldexp((double)acc[s][a][t], e - 7 * (s + 1));
      g.C[(int64_t)i + (int64_t)j * g.ldc] = v;
    }
  }
}

}  // namespace gls
