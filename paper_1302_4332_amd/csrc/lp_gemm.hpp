// Low-precision matrix products for the mixed-precision triangular solve:
//
//   C[i, j] = beta * Cin[i, j] + cscale[j] * sum_k A[i, k] * B[k, j]
//
// A is the lower-triangular inverse factor stored row-major in T (FP32,
// FP16 or BF16), B a column-major block of T, accumulation in FP32 on the
// matrix cores, C in FP64.  cscale[j] undoes the power-of-two scalings of A
// and of column j of B exactly.  Used for the bulk solve X~0 = L^-1 X and for
// the correction solves of the refinement sweeps (beta = 1, Cin = C).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_f64.hpp"

namespace gls {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));

// Row of the accumulator element t held by lane l in the 16x16 FP32-output
// MFMA forms (checked on gfx950 with known operands).
__device__ __forceinline__ int lp_acc_row(int lane, int t) { return 4 * (lane >> 4) + t; }

struct LpArgs {
  const void* A; int64_t lda;     // row-major: A[i * lda + k]
  const void* B; int64_t ldb;     // column-major: B[k + j * ldb]
  const double* Cin; int64_t ldcin;
  double* C; int64_t ldc;
  const double* cscale;           // per column
  int M, mvalid, ncols, K;
  double beta;
  int map_gm, map_gn, map_desc;   // as GemmArgs (XCD mapping, lower-triangular A)
};

template <typename T> struct LpMfma;

template <> struct LpMfma<float> {
  static constexpr int KSTEP = 4;   // k per instruction
  static constexpr int KPL = 1;     // k per lane
  __device__ static f4_t mma(const float* a, const float* b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  }
};
template <> struct LpMfma<_Float16> {
  static constexpr int KSTEP = 32;
  static constexpr int KPL = 8;
  __device__ static f4_t mma(const _Float16* a, const _Float16* b, f4_t c) {
    h8_t av, bv;
#pragma unroll
    for (int e = 0; e < 8; ++e) { av[e] = a[e]; bv[e] = b[e]; }
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
  }
};
template <> struct LpMfma<__bf16> {
  static constexpr int KSTEP = 32;
  static constexpr int KPL = 8;
  __device__ static f4_t mma(const __bf16* a, const __bf16* b, f4_t c) {
    b8_t av, bv;
#pragma unroll
    for (int e = 0; e < 8; ++e) { av[e] = a[e]; bv[e] = b[e]; }
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
  }
};

// 64 x 64 tiles, BK = 64 k per LDS slice, four waves each owning a 64 x 16
// strip (four 16x16 accumulators).  Both operands are k-contiguous in global
// memory and in LDS (As[i][k], Bs[j][k]); 16-byte vector moves.  Requires
// 16-byte aligned A/B, lda and ldb multiples of 8 elements, K a multiple of
// BK (the callers pad every operand).
template <typename T>
__global__ __launch_bounds__(256) void lp_gemm_kernel(LpArgs g) {
  constexpr int BM = 64, BN = 64, BK = 64;
  constexpr int VE = 16 / sizeof(T);           // elements per 16-byte move
  constexpr int PAD = VE;                      // keeps rows 16-byte aligned, staggers banks
  constexpr int SK = BK + PAD;
  constexpr int KSTEP = LpMfma<T>::KSTEP;
  constexpr int KPL = LpMfma<T>::KPL;
  constexpr int CH = BM * BK / VE;             // 16-byte chunks per operand slice
  constexpr int PER = CH / 256;
  static_assert(CH % 256 == 0, "loader");
  __shared__ T As[2][BM * SK];
  __shared__ T Bs[2][BN * SK];

  int ti, tj;
  {
    GemmArgs m{};
    m.map_gm = g.map_gm;
    m.map_gn = g.map_gn;
    m.map_desc = g.map_desc;
    const int Mt = g.M / BM, Nt = (g.ncols + BN - 1) / BN;
    if (!XcdMap::tile(m, blockIdx.x, Mt, Nt, &ti, &tj)) return;
  }
  const int i0 = ti * BM, j0 = tj * BN;
  const int khi = (i0 + BM < g.K) ? i0 + BM : g.K;   // A lower triangular
  const int nk = (khi + BK - 1) / BK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T* A = static_cast<const T*>(g.A);
  const T* B = static_cast<const T*>(g.B);

  f4_t acc[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) acc[a] = f4_t{0.f, 0.f, 0.f, 0.f};

  uint4 ra[PER], rb[PER];
  auto load = [&](int kt) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int c = tid + e * 256;
      const int r = c / (BK / VE), kc = (c % (BK / VE)) * VE;
      ra[e] = *reinterpret_cast<const uint4*>(A + (int64_t)(i0 + r) * g.lda + kt + kc);
      rb[e] = *reinterpret_cast<const uint4*>(B + (int64_t)(kt + kc) + (int64_t)(j0 + r) * g.ldb);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int c = tid + e * 256;
      const int r = c / (BK / VE), kc = (c % (BK / VE)) * VE;
      *reinterpret_cast<uint4*>(&As[buf][r * SK + kc]) = ra[e];
      *reinterpret_cast<uint4*>(&Bs[buf][r * SK + kc]) = rb[e];
    }
  };
  if (nk > 0) {
    load(0);
    store(0);
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int buf = it & 1;
      if (it + 1 < nk) load((it + 1) * BK);
#pragma unroll
      for (int kk = 0; kk < BK; kk += KSTEP) {
        const int ko = kk + (lane >> 4) * KPL;
        T bf[KPL];
#pragma unroll
        for (int e = 0; e < KPL; ++e) bf[e] = Bs[buf][(wave * 16 + (lane & 15)) * SK + ko + e];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          T af[KPL];
#pragma unroll
          for (int e = 0; e < KPL; ++e) af[e] = As[buf][(a * 16 + (lane & 15)) * SK + ko + e];
          acc[a] = LpMfma<T>::mma(af, bf, acc[a]);
        }
      }
      if (it + 1 < nk) store(buf ^ 1);
      __syncthreads();
    }
  }
  const int j = j0 + wave * 16 + (lane & 15);
  if (j >= g.ncols) return;
  const double cs = g.cscale[j];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int i = i0 + a * 16 + lp_acc_row(lane, t);
      if (i >= g.mvalid) continue;
      double v = cs * (double)acc[a][t];
      if (g.beta != 0.0) v += g.beta * g.Cin[(int64_t)i + (int64_t)j * g.ldcin];
      g.C[(int64_t)i + (int64_t)j * g.ldc] = v;
    }
  }
}

// Column-wise power-of-two scaling and conversion of an FP64 block:
//   out[k + j * ldo] = T(src[k + j * lds] * 2^e_j) for k < rows, 0 for rows..N-1,
//   cscale[j] = 2^-e_j * (*ascalep), with e_j chosen so the column's largest
//   magnitude lands in [target/2, target).  One wave per column.
template <typename T>
__global__ __launch_bounds__(256) void scale_convert_kernel(const double* __restrict__ src, int64_t lds, int rows,
                                                            int N, int ncols, T* __restrict__ out, int64_t ldo,
                                                            double target, const double* __restrict__ ascalep,
                                                            double* __restrict__ cscale) {
  const double ascale = *ascalep;
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= ncols) return;
  const double* s = src + (int64_t)j * lds;
  double mx = 0.0;
  for (int k = lane; k < rows; k += 64) mx = fmax(mx, fabs(s[k]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  int e = 0;
  if (mx > 0.0 && mx == mx && mx < __builtin_inf()) {
    int ex;
    frexp(mx / target, &ex);   // mx / target in [2^(ex-1), 2^ex)
    e = -ex;
  }
  const double sc = ldexp(1.0, e);
  T* o = out + (int64_t)j * ldo;
  for (int k = lane; k < N; k += 64) o[k] = (k < rows) ? (T)(s[k] * sc) : (T)0.0f;
  if (lane == 0) cscale[j] = ldexp(ascale, -e);
}

// Row-major low-precision copy of the lower-triangular N x N factor inverse,
// scaled by the power of two 2^e that puts its largest magnitude (*maxp) in
// [target/2, target):  out[i * N + k] = T(Li[i + k * N] * 2^e); *fscale = 2^-e.
template <typename T>
__global__ void convert_factor_kernel(const double* __restrict__ Li, int N, T* __restrict__ out,
                                      const double* __restrict__ maxp, double target, double* __restrict__ fscale) {
  int ex = 0;
  frexp(*maxp / target, &ex);
  const int e = -ex;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx == 0) *fscale = ldexp(1.0, -e);
  const int64_t total = (int64_t)N * N;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / N), k = (int)(idx % N);
    out[idx] = (T)ldexp(Li[(int64_t)i + (int64_t)k * N], e);
  }
}

// Largest magnitude of an array: out[blockIdx.x] = max over a grid-stride
// share (run once over the data with many workgroups, then once with one
// workgroup over the partial maxima).
__global__ __launch_bounds__(256) void maxabs_kernel(const double* __restrict__ p, int64_t count,
                                                     double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
    m = fmax(m, fabs(p[i]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace gls
