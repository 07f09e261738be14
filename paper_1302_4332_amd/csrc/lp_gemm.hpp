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
#include "lds_dma.hpp"

namespace gls {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef __bf16 b8_t __attribute__((ext_vector_type(8)));

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

// One 16-byte chunk of k per lane and operand feeds SUB matrix-core
// instructions.  Operand layouts (gfx950): in the 16x16 forms lane l holds
// row (or column) l % 16 of its operand; for FP16/BF16 (16x16x32) the chunk is
// the 8 consecutive k at 8 (l / 16), one instruction; for FP32 (16x16x4, one k
// per lane) element s of the chunk feeds instruction s, i.e. instruction s
// sums k = 4 (l / 16) + s over the four lane groups (a permutation of k that
// both operands share, so the sum is the same).  Accumulator element t is
// D[4 (l / 16) + t][l % 16].
template <typename T> struct LpMfma;

template <> struct LpMfma<float> {
  static constexpr int SUB = 4;
  __device__ static f4_t mma(uint4 a, uint4 b, f4_t c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
    return c;
  }
};
template <> struct LpMfma<_Float16> {
  static constexpr int SUB = 1;
  __device__ static f4_t mma(uint4 a, uint4 b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8_t, a), __builtin_bit_cast(h8_t, b), c, 0, 0, 0);
  }
};
template <> struct LpMfma<__bf16> {
  static constexpr int SUB = 1;
  __device__ static f4_t mma(uint4 a, uint4 b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(b8_t, a), __builtin_bit_cast(b8_t, b), c, 0, 0,
                                                  0);
  }
};

// Tiles of 256 rows of A x 128 columns of B; eight waves, each a 64 x 64
// block (4 x 4 accumulators of 16 x 16).  Each stage covers 64 bytes of k per
// row (32 FP16/BF16 or 16 FP32 values); the 256 + 128 rows of a stage move
// straight from global memory into a ring of three LDS buffers (1 KB, sixteen
// rows, per wave instruction; two stages in flight ahead of the MFMAs).  A
// stage is 24 KB, so two workgroups share a compute unit (four waves per
// SIMD, 102 VGPRs); with 128-byte stages (48 KB, one workgroup and two waves
// per SIMD) the same MFMA sequence ran 9-12% slower.  Chunk c of LDS row r sits
// in slot c ^ lp_swz(r): eight consecutive lanes of a fragment read fall on
// distinct banks.  The product is formed transposed (B's columns as the
// instruction's first operand) so that the FP64 stores of C run down columns.
// Requires 16-byte aligned A and B, lda and ldb multiples of 8 elements, K a
// multiple of 32 and lane offsets within a tile below 2^32 bytes (the callers
// pad every operand to N, a multiple of 256).
constexpr int LP_BM = 256, LP_BN = 128, LP_RB = 64, LP_THREADS = 512, LP_STAGES = 3;

__device__ __forceinline__ int lp_swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

template <typename T>
__global__ __launch_bounds__(LP_THREADS) __attribute__((amdgpu_waves_per_eu(4, 8)))
void lp_gemm_kernel(LpArgs g) {
  constexpr int BM = LP_BM, BN = LP_BN, RB = LP_RB, NW = LP_THREADS / 64, NS = LP_STAGES;
  constexpr int CPR = RB / 16;               // 16-byte chunks per LDS row
  constexpr int RPI = 1024 / RB;             // rows per 1 KB load instruction
  constexpr int BKE = RB / (int)sizeof(T);   // k per stage
  constexpr int STAGE = (BM + BN) * RB;      // bytes
  constexpr int NLD = (BM + BN) / RPI / NW;  // load instructions per wave and stage
  static_assert(NLD * RPI * NW == BM + BN && BM % RPI == 0 && BM == 4 * 64 && BN == 2 * 64 && NW == 8, "tile split");
  static_assert(RB == 64 && NS * STAGE <= 80 * 1024, "two workgroups per compute unit");
  __shared__ __align__(1024) char smem[NS * STAGE];

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
  const int nk = (khi + BKE - 1) / BKE;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wi = wave & 3, wj = wave >> 2;

  // loader: instruction q of this wave fills stage rows RPI (q NW + wave) ..
  // + RPI - 1, all of A's tile (rows i0..) or all of B's (columns j0..; columns
  // past the end read the last valid one, whose results are dropped); a
  // wave-uniform base per operand plus a 32-bit byte offset per lane
  const char* Abase = static_cast<const char*>(g.A) + (int64_t)i0 * g.lda * (int64_t)sizeof(T);
  const char* Bbase = static_cast<const char*>(g.B) + (int64_t)j0 * g.ldb * (int64_t)sizeof(T);
  uint32_t voff[NLD];
#pragma unroll
  for (int q = 0; q < NLD; ++q) {
    const int r0 = RPI * (q * NW + wave);
    const int r = r0 + lane / CPR;
    const int chunk = (lane % CPR) ^ lp_swz(r);
    if (r0 < BM) {
      voff[q] = (uint32_t)((int64_t)r * g.lda * (int64_t)sizeof(T) + 16 * chunk);
    } else {
      const int jl = min(j0 + r - BM, g.ncols - 1) - j0;
      voff[q] = (uint32_t)((int64_t)jl * g.ldb * (int64_t)sizeof(T) + 16 * chunk);
    }
  }
  const uint32_t lds0 = lds_address(smem);
  auto issue = [&](int kstep) {
    const uint32_t base = lds0 + (uint32_t)((kstep % NS) * STAGE);
    const int64_t kb = (int64_t)kstep * RB;
#pragma unroll
    for (int q = 0; q < NLD; ++q)
      lds_load16_sv((RPI * (q * NW + wave) < BM ? Abase : Bbase) + kb, voff[q], base + 1024 * (q * NW + wave));
  };

  // fragment offsets within a stage: lane group lane >> 4 reads chunk lane >> 4 of its row
  int offa[4], offb[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const int ra = wi * 64 + f * 16 + (lane & 15), rb = BM + wj * 64 + f * 16 + (lane & 15);
    const int c = lane >> 4;
    offa[f] = ra * RB + 16 * (c ^ lp_swz(ra));
    offb[f] = rb * RB + 16 * (c ^ lp_swz(rb));
  }

  f4_t acc[4][4];   // [column block][row block], transposed 16 x 16 products
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[b][a] = f4_t{0.f, 0.f, 0.f, 0.f};

  for (int q = 0; q < NS - 1; ++q)
    if (q < nk) issue(q);
  for (int it = 0; it < nk; ++it) {
    wait_stages<NLD>(min(nk - 1 - it, NS - 2));   // this wave's loads of stage it have landed ...
    __syncthreads();                              // ... and every wave's; stage (it - 1) % NS is free
    if (it + NS - 1 < nk) issue(it + NS - 1);
    const char* st = smem + (it % NS) * STAGE;
    uint4 fa[4], fb[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      fa[f] = *reinterpret_cast<const uint4*>(st + offa[f]);
      fb[f] = *reinterpret_cast<const uint4*>(st + offb[f]);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int a = 0; a < 4; ++a) acc[b][a] = LpMfma<T>::mma(fb[b], fa[a], acc[b][a]);
  }

  // acc[b][a][t] = C[i0 + wi 64 + 16 a + lane % 16][j0 + wj 64 + 16 b + 4 (lane / 16) + t]
#pragma unroll
  for (int b = 0; b < 4; ++b) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = j0 + wj * 64 + b * 16 + 4 * (lane >> 4) + t;
      if (j >= g.ncols) continue;
      const double cs = g.cscale[j];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int i = i0 + wi * 64 + a * 16 + (lane & 15);
        if (i >= g.mvalid) continue;
        double v = cs * (double)acc[b][a][t];
        if (g.beta != 0.0) v += g.beta * g.Cin[(int64_t)i + (int64_t)j * g.ldcin];
        g.C[(int64_t)i + (int64_t)j * g.ldc] = v;
      }
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
