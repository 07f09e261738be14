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
#include "lds_dma.hpp"

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

// Packed dosages: four 2-bit codes per byte, sample k of a column in bits
// [2 (k % 4), 2 (k % 4) + 2) of the column's byte k / 4; code value = dosage
// (0..3).  Bits of the last byte past row n - 1 are ignored.  One thread per
// four output rows; rows n..N-1 are zero.
__device__ __forceinline__ uint32_t unpack_quad(const uint8_t* __restrict__ G2, int64_t ldg, int n, int q, int j) {
  const int k0 = 4 * q;
  if (k0 >= n) return 0u;
  const uint32_t b = G2[(int64_t)j * ldg + q];
  uint32_t w = (b & 3u) | ((b & 0x0cu) << 6) | ((b & 0x30u) << 12) | ((b & 0xc0u) << 18);
  const int rem = n - k0;
  if (rem < 4) w &= (1u << (8 * rem)) - 1u;
  return w;   // byte t = dosage of row k0 + t
}

// Packed dosages of a block into an N-row, zero-padded column-major byte buffer.
__global__ void unpack_u2_kernel(const uint8_t* __restrict__ G2, int64_t ldg, int n, int N, int mb,
                                 uint32_t* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int Q = N / 4;
  const int64_t total = (int64_t)Q * mb;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(idx % Q), j = (int)(idx / Q);
    out[idx] = unpack_quad(G2, ldg, n, q, j);
  }
}

// Packed dosages of a block as FP64 (exact), N-row zero-padded, ld N.
__global__ void unpack_u2_f64_kernel(const uint8_t* __restrict__ G2, int64_t ldg, int n, int N, int mb,
                                     double* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int Q = N / 4;
  const int64_t total = (int64_t)Q * mb;
  for (; idx < total; idx += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(idx % Q), j = (int)(idx / Q);
    const uint32_t w = unpack_quad(G2, ldg, n, q, j);
    double2* o = reinterpret_cast<double2*>(out + (int64_t)j * N + 4 * q);
    o[0] = double2{(double)(w & 0xffu), (double)((w >> 8) & 0xffu)};
    o[1] = double2{(double)((w >> 16) & 0xffu), (double)(w >> 24)};
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
// for bytes e = 0..15 (any k order shared by A and B gives the same sum);
// accumulator element t is D[4 (l / 16) + t][l % 16].
//
// The kernel computes the transpose, D = X^T a_s^T, so that the accumulator's
// fast index (l % 16) runs down a column of the column-major result and the
// FP64 stores are 128-byte runs.  A workgroup of sixteen waves owns a 32 x 256
// output tile: wave w takes the 16-row strip w & 1, the 64-column strip
// (w >> 1) & 3 and the slice half w >> 3 (slices 0..3 or 4..7), holding 4 x 4
// accumulators (one per slice and 16-column group).  Splitting the slices over
// two waves halves the accumulators, so four waves share each SIMD instead of
// two and one wave's wait at the stage barrier no longer idles the matrix
// pipe as often (5% faster than eight waves holding all eight slices, with
// bitwise the same results).  Per 64-deep k step a wave reads four byte
// fragments and one fragment per slice from LDS and issues 16 MFMAs.  At the
// end the second half adds its slices 7..4 into an LDS buffer (reusing the
// ring) and the first half continues with 3..0: the same order as one wave
// summing all eight.
//
// Operands reach LDS by direct global-to-LDS loads (global_load_lds_dwordx4:
// no staging registers) into a ring of OZ_STAGES buffers, OZ_STAGES - 1 steps
// ahead of the MFMAs (see lds_dma.hpp).  One load instruction moves 1 KB: sixteen 64-byte rows, lane l
// writing bytes [16 l, 16 l + 16) of it.  Chunk c of row r is stored in slot
// c ^ oz_swz(r), so that a fragment read (sixteen rows, one chunk each) puts
// every eight consecutive lanes on distinct 128-byte bank lines and all sixteen
// on distinct 256-byte lines.
constexpr int OZ_BM = 32, OZ_BN = 256, OZ_BK = 64, OZ_THREADS = 1024, OZ_STAGES = 4;

__device__ __forceinline__ int oz_swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

__global__ __launch_bounds__(OZ_THREADS) void ozaki_i8_kernel(OzArgs g) {
  constexpr int BM = OZ_BM, BN = OZ_BN, BK = OZ_BK, S = OZ_SLICES, NW = OZ_THREADS / 64, NS = OZ_STAGES;
  constexpr int SH = S / 2;                      // slices per wave: the two wave halves take slices 0..3 and 4..7
  constexpr int RB = BK;                         // bytes per LDS row
  constexpr int ABYTES = S * BM * RB, STAGE = ABYTES + BN * RB;
  constexpr int QA = S * BM / 16 / NW;           // 1 KB load instructions per wave and stage
  constexpr int QB = BN / 16 / NW;
  static_assert(BK == 64 && BM == 32 && NW == 4 * (BN / 64), "two row strips x BN / 64 column strips x two slice halves");
  static_assert(QA * 16 * NW == S * BM && QB * 16 * NW == BN && NS >= 2 && NS <= 5, "loader split");
  constexpr int PS = BN + 2;                     // row stride of the partial sums: 16 rows on distinct banks
  static_assert(NS * STAGE <= 160 * 1024 && BM * PS * 8 <= NS * STAGE, "LDS (the ring holds the partial sums at the end)");
  __shared__ __align__(1024) int8_t smem[NS * STAGE];

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
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wi = wave & 1, wj = (wave >> 1) & 3, wsl = wave >> 3;
  const int64_t plane = (int64_t)g.N * g.N;

  const int lrow = lane >> 2, lchunk = ((lane & 3) ^ oz_swz(lrow)) * 16;
  const int8_t* pa[QA];
  const uint8_t* pb[QB];
#pragma unroll
  for (int q = 0; q < QA; ++q) {
    const int r = 16 * (q * NW + wave) + lrow, s = r / BM, ri = r % BM;
    pa[q] = g.A + s * plane + (int64_t)(i0 + ri) * g.N + lchunk;
  }
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int j = min(j0 + 16 * (q * NW + wave) + lrow, g.ncols - 1);   // columns past the end: any valid
    pb[q] = g.B + (int64_t)j * g.N + lchunk;                            // column, their results are dropped
  }
  const uint32_t lds0 = lds_address(smem);
  auto issue = [&](int kstep) {
    const uint32_t base = lds0 + (uint32_t)((kstep % NS) * STAGE);
    const int kt = kstep * BK;
#pragma unroll
    for (int q = 0; q < QA; ++q)
      lds_load16(pa[q] + kt, __builtin_amdgcn_readfirstlane(base + 1024 * (q * NW + wave)));
#pragma unroll
    for (int q = 0; q < QB; ++q)
      lds_load16(pb[q] + kt, __builtin_amdgcn_readfirstlane(base + ABYTES + 1024 * (q * NW + wave)));
  };

  i4_t acc[SH][4];
#pragma unroll
  for (int s = 0; s < SH; ++s)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[s][c] = i4_t{0, 0, 0, 0};

  const int fr = lane & 15, slot = ((lane >> 4) ^ oz_swz(fr)) * 16;
  const int oa = (wsl * SH * BM + wi * 16 + fr) * RB + slot;
  const int ob = ABYTES + (wj * 64 + fr) * RB + slot;

  for (int q = 0; q < NS - 1; ++q)
    if (q < nk) issue(q);
  for (int it = 0; it < nk; ++it) {
    wait_stages<QA + QB>(min(nk - 1 - it, NS - 2));
    __syncthreads();
    if (it + NS - 1 < nk) issue(it + NS - 1);
    const int8_t* st = smem + (it % NS) * STAGE;
    i4_t bf[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) bf[c] = *reinterpret_cast<const i4_t*>(st + ob + c * 16 * RB);
#pragma unroll
    for (int s = 0; s < SH; ++s) {
      const i4_t af = *reinterpret_cast<const i4_t*>(st + oa + s * BM * RB);
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[s][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(bf[c], af, acc[s][c], 0, 0, 0);
    }
  }

  // slices 7..4 (second half) first, then 3..0, the same order as one wave holding all eight
  const int i = i0 + wi * 16 + fr;
  const int e = g.ex[i];
  double* part = reinterpret_cast<double*>(smem);   // 32 x 256 partial sums of the second half (row stride PS)
  wait_vmcnt<0>();
  __syncthreads();                                  // every wave is done with the ring
  if (wsl == 1) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double v = 0.0;
#pragma unroll
        for (int s = SH - 1; s >= 0; --s) v += ldexp((double)acc[s][c][t], e - 7 * (SH + s + 1));
        part[(wi * 16 + fr) * PS + wj * 64 + c * 16 + 4 * (lane >> 4) + t] = v;
      }
  }
  __syncthreads();
  if (wsl == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int jl = wj * 64 + c * 16 + 4 * (lane >> 4) + t;
        const int j = j0 + jl;
        double v = part[(wi * 16 + fr) * PS + jl];
#pragma unroll
        for (int s = SH - 1; s >= 0; --s) v += ldexp((double)acc[s][c][t], e - 7 * (s + 1));
        if (j < g.ncols) g.C[(int64_t)i + (int64_t)j * g.ldc] = v;
      }
    }
  }
}

}  // namespace gls
