// FP64 product C = alpha op(A) B + beta Cin for the per-block solve
// X~ = L^-1 X and the refinement residual X - L X~ (also the setup's panel and
// trailing products and the adjoint's L-bar update): A column-major and lower
// or upper triangular (or full), B column-major (full, or lower triangular
// under a full A), C column-major, optionally only the tiles that reach C's
// lower part.  The same
// v_mfma_f64_4x4x4_4b_f64 accumulation as gemm_f64_kernel with the k order
// permuted within each 16-deep stage; operands reach LDS by direct
// global-to-LDS loads into a ring of stages.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gemm_f64.hpp"
#include "lds_dma.hpp"

namespace gls {

// 128 x 64 tiles, 16 k per stage, eight waves of 64 x 16 (two row strips x four
// column strips; each wave 4 x 4 v_mfma_f64_4x4x4_4b_f64 accumulators as in
// gemm_f64_kernel).  Permuting k saves half of the B fragment reads.  A stage
// is 16 KB of A (16 k-columns of 128 rows, one 1 KB load instruction each) and
// 8 KB of B (64 columns of 16 k, eight columns per instruction), in a ring of
// two stages.  16-byte chunks are placed so that both fragment reads are
// conflict-free: in A's k-column kc, chunk c (rows 2c, 2c + 1) sits in slot
// c ^ 8 (kc & 1); in B's column j, chunk c (k = 2c, 2c + 1) sits in slot
// c ^ (j & 7).
//
// Occupancy is what bounds this kernel: a workgroup takes 48 KB of LDS, so
// three fit on a compute unit (six waves per SIMD) only if a wave stays within
// 80 VGPRs.  The loads therefore address global memory as a scalar base plus a
// 32-bit lane offset, the B pairs are read one half-stage at a time, and the
// compiler is held to six waves per SIMD (76 VGPRs, no spills).  With 99 VGPRs
// (two workgroups per compute unit) the same instruction stream ran 6-8%
// slower at n = 10,000 and n = 20,000.
constexpr int DB_BM = 128, DB_BN = 64, DB_BK = 16, DB_THREADS = 512, DB_STAGES = 2;

__global__ __launch_bounds__(DB_THREADS) __attribute__((amdgpu_waves_per_eu(6, 8)))
void trmm_f64_dma_kernel(GemmArgs g) {
  constexpr int BM = DB_BM, BN = DB_BN, BK = DB_BK, NS = DB_STAGES, NW = DB_THREADS / 64;
  constexpr int WGM = BM / 64, WTN = BN / (NW / WGM), FC = WTN / 4;
  constexpr int ASZ = BM * BK * 8, BSZ = BN * BK * 8, STAGE = ASZ + BSZ;
  constexpr int AINS = ASZ / 1024;   // load instructions of A per stage, one k-column each
  static_assert(BM == 128 && BK == 16 && FC == 4 && AINS == 2 * NW && BSZ == NW * 1024, "tile split");
  static_assert(2 * 21 * BN * 8 <= NS * STAGE, "the ring holds the fused sums (p + 1 <= 21)");
  __shared__ __align__(1024) char smem[NS * STAGE];

  int ti, tj;
  const int Mt = g.M / BM, Nt = (g.ncols + BN - 1) / BN;
  if (!XcdMap::tile(g, blockIdx.x, Mt, Nt, &ti, &tj)) return;
  const int i0 = ti * BM, j0 = tj * BN;
  if (g.c_lower && (i0 + BM - 1) < (j0 + g.c_diag)) return;   // a tile wholly above the lower part
  // k range of the tile: a lower-triangular A ends at the tile's last row, an upper-triangular one starts at its
  // first, a lower-triangular B starts at the tile's first column (each holds explicit zeros across its diagonal
  // block)
  int khi = g.K;
  if (g.a_tri == TRI_LOWER) khi = imin(khi, i0 + BM);
  const int nk = (khi + BK - 1) / BK;
  int k0 = (g.a_tri == TRI_UPPER) ? i0 / BK : 0;
  if (g.b_tri == TRI_LOWER) k0 = imax(k0, j0 / BK);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WGM, wn = wave / WGM;

  // loader: this wave issues instructions wave and wave + 8 (A's k-columns) and
  // wave + 16 (B's columns 8 wave .. 8 wave + 7) of every stage
  uint32_t voff[3];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int kc = q * NW + wave;
    const int c = lane ^ ((kc & 1) << 3);
    voff[q] = (uint32_t)((2 * c + (int64_t)kc * g.lda) * 8);
  }
  {
    const int jl = 8 * wave + (lane >> 3);
    const int c = (lane & 7) ^ (jl & 7);
    const int j = imin(j0 + jl, g.ncols - 1) - j0;   // columns past the end: any valid one, dropped
    voff[2] = (uint32_t)((2 * c + (int64_t)j * g.ldb) * 8);
  }
  const double* Abase = g.A + i0;
  const double* Bbase = g.B + (int64_t)j0 * g.ldb;
  const uint32_t lds0 = lds_address(smem);
  auto issue = [&](int kstep) {
    const uint32_t base = lds0 + (uint32_t)((kstep % NS) * STAGE);
    const int kt = kstep * BK;
    const double* a = Abase + (int64_t)kt * g.lda;   // A advances kt columns, B kt rows
    const double* b = Bbase + kt;
    lds_load16_sv(a, voff[0], base + (uint32_t)(wave * 1024));
    lds_load16_sv(a, voff[1], base + (uint32_t)((NW + wave) * 1024));
    lds_load16_sv(b, voff[2], base + (uint32_t)(ASZ + wave * 1024));
  };

  double acc[4][FC];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < FC; ++c) acc[a][c] = 0.0;
  if (g.acc_cin) {   // start from alpha Cin (alpha = +-1: exact)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = i0 + wm * 64 + a * 16 + 4 * ((lane >> 2) & 3) + (lane >> 4);
#pragma unroll
      for (int c = 0; c < FC; ++c) {
        const int j = j0 + wn * WTN + c * 4 + (lane & 3);
        if (i < g.mvalid && j < g.ncols) acc[a][c] = g.alpha * g.Cin[(int64_t)i + (int64_t)j * g.ldcin];
      }
    }
  }

  // k order within a stage: MFMA s sums k = 4 (lane / 16) + s over the four lane groups (a permutation of the
  // stage's 16 k that both operands share), so a lane's four B values of a column are adjacent: two 16-byte reads
  // per column and stage instead of four 8-byte ones.  A's fragment of MFMA s, row block a sits at
  // abase + 1024 s + 128 (a ^ (s & 1)) (the chunk swizzle flips bit 0 of a on odd k).
  const int g4 = 4 * (lane >> 4);
  const int abase = g4 * (8 * BM) + wm * 512 + ((lane & 15) >> 1) * 16 + (lane & 1) * 8;

  if (k0 < nk) issue(k0);
  for (int it = k0; it < nk; ++it) {
    wait_vmcnt<0>();   // this wave's loads of stage it have landed ...
    __syncthreads();   // ... and every wave's; the other stage is free
    if (it + 1 < nk) issue(it + 1);
    const char* st = smem + (it % NS) * STAGE;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double2 bq[FC];
#pragma unroll
      for (int c = 0; c < FC; ++c) {
        const int j = wn * WTN + c * 4 + (lane & 3);
        bq[c] = *reinterpret_cast<const double2*>(st + ASZ + j * 128 + ((((g4 >> 1) + h) ^ (j & 7)) << 4));
      }
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) {
        const int s = 2 * h + s2;
        double af[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          af[a] = *reinterpret_cast<const double*>(st + abase + s * (8 * BM) + ((a ^ (s & 1)) * 128));
#pragma unroll
        for (int c = 0; c < FC; ++c) {
          const double bf = s2 ? bq[c].y : bq[c].x;
#pragma unroll
          for (int a = 0; a < 4; ++a) acc[a][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[a], bf, acc[a][c], 0, 0, 0);
        }
      }
    }
  }

  // lane holds C[4 ((lane >> 2) & 3) + (lane >> 4)][lane & 3] of each 16 x 4 slice
  if (g.red_q > 0) {
    // Per-column sums over this tile's rows instead of C: each lane sums its four rows (a ascending), a
    // butterfly over the sixteen lanes of a column adds those (every lane ends with the same sum), and the
    // two row-strip waves are added in the order wm = 0, 1.  The order depends only on the tile, so every
    // column's sums are independent of the block's width and of the column's place in it.
    __syncthreads();   // every wave is done with the ring, which now holds the two strips' sums
    double* red = reinterpret_cast<double*>(smem);   // [wm][q][64 columns]
    for (int q = 0; q < g.red_q; ++q) {
      const bool norm = q == g.red_q - 1;
      double w[4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
        w[a] = norm ? 0.0 : g.red_W[(int64_t)(i0 + wm * 64 + a * 16 + 4 * ((lane >> 2) & 3) + (lane >> 4)) +
                                   (int64_t)q * g.ld_red_W];
#pragma unroll
      for (int c = 0; c < FC; ++c) {
        double t = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) t += acc[a][c] * (norm ? acc[a][c] : w[a]);
#pragma unroll
        for (int off = 4; off < 64; off <<= 1) t += __shfl_xor(t, off, 64);
        if (lane < 4) red[(wm * g.red_q + q) * BN + wn * WTN + c * 4 + lane] = t;
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < g.red_q * BN; e += DB_THREADS) {
      const int q = e / BN, jl = e % BN;
      if (j0 + jl < g.ncols)
        g.red_part[(int64_t)(ti * g.red_q + q) * g.ncols + j0 + jl] = red[q * BN + jl] + red[(g.red_q + q) * BN + jl];
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + wm * 64 + a * 16 + 4 * ((lane >> 2) & 3) + (lane >> 4);
    if (i >= g.mvalid) continue;
#pragma unroll
    for (int c = 0; c < FC; ++c) {
      const int j = j0 + wn * WTN + c * 4 + (lane & 3);
      if (j >= g.ncols) continue;
      double val = g.alpha * acc[a][c];
      if (g.beta != 0.0 && !g.acc_cin) val += g.beta * g.Cin[(int64_t)i + (int64_t)j * g.ldcin];
      g.C[(int64_t)i + (int64_t)j * g.ldc] = val;
    }
  }
}

// Whether trmm_f64_dma_kernel applies to a product without transposes: A
// full, lower or upper triangular (diagonal offset 0), no triangular B,
// 16-byte aligned operands with even leading dimensions,
// K a multiple of 16, the rows of A up to M rounded up to 128 inside A's
// leading dimension (they are read; rows past M are not stored), and lane
// offsets within a stage (15 columns of A, 63 columns of B) below 2^32 bytes.
inline bool trmm_dma_ok(const GemmArgs& g) {
  auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  if (!al16(g.A) || !al16(g.B) || (g.lda & 1) || (g.ldb & 1)) return false;
  if (g.b_tri == TRI_UPPER || (g.b_tri == TRI_LOWER && (g.b_diag != 0 || g.a_tri != TRI_NONE)) || g.a_diag != 0)
    return false;
  if (g.M <= 0 || g.K % DB_BK || g.K <= 0 || g.ncols <= 0 || g.mvalid > g.M) return false;
  if (g.lda < (int64_t)(g.M + DB_BM - 1) / DB_BM * DB_BM || g.ldb < g.K) return false;
  if ((15 * g.lda + DB_BM) * 8 >= ((int64_t)1 << 32) || (63 * g.ldb + DB_BK) * 8 >= ((int64_t)1 << 32)) return false;
  return true;
}

// Whether a column-major B operand with K rows can feed trmm_f64_dma_kernel
// as it is (otherwise it is first copied into a buffer of that shape).
inline bool dma_b_operand_ok(const double* B, int64_t ldb, int64_t K) {
  return ((uintptr_t)B & 15) == 0 && (ldb & 1) == 0 && K % DB_BK == 0 && ldb >= K &&
         (63 * ldb + DB_BK) * 8 < ((int64_t)1 << 32);
}

}  // namespace gls
