// FP64 product C = alpha op(A) B + beta Cin for the per-block solve
// X~ = L^-1 X and the refinement residual X - L X~ (also the setup's panel and
// trailing products and the adjoint's L-bar update): A column-major and lower
// triangular (or full), B column-major, C column-major, optionally only the
// tiles that reach C's lower part.  The same
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
// gemm_f64_kernel).  Permuting k saves half of the B fragment reads: 5% at
// n = 10,000 (13.3 instead of 14.0 ms per 8,192-SNP launch).  A stage is 16 KB of A (16 k-columns of 128 rows, one
// 1 KB load instruction each) and 8 KB of B (64 columns of 16 k, eight
// columns per instruction), in a ring of two stages that leaves room for
// several workgroups per CU.  16-byte chunks are placed so that both fragment reads
// are conflict-free: in A's k-column kc, chunk c (rows 2c, 2c + 1) sits in
// slot c ^ 8 (kc & 1); in B's column j, chunk c (k = 2c, 2c + 1) sits in slot
// c ^ (j & 7).  Two stages (48 KB) were measured best at n = 10,000 (three:
// 3% slower, four: 15% slower; XCD groups other than 1 x 16 slower still); a
// 64 x 64 tile with four waves (two k-columns of A per load instruction) runs
// within 0.3% of this one.
constexpr int DB_BM = 128, DB_BN = 64, DB_BK = 16, DB_THREADS = 512, DB_STAGES = 2;

__global__ __launch_bounds__(DB_THREADS) void trmm_f64_dma_kernel(GemmArgs g) {
  constexpr int BM = DB_BM, BN = DB_BN, BK = DB_BK, NS = DB_STAGES, NW = DB_THREADS / 64;
  constexpr int WGM = BM / 64, WGN = NW / WGM;   // waves along rows (64 each) and columns
  constexpr int WTN = BN / WGN, FC = WTN / 4;    // columns per wave, 4-column accumulator slices per wave
  constexpr int ASZ = BM * BK * 8, BSZ = BN * BK * 8, STAGE = ASZ + BSZ;
  constexpr int AINS = ASZ / 1024;               // load instructions of A per stage (1024 / (8 BM) k-columns each)
  constexpr int KPI = BK / AINS;
  constexpr int NLD = (ASZ + BSZ) / 1024 / NW;   // load instructions per wave and stage
  static_assert(NLD * NW * 1024 == STAGE && (BM == 128 || BM == 64) && (FC == 4 || FC == 8) && BK == 16, "tile split");
  __shared__ __align__(1024) char smem[NS * STAGE];

  int ti, tj;
  const int Mt = g.M / BM, Nt = (g.ncols + BN - 1) / BN;
  if (!XcdMap::tile(g, blockIdx.x, Mt, Nt, &ti, &tj)) return;
  const int i0 = ti * BM, j0 = tj * BN;
  if (g.c_lower && (i0 + BM - 1) < (j0 + g.c_diag)) return;   // a tile wholly above the lower part
  int khi = g.K;
  if (g.a_tri == TRI_LOWER) khi = imin(khi, i0 + BM + g.a_diag);
  const int nk = (khi + BK - 1) / BK;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % WGM, wn = wave / WGM;

  // loader: this wave issues instructions wave, wave + 8, wave + 16 of a stage
  // (0..15: A's k-columns, 16..23: B's column groups of eight)
  const char* src[NLD];
  int dst[NLD];
#pragma unroll
  for (int q = 0; q < NLD; ++q) {
    const int ins = q * NW + wave;
    if (ins < AINS) {
      // k-columns KPI ins .. KPI ins + KPI - 1, BM / 2 chunks (two rows each) per column
      const int kc = KPI * ins + lane / (BM / 2), slot = lane % (BM / 2);
      const int c = slot ^ ((kc & 1) << 3);
      src[q] = reinterpret_cast<const char*>(g.A + (int64_t)(i0 + 2 * c) + (int64_t)kc * g.lda);
      dst[q] = ins * 1024;
    } else {
      const int jl = 8 * (ins - AINS) + (lane >> 3);
      const int c = (lane & 7) ^ (jl & 7);
      const int j = imin(j0 + jl, g.ncols - 1);   // columns past the end: any valid one, dropped
      src[q] = reinterpret_cast<const char*>(g.B + (int64_t)(2 * c) + (int64_t)j * g.ldb);
      dst[q] = ASZ + (ins - AINS) * 1024;
    }
  }
  const uint32_t lds0 = lds_address(smem);
  auto issue = [&](int kstep) {
    const uint32_t base = lds0 + (uint32_t)((kstep % NS) * STAGE);
    const int kt = kstep * BK;
#pragma unroll
    for (int q = 0; q < NLD; ++q) {
      const int ins = q * NW + wave;
      // A advances kt columns (kt * lda doubles), B kt rows
      const int64_t step = (ins < AINS) ? (int64_t)kt * g.lda * 8 : (int64_t)kt * 8;
      lds_load16(src[q] + step, __builtin_amdgcn_readfirstlane(base + dst[q]));
    }
  };

  double acc[4][FC];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < FC; ++c) acc[a][c] = 0.0;

  // k order within a stage: MFMA s sums k = 4 (lane / 16) + s over the four lane groups (a permutation of the
  // stage's 16 k that both operands share), so a lane's four B values of a column are adjacent: two 16-byte reads
  // per column and stage instead of four 8-byte ones
  const int g4 = 4 * (lane >> 4);
  int offa[4][4], offb[FC][2];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int kr = g4 + s;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int i = wm * 64 + a * 16 + (lane & 15);
      offa[s][a] = kr * (8 * BM) + (((i >> 1) ^ ((kr & 1) << 3)) << 4) + ((i & 1) << 3);
    }
  }
#pragma unroll
  for (int c = 0; c < FC; ++c) {
    const int j = wn * WTN + c * 4 + (lane & 3);
#pragma unroll
    for (int h = 0; h < 2; ++h) offb[c][h] = ASZ + j * 128 + ((((g4 >> 1) + h) ^ (j & 7)) << 4);
  }

  for (int q = 0; q < NS - 1; ++q)
    if (q < nk) issue(q);
  for (int it = 0; it < nk; ++it) {
    wait_stages<NLD>(min(nk - 1 - it, NS - 2));   // this wave's loads of stage it have landed ...
    __syncthreads();                              // ... and every wave's; stage (it - 1) % NS is free
    if (it + NS - 1 < nk) issue(it + NS - 1);
    const char* st = smem + (it % NS) * STAGE;
    double2 bq[FC][2];
#pragma unroll
    for (int c = 0; c < FC; ++c)
#pragma unroll
      for (int h = 0; h < 2; ++h) bq[c][h] = *reinterpret_cast<const double2*>(st + offb[c][h]);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double af[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) af[a] = *reinterpret_cast<const double*>(st + offa[s][a]);
#pragma unroll
      for (int c = 0; c < FC; ++c) {
        const double bf = (s & 1) ? bq[c][s >> 1].y : bq[c][s >> 1].x;
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[a][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[a], bf, acc[a][c], 0, 0, 0);
      }
    }
  }

  // lane holds C[4 ((lane >> 2) & 3) + (lane >> 4)][lane & 3] of each 16 x 4 slice
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int i = i0 + wm * 64 + a * 16 + 4 * ((lane >> 2) & 3) + (lane >> 4);
    if (i >= g.mvalid) continue;
#pragma unroll
    for (int c = 0; c < FC; ++c) {
      const int j = j0 + wn * WTN + c * 4 + (lane & 3);
      if (j >= g.ncols) continue;
      double val = g.alpha * acc[a][c];
      if (g.beta != 0.0) val += g.beta * g.Cin[(int64_t)i + (int64_t)j * g.ldcin];
      g.C[(int64_t)i + (int64_t)j * g.ldc] = val;
    }
  }
}

// Whether trmm_f64_dma_kernel applies to a product without transposes: no
// triangular B, 16-byte aligned operands with even leading dimensions,
// K a multiple of 16, and the rows of A up to M rounded up to 128 inside A's
// leading dimension (they are read; rows past M are not stored).
inline bool trmm_dma_ok(const GemmArgs& g) {
  auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  if (!al16(g.A) || !al16(g.B) || (g.lda & 1) || (g.ldb & 1)) return false;
  if (g.b_tri != TRI_NONE || (g.a_tri != TRI_NONE && g.a_tri != TRI_LOWER)) return false;
  if (g.a_tri == TRI_LOWER && g.a_diag != 0) return false;
  if (g.M <= 0 || g.K % DB_BK || g.K <= 0 || g.ncols <= 0 || g.mvalid > g.M) return false;
  if (g.lda < (int64_t)(g.M + DB_BM - 1) / DB_BM * DB_BM || g.ldb < g.K) return false;
  return true;
}

}  // namespace gls
