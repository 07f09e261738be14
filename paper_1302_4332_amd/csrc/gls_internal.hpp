// Internal state of a libgls handle and the shared host-side helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "gls.h"

namespace gls {

constexpr int PMAX = 20;    // p ranges from 4 to 20 in practice (Sec. 1.4)
constexpr int64_t NPAD = 256;  // internal row padding of every n-sized dimension

// Byte offsets of every region inside the caller's workspace.
struct Plan {
  int64_t n = 0, N = 0, bc = 0;
  int p = 0;
  size_t off_info = 0, off_small = 0, off_gram = 0;
  size_t off_L = 0, off_Linv = 0, off_W = 0, off_Xt = 0;
  size_t off_buf0 = 0, off_buf1 = 0;
  size_t off_ob = 0, off_os2 = 0, off_ov = 0, off_ost = 0;
  // mixed precision
  int lp_bytes = 0;          // element size of the low-precision type (0: plain FP64)
  int64_t bcp = 0;           // block columns rounded up to the tile width
  size_t off_Llp = 0, off_Blp = 0, off_R = 0, off_cs = 0, off_red = 0;
  // byte input
  size_t off_ub0 = 0, off_ub1 = 0, off_ubp = 0, off_x64 = 0, off_sl = 0, off_ex = 0;
  // adjoint (GLS_KEEP_FOR_GRAD)
  size_t off_Phi = 0, off_Lbar = 0, off_T1 = 0, off_T2 = 0, off_Xtb = 0, off_Xb = 0;
  size_t off_Cb = 0, off_eb = 0, off_ct = 0, off_Wb = 0, off_W0b = 0, off_acc = 0;
  // setup: scratch of the inverse-factor products that run on the side stream,
  // one region per recursion depth (offsets in doubles from off_side)
  size_t off_side = 0;
  int64_t side_at[16] = {0};
  int leaves = 0;   // NB_LEAF-row diagonal blocks factored: rows n..N-1 past them are the identity
  size_t total = 0;
};

}  // namespace gls

struct gls_ctx {
  gls::Plan plan;
  gls_opts opts{};
  int64_t n = 0, N = 0, bc = 0;
  int p = 0;
  double h2 = 0.0;
  bool ready = false;
  // device regions (inside the workspace)
  int* info = nullptr;      // [0] pivot of M, [1] pivot of S_TL
  double* small = nullptr;  // factor of S_TL and hoisted right-hand side
  double* gram = nullptr;   // [X~_L | y~]^T [X~_L | y~]  (p x p)
  double* L = nullptr;      // N x N lower Cholesky factor of M (identity padding)
  double* Linv = nullptr;   // N x N lower, L^-1
  double* W = nullptr;      // N x p, [X~_L | y~]
  double* Xt = nullptr;     // N x block_cols, X~_R of the current block (also setup scratch)
  double* buf[2] = {nullptr, nullptr};  // streaming: alpha / beta SNP blocks, n x block_cols
  double* ob = nullptr;     // streaming outputs: b (p x block_cols)
  double* os2 = nullptr;
  double* ov = nullptr;
  int* ost = nullptr;
  // mixed precision (precision != GLS_FP64)
  void* Llp = nullptr;      // N x N row-major low-precision L^-1 * 2^e
  void* Blp = nullptr;      // N x bcp low-precision right-hand sides
  double* R = nullptr;      // N x bcp FP64 refinement residuals
  double* cs = nullptr;     // bcp per-column scale factors
  double* red = nullptr;    // [0]: 2^-e of the factor; [8..]: reduction scratch
  // byte input
  uint8_t* ub[2] = {nullptr, nullptr};  // streaming staging, n x block_cols bytes
  uint8_t* ubp = nullptr;   // N x bcp packed bytes (GLS_INT8_EMU operand)
  double* x64 = nullptr;    // N x block_cols FP64: bytes widened, or a block copied with zero rows past n
  int8_t* sl = nullptr;     // OZ_SLICES x N x N int8 slices of L^-1 (GLS_INT8_EMU)
  int* ex = nullptr;        // N row exponents of L^-1 (GLS_INT8_EMU)
  // adjoint state (GLS_KEEP_FOR_GRAD)
  bool grad = false;
  double* Phi = nullptr;    // N x N, lower triangle of Phi (zero padding)
  double* Lbar = nullptr;   // N x N accumulated adjoint of L (lower part meaningful)
  double* T1 = nullptr;     // N x N scratch of the Cholesky adjoint
  double* T2 = nullptr;     // N x N scratch
  double* Xtb = nullptr;    // N x bcp adjoint of X~_R of the current block
  double* Xb = nullptr;     // N x bcp adjoint of X_R of the current block
  double* Cb = nullptr;     // p x bcp per-SNP coefficients of x~bar on [X~_L | y~]
  double* eb = nullptr;     // bcp per-SNP coefficient of x~bar on x~
  double* ct = nullptr;     // nc x bcp per-SNP shared-term contributions
  double* Wb = nullptr;     // N x p accumulated adjoint of [X~_L | y~]
  double* W0b = nullptr;    // N x p adjoint of [X_L | y]
  double* acc = nullptr;    // nc accumulated shared adjoints, then partial sums
  hipEvent_t ev_copy[2] = {nullptr, nullptr};
  hipEvent_t ev_comp[2] = {nullptr, nullptr};
  // the handle's own compute and copy streams for streamed studies, and the
  // event that orders them after the caller's stream
  hipStream_t own_st[2] = {nullptr, nullptr};
  hipEvent_t ev_join = nullptr;
  // phase timing (gls_profile_*)
  struct ProfRec {
    int phase;
    hipEvent_t a, b;
  };
  bool prof_on = false;
  std::vector<ProfRec> prof_pending;
  std::vector<hipEvent_t> prof_free;
  int64_t prof_n[GLS_NUM_PHASES] = {0, 0, 0, 0};
  double prof_ms[GLS_NUM_PHASES] = {0, 0, 0, 0};
};

namespace gls {

using Ctx = gls_ctx;

enum { PH_WHITEN = 0, PH_RESIDUAL = 1, PH_SNP = 2, PH_BACKWARD = 3 };

// Records an event pair around a phase on stream s when profiling is on.
class PhaseTimer {
 public:
  PhaseTimer(Ctx* c, int phase, hipStream_t s);
  ~PhaseTimer();

 private:
  Ctx* c_;
  int phase_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr;
};

gls_status hip_fail(hipError_t e, const char* what);
gls_status arg_fail(const char* what);
void set_last_error_str(const char* what);
int64_t padded_n(int64_t n);
bool plan_workspace(int64_t n, int32_t p, const gls_opts* o, Plan* pl);

void whiten_fp64(Ctx* c, const double* X, int64_t ldx, int mb, int K, int rows, double* Xt, hipStream_t s);
void prepare_low_precision(Ctx* c, hipStream_t s);
void reset_adjoint(Ctx* c, hipStream_t s);
void snp_reduce_solve(Ctx* c, const double* Xt, int mb, double* b, int64_t ldb, double* s2, double* v, int* st,
                      hipStream_t s);
gls_status block_forward(Ctx* c, int mb, const double* XR, int64_t ld_xr, double* b, int64_t ld_b, double* s2,
                         double* v, int* st, hipStream_t s);
gls_status block_forward_u8(Ctx* c, int mb, const uint8_t* G, int64_t ldg, double* b, int64_t ld_b, double* s2,
                            double* v, int* st, hipStream_t s);
gls_status block_forward_u2(Ctx* c, int mb, const uint8_t* G2, int64_t ldg, double* b, int64_t ld_b, double* s2,
                            double* v, int* st, hipStream_t s);
gls_status block_backward(Ctx* c, int mb, const double* XR, int64_t ld_xr, const double* bbar, const double* s2bar,
                          const double* vbar, double* XR_grad, hipStream_t s);
void widen_u8(Ctx* c, const uint8_t* G, int64_t ldg, int mb, hipStream_t s);
void widen_u2(Ctx* c, const uint8_t* G2, int64_t ldg, int mb, hipStream_t s);

}  // namespace gls
