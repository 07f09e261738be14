"""The largest workload with both forms combined (GPU, through the C-ABI):
n = 20,000, p = 8 (intercept and Gaussian covariates), blocks of 16,384, the
triangular solve in refined FP32, and the h^2 gradient of the loss
sum_i t_i^2 from the hand-written adjoint.

The SNPs are the study's first block of 16,384 and a ragged block of 1,152
(2,000,000 mod 16,384), in the same block configuration as the full study.
At this size the FP64 autograd reference is out of reach, so the checks are:
- the refined forward against the oracle on sampled SNPs (bar 1e-8);
- the adjoint's d loss / d h^2 against central differences of the CPU
  oracle's loss on the same 17,536 SNPs (step 1e-6, full re-solves including
  the Cholesky of M at h^2 +- 1e-6), and against central differences of the GPU
  loss itself, both with the gradient tolerance |FD - g| <= 1e-5 max(|FD|, |g|);
- peak device memory below half of the device's memory.
"""
import numpy as np
import pytest
import torch

from oracle import gls_oracle as O
from paper_1302_4332_amd import synth
from paper_1302_4332_amd.gls import GLSContext, GLSFunction, t2_loss

pytestmark = pytest.mark.gpu
DEV = "cuda"
PREC, SWEEPS = "fp32_ir", 2


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _loss(Phi, XL, y, X, h2, bc):
    ctx = GLSContext(Phi, h2, XL, y, block_cols=bc, precision=PREC, refine_sweeps=SWEEPS)
    outs = [ctx.block(X[j:j + bc]) for j in range(0, X.shape[0], bc)]
    b, s2, v = (torch.cat([o[i] for o in outs]) for i in range(3))
    ctx.close()
    return float(t2_loss(b, s2, v)), b


def _oracle_loss(st, h2, Xh):
    """Sum of t^2 over the SNPs of Xh (one per row) from the CPU oracle."""
    ost = O.Study(st.Phi, h2, st.XL, st.y)
    r = ost.block(Xh.T)
    assert (r["status"] == 0).all()
    return O.loss_t2(r["b"], r["sigma2"], r["v"])


@pytest.mark.timeout(1500)
def test_n20k_p8_refined_fp32_with_h2_gradient():
    w = synth.WORKLOADS["c4_n20k_p8"]
    st = synth.make_study(w)
    bc, tail = w.block_cols, w.m % w.block_cols
    cols = np.r_[np.arange(0, bc), np.arange(w.m - tail, w.m)]
    Xh = np.concatenate([st.snps(0, bc), st.snps(w.m - tail, w.m)])
    torch.cuda.reset_peak_memory_stats()
    Phi, XL, y, X = _t(st.Phi), _t(st.XL), _t(st.y), _t(Xh)
    h2 = torch.tensor(w.h2, dtype=torch.float64, device=DEV, requires_grad=True)
    b, s2, v = GLSFunction.apply(y, X, h2, Phi, XL, bc, PREC, SWEEPS)
    loss = t2_loss(b, s2, v)
    loss.backward()
    g = float(h2.grad)
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated()
    total = torch.cuda.get_device_properties(0).total_memory
    print(f"peak device memory {peak / 1e9:.1f} GB of {total / 1e9:.0f} GB", flush=True)
    assert peak < 0.5 * total

    eps = 1e-6
    lp, _ = _loss(Phi, XL, y, X, w.h2 + eps, bc)
    lm, _ = _loss(Phi, XL, y, X, w.h2 - eps, bc)
    fd = (lp - lm) / (2 * eps)
    print(f"loss {float(loss.detach()):.6e}  d/dh2 adjoint {g:.9e}  central difference {fd:.9e}", flush=True)
    assert abs(fd - g) <= 1e-5 * max(abs(fd), abs(g))

    # the same derivative from the CPU oracle: central differences of its loss
    lpo = _oracle_loss(st, w.h2 + eps, Xh)
    print("oracle loss at h2 + 1e-6 done", flush=True)
    lmo = _oracle_loss(st, w.h2 - eps, Xh)
    fdo = (lpo - lmo) / (2 * eps)
    print(f"oracle loss {0.5 * (lpo + lmo):.6e}  oracle central difference {fdo:.9e}", flush=True)
    assert abs(fdo - g) <= 1e-5 * max(abs(fdo), abs(g))

    # refined forward against the oracle on sampled SNPs of both blocks
    rng = np.random.default_rng(7)
    idx = np.unique(np.r_[0, bc - 1, bc, len(cols) - 1, rng.integers(0, len(cols), size=40)])
    ref = O.Study(st.Phi, w.h2, st.XL, st.y).block(Xh[idx].T)
    bg = b.detach().cpu().numpy()[idx]
    ok = ref["status"] == 0
    err = np.max(np.abs(bg[ok] - ref["b"][ok]), axis=1) / np.max(np.abs(ref["b"][ok]), axis=1)
    print(f"refined FP32 max rel err of b {err.max():.2e}", flush=True)
    assert err.max() <= 1e-8
    assert np.allclose(s2.detach().cpu().numpy()[idx][ok], ref["sigma2"][ok], rtol=1e-8, atol=0)
