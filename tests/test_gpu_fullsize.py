"""GPU parity at the full study sizes, in the launch configuration bench.py
times (same block sizes, full blocks and the study's real ragged tail), on
sampled SNPs that the CPU oracle solves one by one.

- n = 10,000, p = 4 (sex/age covariates, causal SNP), blocks of 8,192: the
  first block and the last (1,696 SNPs: 100,000 mod 8,192), FP64 path and the
  int8-slice path on the same SNPs as bytes and as packed 2-bit dosages;
- n = 10,000, p = 4, m = 1,000,000 (no causal SNP), blocks of 8,192: the first
  block and the last (576 SNPs), in the refined mixed forms (FP32 one sweep;
  FP16 two and three; BF16 three and four: the fewest sweeps that meet the bar
  and the counts that reach the FP64 level);
- n = 20,000, p = 8 (Gaussian covariates), blocks of 16,384: the first block and
  a ragged block of 1,152 (2,000,000 mod 16,384);
- n = 10,007 (not a multiple of the product's 16-deep k step, odd leading
  dimension), otherwise the n = 10,000 study: the first block and the last
  (1,696 SNPs), plain FP64 (the block is first copied into a zero-padded
  buffer so that the direct-load product applies) and refined FP32.

Bar: per SNP ||b - b_oracle||_inf / ||b_oracle||_inf <= 1e-10 for the plain
FP64 and int8-slice paths, 1e-8 for the refined forms; sigma2 and v relative
to the same bar; status equal.
"""
import numpy as np
import pytest
import torch

from oracle import gls_oracle as O
from paper_1302_4332_amd import synth
from paper_1302_4332_amd.gls import GLSContext

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = {"fp64": 1e-10, "int8_emu": 1e-10, "fp32_ir": 1e-8, "fp16_ir": 1e-8, "bf16_ir": 1e-8}


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _check(g, r, tol):
    assert np.array_equal(g["status"], r["status"])
    ok = r["status"] == 0
    err = np.max(np.abs(g["b"][ok] - r["b"][ok]), axis=1) / np.max(np.abs(r["b"][ok]), axis=1)
    assert err.max() <= tol, f"max rel err b {err.max():.3e}"
    assert np.allclose(g["sigma2"][ok], r["sigma2"][ok], rtol=tol, atol=0)
    assert np.allclose(g["v"][ok], r["v"][ok], rtol=tol, atol=0)
    return float(err.max())


def _study_blocks(name, tail, n=None):
    w = synth.WORKLOADS[name]
    st = synth.make_study(w, n=n) if n else synth.make_study(w)
    bc = w.block_cols
    first = (0, bc)
    last = (w.m - tail, w.m)
    assert (w.m - tail) % bc == 0   # the study's own last block
    return w, st, bc, [first, last]


def _sample(j0, j1, k, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.r_[j0, j1 - 1, rng.integers(j0, j1, size=k)])


def _run(name, tail, forms, k=48, n=None):
    """forms: (precision, refinement sweeps, input) with input "f64", "u8" or "u2"."""
    w, st, bc, blocks = _study_blocks(name, tail, n)
    print(f"{name}: n={st.Phi.shape[0]} p={w.p} blocks {blocks}", flush=True)
    ost = O.Study(st.Phi, w.h2, st.XL, st.y)
    Phi, XL, y = _t(st.Phi), _t(st.XL), _t(st.y)
    errs = {}
    for prec, sweeps, inp in forms:
        ctx = GLSContext(Phi, w.h2, XL, y, block_cols=bc, precision=prec, refine_sweeps=sweeps)
        for bi, (j0, j1) in enumerate(blocks):
            if inp == "u8":
                b, s2, v, status = ctx.block_u8(_t(st.snps_u8(j0, j1)))
            elif inp == "u2":
                b, s2, v, status = ctx.block_u2(_t(st.snps_u2(j0, j1)))
            else:
                b, s2, v, status = ctx.block(_t(st.snps(j0, j1)))
            torch.cuda.synchronize()
            idx = _sample(j0, j1, k, 100 + bi)
            if st.causal is not None and j0 <= st.causal < j1:
                idx = np.unique(np.r_[idx, st.causal])
            g = {"b": b.cpu().numpy()[idx - j0], "sigma2": s2.cpu().numpy()[idx - j0],
                 "v": v.cpu().numpy()[idx - j0], "status": status.cpu().numpy()[idx - j0]}
            cols = np.concatenate([st.snps(int(j), int(j) + 1) for j in idx])
            r = ost.block(cols.T)
            errs[(f"{prec}x{sweeps}/{inp}", bi)] = _check(g, r, TOL[prec])
        ctx.close()
    print({f"{p}/{b}": f"{e:.1e}" for (p, b), e in errs.items()}, flush=True)


def test_fullsize_n10k_fp64_and_int8_slices():
    _run("c1_n10k_m100k", 100000 % 8192, (("fp64", 0, "f64"), ("int8_emu", 0, "u8"), ("int8_emu", 0, "u2")))


def test_fullsize_n10k_m1M_mixed():
    _run("c2_n10k_m1M", 1000000 % 8192, (("fp32_ir", 1, "f64"), ("fp16_ir", 2, "f64"), ("fp16_ir", 3, "f64"),
                                         ("bf16_ir", 3, "f64"), ("bf16_ir", 4, "f64")))


def test_fullsize_n20k_p8_fp64():
    _run("c4_n20k_p8", 2000000 % 16384, (("fp64", 0, "f64"),))


def test_fullsize_n10007_fp64_and_refined():
    _run("c1_n10k_m100k", 100000 % 8192, (("fp64", 0, "f64"), ("fp32_ir", 1, "f64")), n=10007)
