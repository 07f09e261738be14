"""GPU parity at the edges of the method's inputs (through the C-ABI).

- h2 at the ends of its range with the kinship Phi (Eq. 1 with
  M = h2 Phi + (1 - h2) I): h2 = 0 (M = I, ordinary least squares), 0.95 and
  1.0 (M = Phi).  With n = 2,304 samples and Phi built from 2,000 markers, Phi
  has rank 2,000 plus its 1e-3 ridge, so at h2 = 1 the condition number of M
  is about 4e3 (about 65 for L): the explicit-inverse product and the
  low-precision refinement are least safe here.
- The int8-slice product on genotype bytes at the same three h2 values, to
  the plain-FP64 bar.
- Non-integer SNP values (imputed-style dosages x + U(-0.5, 0.5), and
  standardized genotypes): the FP16/BF16 first solve is no longer exact on them.

Bars, per SNP against the oracle: ||b - b_oracle||_inf / ||b_oracle||_inf <=
1e-10 for plain FP64, <= 1e-8 for the refined forms after the sweep count
given for that case (sigma2 and v relative to the same bar, status equal);
refinement errors may not grow from one sweep to the next.
"""
import numpy as np
import pytest
import torch

from oracle import gls_oracle as O
from paper_1302_4332_amd import synth
from paper_1302_4332_amd.gls import GLSContext
from parity_util import compare

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _run(Phi, h2, XL, y, XR, bc, precision, sweeps):
    ctx = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=bc, precision=precision, refine_sweeps=sweeps)
    X = _t(XR)
    outs = [ctx.block(X[j:j + bc]) for j in range(0, X.shape[0], bc)]
    torch.cuda.synchronize()
    ctx.close()
    return {k: torch.cat([o[i] for o in outs]).cpu().numpy() for i, k in enumerate(["b", "sigma2", "v", "status"])}


def _err(g, r):
    assert np.array_equal(g["status"], r["status"])
    ok = r["status"] == 0
    return float(np.max(np.max(np.abs(g["b"][ok] - r["b"][ok]), axis=1) / np.max(np.abs(r["b"][ok]), axis=1)))


def _sweep_errors(Phi, h2, XL, y, XR, bc, precision, r):
    errs = [_err(_run(Phi, h2, XL, y, XR, bc, precision, k), r) for k in range(5)]
    print(f"h2={h2} {precision}: " + " ".join(f"{e:.1e}" for e in errs), flush=True)
    return errs


def _contracts(errs):
    for a, b in zip(errs, errs[1:]):
        assert b <= max(a, 1e-12) * 1.5, errs


# sweeps after which each refined form meets 1e-8, per h2 (measured on MI355X)
EDGE_SWEEPS = {0.0: {"fp32_ir": 1, "fp16_ir": 2, "bf16_ir": 3},
               0.95: {"fp32_ir": 1, "fp16_ir": 3, "bf16_ir": 4},
               1.0: {"fp32_ir": 1, "fp16_ir": 3, "bf16_ir": 4}}


@pytest.fixture(scope="module")
def kin2304():
    n, p, m = 2304, 4, 300
    Phi = synth.kinship(n, 2304)
    XL = synth.covariates(n, p, 2304, "sex_age")
    y = synth.phenotype(n, 2304)
    XR = synth.genotypes(n, 0, m, 2304)
    return Phi, XL, y, XR


@pytest.mark.parametrize("h2", [0.0, 0.95, 1.0])
def test_h2_edges_fp64(kin2304, h2):
    Phi, XL, y, XR = kin2304
    r = O.gls_sequence(Phi, h2, XL, y, XR)
    g = _run(Phi, h2, XL, y, XR, 128, "fp64", 0)
    err = compare(g, r, 1e-10)
    print(f"h2={h2} fp64: max rel err b {err:.1e}")
    if h2 == 0.0:   # M = I: ordinary least squares of [X_L | x_i] on y
        for i in (0, 137, 299):
            Xi = np.c_[XL, XR[i]]
            ols = np.linalg.lstsq(Xi, y, rcond=None)[0]
            assert np.max(np.abs(g["b"][i] - ols)) <= 1e-10 * np.max(np.abs(ols))


@pytest.mark.parametrize("precision", ["fp32_ir", "fp16_ir", "bf16_ir"])
@pytest.mark.parametrize("h2", [0.0, 0.95, 1.0])
def test_h2_edges_refined(kin2304, h2, precision):
    Phi, XL, y, XR = kin2304
    r = O.gls_sequence(Phi, h2, XL, y, XR)
    errs = _sweep_errors(Phi, h2, XL, y, XR, 128, precision, r)
    _contracts(errs)
    k = EDGE_SWEEPS[h2][precision]
    g = _run(Phi, h2, XL, y, XR, 128, precision, k)
    compare(g, r, 1e-8)


@pytest.mark.parametrize("h2", [0.0, 0.95, 1.0])
def test_h2_edges_int8_slices(kin2304, h2):
    """The int8-slice product at the ends of h2: only the slicing of L^-1 (below
    2^-56 of each row's largest entry) differs from FP64, so the plain-FP64 bar
    holds, and at h2 = 0 (L^-1 = I, one nonzero slice per row) the results are
    the ordinary least-squares ones."""
    Phi, XL, y, XR = kin2304
    r = O.gls_sequence(Phi, h2, XL, y, XR)
    G = torch.tensor(XR.astype(np.uint8), device=DEV)
    ctx = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=128, precision="int8_emu")
    outs = [ctx.block_u8(G[j:j + 128]) for j in range(0, G.shape[0], 128)]
    torch.cuda.synchronize()
    ctx.close()
    g = {k: torch.cat([o[i] for o in outs]).cpu().numpy() for i, k in enumerate(["b", "sigma2", "v", "status"])}
    err = compare(g, r, 1e-10)
    print(f"h2={h2} int8 slices: max rel err b {err:.1e}")
    if h2 == 0.0:
        for i in (0, 137, 299):
            ols = np.linalg.lstsq(np.c_[XL, XR[i]], y, rcond=None)[0]
            assert np.max(np.abs(g["b"][i] - ols)) <= 1e-10 * np.max(np.abs(ols))


# sweeps after which each refined form meets 1e-8 on non-integer SNP values
REAL_SWEEPS = {"fp32_ir": 1, "fp16_ir": 3, "bf16_ir": 4}


@pytest.mark.parametrize("kind", ["jitter", "standardized"])
def test_non_integer_snps(kind):
    n, p, m, bc = 700, 4, 333, 128
    Phi = synth.kinship(n, 70)
    XL = synth.covariates(n, p, 70, "sex_age")
    y = synth.phenotype(n, 70)
    XR = synth.imputed_dosages(n, 0, m, 70, kind)
    h2 = 0.5
    r = O.gls_sequence(Phi, h2, XL, y, XR)
    err = compare(_run(Phi, h2, XL, y, XR, bc, "fp64", 0), r, 1e-10)
    print(f"{kind} fp64: max rel err b {err:.1e}")
    for prec, k in REAL_SWEEPS.items():
        errs = _sweep_errors(Phi, h2, XL, y, XR, bc, prec, r)
        _contracts(errs)
        assert errs[0] > 1e-12            # the first solve is genuinely low precision
        compare(_run(Phi, h2, XL, y, XR, bc, prec, k), r, 1e-8)


def test_non_integer_snps_full_size_sample():
    """n = 10,000 (the headline shape), 512 imputed-style SNPs: plain FP64 and
    refined FP32 (one sweep) against the oracle."""
    w = synth.WORKLOADS["c1_n10k_m100k"]
    st = synth.make_study(w)
    XR = synth.imputed_dosages(w.n, 0, 512, w.seed)
    r = O.Study(st.Phi, w.h2, st.XL, st.y).block(XR.T)
    compare(_run(st.Phi, w.h2, st.XL, st.y, XR, 512, "fp64", 0), r, 1e-10)
    compare(_run(st.Phi, w.h2, st.XL, st.y, XR, 512, "fp32_ir", 1), r, 1e-8)
