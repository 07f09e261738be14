"""Genotype-byte input (GPU, through the C-ABI).

FP64 handles: byte input widened on the device gives bitwise the results of
FP64 input.  GLS_INT8_EMU: the product as exact int8 slice products on the
integer matrix cores, held to the plain-FP64 bar against the oracle
(max relative error of b <= 1e-10, sigma2 and v relative 1e-10).
"""
import numpy as np
import pytest
import torch

from oracle import gls_oracle as O
from paper_1302_4332_amd import synth
from paper_1302_4332_amd.gls import GLSContext
from parity_util import as_numpy, compare

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _inputs(n, p, m, seed, kind="gauss"):
    Phi = synth.kinship(n, seed)
    XL = synth.covariates(n, p, seed, kind)
    if p > 1:
        XL[:, 0] = 1.0
    y = synth.phenotype(n, seed)
    G = synth.genotypes_u8(n, 0, m, seed)
    return Phi, XL, y, G


def _run_u8(ctx, G, bc):
    Gd = _t(G)
    outs = [ctx.block_u8(Gd[j:j + bc]) for j in range(0, Gd.shape[0], bc)]
    torch.cuda.synchronize()
    return {k: torch.cat([o[i] for o in outs]).cpu().numpy() for i, k in enumerate(["b", "sigma2", "v", "status"])}


def _err(g, r):
    ok = r["status"] == 0
    return float(np.max(np.max(np.abs(g["b"][ok] - r["b"][ok]), axis=1) / np.max(np.abs(r["b"][ok]), axis=1)))


def test_bytes_fp64_bitwise_equal_to_double_input():
    Phi, XL, y, G = _inputs(420, 4, 300, 3)
    ctx = GLSContext(_t(Phi), 0.4, _t(XL), _t(y), block_cols=128)
    a = _run_u8(ctx, G, 128)
    X = _t(G.astype(np.float64))
    outs = [ctx.block(X[j:j + 128]) for j in range(0, 300, 128)]
    b = {k: torch.cat([o[i] for o in outs]).cpu().numpy() for i, k in enumerate(["b", "sigma2", "v", "status"])}
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("n,p,m,bc,h2", [(512, 4, 2048, 2048, 0.5), (300, 3, 333, 100, 0.45), (1100, 8, 257, 257, 0.3),
                                          (257, 1, 70, 64, 0.6), (2900, 4, 1000, 1000, 0.4)])
def test_int8_emulation_matches_oracle(n, p, m, bc, h2):
    Phi, XL, y, G = _inputs(n, p, m, n + p, "gauss" if p != 4 else "sex_age")
    ctx = GLSContext(_t(Phi), h2, _t(XL) if p > 1 else None, _t(y), block_cols=bc, precision="int8_emu")
    g = _run_u8(ctx, G, bc)
    r = O.gls_sequence(Phi, h2, XL, y, G.astype(np.float64))
    assert np.array_equal(g["status"], r["status"])
    err = _err(g, r)
    ok = r["status"] == 0
    assert err <= 1e-10, err
    assert np.allclose(g["sigma2"][ok], r["sigma2"][ok], rtol=1e-10, atol=0)
    assert np.allclose(g["v"][ok], r["v"][ok], rtol=1e-10, atol=0)
    print(f"int8 emulation n={n} p={p}: max rel err b {err:.2e}")


def test_int8_emulation_block_independent_and_streamed():
    Phi, XL, y, G = _inputs(600, 4, 700, 8, "sex_age")
    ctx = GLSContext(_t(Phi), 0.4, _t(XL), _t(y), block_cols=256, precision="int8_emu")
    a = _run_u8(ctx, G, 256)
    b = _run_u8(ctx, G, 64)
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    (bs, s2, v, st), stats = ctx.stream(torch.tensor(G).pin_memory())
    assert stats.h2d_bytes == 600 * 700
    assert np.array_equal(bs.numpy(), a["b"]) and np.array_equal(st.numpy(), a["status"])
    compare(as_numpy((bs, s2, v, st)), O.gls_sequence(Phi, 0.4, XL, y, G.astype(np.float64)), 1e-10)


def test_bytes_stream_fp64_equals_double_stream():
    Phi, XL, y, G = _inputs(330, 4, 500, 12, "sex_age")
    ctx = GLSContext(_t(Phi), 0.4, _t(XL), _t(y), block_cols=128)
    out1, s1 = ctx.stream(torch.tensor(G).pin_memory())
    (b2, *_), s2 = ctx.stream(torch.tensor(G.astype(np.float64)).pin_memory())
    assert s1.h2d_bytes * 8 == s2.h2d_bytes
    assert np.array_equal(out1[0].numpy(), b2.numpy(), equal_nan=True)
    compare(as_numpy(out1), O.gls_sequence(Phi, 0.4, XL, y, G.astype(np.float64)), 1e-10)
