"""GPU parity of the FP64 path against the CPU oracle, through the C-ABI.

Tolerances (plain FP64): per SNP, ||b_i - b_i,oracle||_inf / ||b_i,oracle||_inf
<= 1e-10, and relative 1e-10 on sigma2_i and v_i; status bit-exact.  Streamed
outputs (overlapped, serial, resumed, with the opening ramp) are held to the
same bar against the oracle, and are also bitwise those of the block path.
"""
import numpy as np
import pytest
import torch

from oracle import gls_oracle as O
from paper_1302_4332_amd import synth
from paper_1302_4332_amd.gls import GLSContext, GLSError
from parity_util import as_numpy, compare, slice_out

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL_B = 1e-10
TOL_S = 1e-10


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _problem(n, p, m, seed, h2=0.45, kind="gauss"):
    Phi = synth.kinship(n, seed)
    XL = synth.covariates(n, p, seed, kind) if p > 1 else np.zeros((n, 0))
    y = synth.phenotype(n, seed)
    XR = synth.genotypes(n, 0, m, seed)
    return Phi, h2, XL, y, XR


def _gpu(Phi, h2, XL, y, XR, bc, **kw):
    ctx = GLSContext(_t(Phi), h2, _t(XL) if XL.shape[1] else None, _t(y), block_cols=bc, **kw)
    X = _t(XR)
    outs = [ctx.block(X[j:j + bc]) for j in range(0, X.shape[0], bc)]
    torch.cuda.synchronize()
    return {k: torch.cat([o[i] for o in outs]).cpu().numpy() for i, k in enumerate(["b", "sigma2", "v", "status"])}


def _compare(g, r, tol_b=TOL_B, tol_s=TOL_S):
    ok = r["status"] == 0
    assert np.array_equal(g["status"], r["status"])
    err = np.max(np.abs(g["b"][ok] - r["b"][ok]), axis=1) / np.max(np.abs(r["b"][ok]), axis=1)
    assert err.max(initial=0) <= tol_b, f"max rel err b {err.max():.3e}"
    assert np.allclose(g["sigma2"][ok], r["sigma2"][ok], rtol=tol_s, atol=0)
    assert np.allclose(g["v"][ok], r["v"][ok], rtol=tol_s, atol=0)
    assert np.isnan(g["b"][~ok]).all()
    return err.max(initial=0)


def test_c0_small_full():
    st = synth.make_study("c0_small")
    XR = st.snps(0, st.w.m)
    g = _gpu(st.Phi, st.w.h2, st.XL, st.y, XR, st.w.block_cols)
    r = O.gls_sequence(st.Phi, st.w.h2, st.XL, st.y, XR)
    err = _compare(g, r)
    print(f"c0: n={st.w.n} p={st.w.p} m={st.w.m} max rel err b {err:.2e}")


@pytest.mark.parametrize("n,p,m,bc", [
    (300, 3, 700, 256),     # n not a multiple of the padding, ragged last block
    (257, 1, 130, 64),      # no covariates
    (700, 8, 333, 128),
    (520, 20, 200, 200),    # largest supported p
    (130, 2, 1, 1),         # one SNP
    (1100, 4, 517, 517),
])
def test_ragged_shapes(n, p, m, bc):
    Phi, h2, XL, y, XR = _problem(n, p, m, seed=n + p)
    if p > 1:
        XL[:, 0] = 1.0
    g = _gpu(Phi, h2, XL, y, XR, bc)
    r = O.gls_sequence(Phi, h2, XL, y, XR)
    _compare(g, r)


def test_block_size_bitwise():
    Phi, h2, XL, y, XR = _problem(600, 4, 900, seed=5)
    a = _gpu(Phi, h2, XL, y, XR, 900)
    b = _gpu(Phi, h2, XL, y, XR, 96)
    c = _gpu(Phi, h2, XL, y, XR, 7)
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True) and np.array_equal(a[k], c[k], equal_nan=True), k


def test_degenerate_snps():
    Phi, h2, XL, y, XR = _problem(400, 4, 64, seed=9)
    XL[:, 0] = 1.0
    XR[3] = 2.0                  # constant: collinear with the intercept
    XR[10] = 0.0                 # all zero
    XR[11] = 4.0 * XL[:, 1]      # a multiple of a covariate
    XR[20, 5] = np.nan           # NaN sample: only this SNP is affected
    g = _gpu(Phi, h2, XL, y, XR, 64)
    r = O.gls_sequence(Phi, h2, XL, y, XR)
    assert list(np.nonzero(g["status"])[0]) == [3, 10, 11, 20]
    assert np.isnan(g["b"][[3, 10, 11, 20]]).all()
    _compare(g, r)


def test_not_spd_reports_pivot():
    n = 300
    Phi = np.eye(n)
    Phi[137, 137] = -2.0
    XL = synth.covariates(n, 3, 1, "gauss")
    y = synth.phenotype(n, 1)
    with pytest.raises(GLSError) as e:
        GLSContext(_t(Phi), 1.0, _t(XL), _t(y), block_cols=8)
    assert e.value.status == -2 and e.value.info == 138
    with pytest.raises(O.NotSPDError) as eo:
        O.Study(Phi, 1.0, XL, y)
    assert eo.value.pivot == 138


def test_rank_deficient_covariates():
    n = 200
    Phi = synth.kinship(n, 2)
    XL = synth.covariates(n, 4, 2, "gauss")
    XL[:, 2] = 3.0 * XL[:, 1]
    with pytest.raises(GLSError) as e:
        GLSContext(_t(Phi), 0.3, _t(XL), _t(synth.phenotype(n, 2)), block_cols=8)
    assert e.value.status == -6 and e.value.info == 3


def test_argument_errors():
    st = synth.make_study("c0_small", m=8)
    ctx = GLSContext(_t(st.Phi), 0.5, _t(st.XL), _t(st.y), block_cols=8)
    with pytest.raises(GLSError) as e:
        ctx.block(_t(st.snps(0, 9)))          # mb > block_cols
    assert e.value.status == -1
    with pytest.raises(GLSError):
        GLSContext(_t(st.Phi), 1.5, _t(st.XL), _t(st.y), block_cols=8)   # h2 outside [0, 1]


def test_stream_matches_block_and_resumes():
    Phi, h2, XL, y, XR = _problem(520, 4, 1300, seed=21)
    bc = 256
    ref = _gpu(Phi, h2, XL, y, XR, bc)
    ctx = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=bc)
    host = torch.tensor(XR).pin_memory()
    (b, s2, v, st), stats = ctx.stream(host)
    assert stats.blocks == 6 and stats.h2d_bytes == 8 * 520 * 1300
    assert np.array_equal(b.numpy(), ref["b"]) and np.array_equal(s2.numpy(), ref["sigma2"])
    assert np.array_equal(v.numpy(), ref["v"]) and np.array_equal(st.numpy(), ref["status"])
    # resume: outputs for columns < col0 untouched, the rest identical
    f64 = torch.float64
    out = (torch.full((1300, 4), -7.0, dtype=f64).pin_memory(), torch.full((1300,), -7.0, dtype=f64).pin_memory(),
           torch.full((1300,), -7.0, dtype=f64).pin_memory(), torch.full((1300,), -7, dtype=torch.int32).pin_memory())
    (b2, s22, v2, st2), stats2 = ctx.stream(host, col0=700, out=out)
    assert stats2.blocks == 3
    assert (b2.numpy()[:700] == -7.0).all()
    assert np.array_equal(b2.numpy()[700:], ref["b"][700:])
    assert np.array_equal(st2.numpy()[700:], ref["status"][700:])
    # both streamed outputs against the oracle
    r = O.gls_sequence(Phi, h2, XL, y, XR)
    compare(as_numpy((b, s2, v, st)), r, TOL_B)
    compare(slice_out(as_numpy((b2, s22, v2, st2)), 700), slice_out(r, 700), TOL_B)


def test_serial_stream_equals_overlapped():
    """The no-overlap ablation gives bitwise the same results as the double-buffered stream."""
    Phi, h2, XL, y, XR = _problem(330, 4, 700, seed=23)
    host = torch.tensor(XR).pin_memory()
    a = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=128)
    b = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=128, serial_stream=True)
    (ra, _, _, sa), _ = a.stream(host)
    outb, stats = b.stream(host)
    rb, sb = outb[0], outb[3]
    assert stats.blocks == 6 and stats.h2d_bytes == 8 * 330 * 700
    assert np.array_equal(ra.numpy(), rb.numpy()) and np.array_equal(sa.numpy(), sb.numpy())
    compare(as_numpy(outb), O.gls_sequence(Phi, h2, XL, y, XR), TOL_B)


def _ramp_blocks(m, col0, bc):
    """Block count of the stream's schedule: with bc >= 2,048 it opens with
    bc / 8 and grows by a quarter per block (multiples of 64) up to bc."""
    pos, ln, k = 0, (max(64, bc // 8 // 64 * 64) if bc >= 2048 else bc), 0
    while pos < m - col0:
        pos += min(ln, m - col0 - pos)
        ln = min(bc, (ln * 5 // 4 + 63) // 64 * 64)
        k += 1
    return k


def test_stream_ramp_bitwise():
    """Large blocks: the stream opens with shorter blocks; results stay bitwise
    those of full blocks, also on resume in the middle of the ramp."""
    Phi, h2, XL, y, XR = _problem(300, 4, 9000, seed=25)
    bc = 2048
    ref = _gpu(Phi, h2, XL, y, XR, bc)
    ctx = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=bc)
    host = torch.tensor(XR).pin_memory()
    (b, s2, v, st), stats = ctx.stream(host)
    assert stats.blocks == _ramp_blocks(9000, 0, bc) == 10
    assert np.array_equal(b.numpy(), ref["b"]) and np.array_equal(s2.numpy(), ref["sigma2"])
    assert np.array_equal(v.numpy(), ref["v"]) and np.array_equal(st.numpy(), ref["status"])
    out2, stats2 = ctx.stream(host, col0=300)
    b2, st2 = out2[0], out2[3]
    assert stats2.blocks == _ramp_blocks(9000, 300, bc)
    assert np.array_equal(b2.numpy()[300:], ref["b"][300:]) and np.array_equal(st2.numpy()[300:], ref["status"][300:])
    r = O.gls_sequence(Phi, h2, XL, y, XR)
    compare(as_numpy((b, s2, v, st)), r, TOL_B)
    compare(slice_out(as_numpy(out2), 300), slice_out(r, 300), TOL_B)


def test_empty_inputs():
    """Empty blocks and streams are no-ops: mb = 0, m = 0 and col0 = m."""
    Phi, h2, XL, y, XR = _problem(260, 4, 5, seed=31)
    ctx = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=16)
    b, s2, v, st = ctx.block(_t(XR[:0]))
    assert b.shape == (0, 4) and s2.shape == (0,)
    (bs, *_), stats = ctx.stream(torch.empty((0, 260), dtype=torch.float64).pin_memory())
    assert stats.blocks == 0 and stats.h2d_bytes == 0 and bs.shape == (0, 4)
    host = torch.tensor(XR).pin_memory()
    (bs, *_), stats = ctx.stream(host, col0=5)
    assert stats.blocks == 0 and np.isnan(bs.numpy()).all()
