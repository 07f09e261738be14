"""Packed 2-bit dosages (GPU, through the C-ABI): four samples to a byte,
expanded on the device.  The expansion is exact, so results must be bitwise
those of the byte entry points on the same dosages, for FP64, refined and
int8-slice handles.  Pad bits of a column's last byte are ignored and the
column stride may exceed a column.  The oracle bar (max relative error of b
<= 1e-10, sigma2 and v relative 1e-10, status equal) is checked directly on a
block, on the in-memory and file streams and on a resumed stream."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import gls_oracle as O
from paper_1302_4332_amd import synth
from paper_1302_4332_amd.gls import GLSContext, GLSError, lib
from parity_util import as_numpy, compare, slice_out

pytestmark = pytest.mark.gpu
DEV = "cuda"
KEYS = ["b", "sigma2", "v", "status"]


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _inputs(n, p, m, seed):
    Phi = synth.kinship(n, seed)
    XL = synth.covariates(n, p, seed, "sex_age" if p == 4 else "gauss")
    y = synth.phenotype(n, seed)
    G = synth.genotypes_u8(n, 0, m, seed)
    G[::7, ::5] = 3                       # the fourth code is a dosage too
    return Phi, XL, y, G


def _packed_wide(G, extra):
    """Packed columns at a stride of ceil(n/4) + extra bytes, with every pad bit
    and pad byte set to ones."""
    m, n = G.shape
    q = (n + 3) // 4
    P = synth.pack_dosages_2bit(G)
    out = np.full((m, q + extra), 0xFF, dtype=np.uint8)
    out[:, :q] = P
    r = n % 4
    if r:
        out[:, q - 1] |= np.uint8((0xFF << (2 * r)) & 0xFF)
    return out


def _collect(outs):
    torch.cuda.synchronize()
    return {k: torch.cat([o[i] for o in outs]).cpu().numpy() for i, k in enumerate(KEYS)}


def _run_u8(ctx, G, bc):
    Gd = _t(G)
    return _collect([ctx.block_u8(Gd[j:j + bc]) for j in range(0, Gd.shape[0], bc)])


def _run_u2_raw(ctx, W, bc):
    """gls_block_u2 called directly, with the stride W.shape[1] >= ceil(n/4)."""
    Wd = _t(W)
    outs = []
    for j in range(0, Wd.shape[0], bc):
        blk = Wd[j:j + bc]
        mb = blk.shape[0]
        o = ctx._outputs(mb, Wd.device)
        st = lib().gls_block_u2(ctx.handle, mb, ctypes.c_void_p(blk.data_ptr()), Wd.shape[1],
                                ctypes.c_void_p(o[0].data_ptr()), ctx.p, ctypes.c_void_p(o[1].data_ptr()),
                                ctypes.c_void_p(o[2].data_ptr()), ctypes.c_void_p(o[3].data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == 0, lib().gls_last_error()
        outs.append(o)
    return _collect(outs)


@pytest.mark.parametrize("precision,sweeps", [("fp64", 0), ("int8_emu", 0), ("fp32_ir", 1)])
@pytest.mark.parametrize("n", [330, 257, 512])
def test_block_u2_bitwise_equals_bytes(precision, sweeps, n):
    Phi, XL, y, G = _inputs(n, 4, 300, n)
    ctx = GLSContext(_t(Phi), 0.4, _t(XL), _t(y), block_cols=128, precision=precision, refine_sweeps=sweeps)
    a = _run_u8(ctx, G, 128)
    b = _run_u2_raw(ctx, _packed_wide(G, 3), 128)
    Gp = _t(synth.pack_dosages_2bit(G))
    c = _collect([ctx.block_u2(Gp[j:j + 100]) for j in range(0, 300, 100)])
    for k in KEYS:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
        assert np.array_equal(a[k], c[k], equal_nan=True), k


def test_block_u2_int8_matches_oracle():
    n, p, m = 2901, 4, 512
    Phi, XL, y, G = _inputs(n, p, m, 77)
    ctx = GLSContext(_t(Phi), 0.4, _t(XL), _t(y), block_cols=m, precision="int8_emu")
    g = _collect([ctx.block_u2(_t(synth.pack_dosages_2bit(G)))])
    r = O.gls_sequence(Phi, 0.4, XL, y, G.astype(np.float64))
    assert np.array_equal(g["status"], r["status"])
    ok = r["status"] == 0
    err = float(np.max(np.max(np.abs(g["b"][ok] - r["b"][ok]), axis=1) / np.max(np.abs(r["b"][ok]), axis=1)))
    assert err <= 1e-10, err
    assert np.allclose(g["sigma2"][ok], r["sigma2"][ok], rtol=1e-10, atol=0)
    assert np.allclose(g["v"][ok], r["v"][ok], rtol=1e-10, atol=0)


@pytest.mark.parametrize("precision", ["fp64", "int8_emu"])
def test_stream_u2_equals_bytes_stream(precision):
    n, m = 331, 700
    Phi, XL, y, G = _inputs(n, 4, m, 5)
    ctx = GLSContext(_t(Phi), 0.4, _t(XL), _t(y), block_cols=256, precision=precision)
    (b8, s8, v8, t8), st8 = ctx.stream(torch.tensor(G).pin_memory())
    (b2, s2, v2, t2), st2 = ctx.stream(torch.tensor(synth.pack_dosages_2bit(G)).pin_memory(), packed=True)
    assert st2.h2d_bytes == ((n + 3) // 4) * m and st8.h2d_bytes == n * m
    for x, z in ((b8, b2), (s8, s2), (v8, v2), (t8, t2)):
        assert np.array_equal(x.numpy(), z.numpy(), equal_nan=True)
    compare(as_numpy((b2, s2, v2, t2)), O.gls_sequence(Phi, 0.4, XL, y, G.astype(np.float64)), 1e-10)


@pytest.mark.parametrize("serial", [False, True])
def test_file_stream_u2_equals_bytes(tmp_path, serial):
    n, m = 330, 1000
    Phi, XL, y, G = _inputs(n, 4, m, 31)
    f2 = str(tmp_path / "x.u2")
    with open(f2, "wb") as f:
        f.write(b"\xff" * 7)                        # a header the offset skips
        f.write(synth.pack_dosages_2bit(G).tobytes())
    ctx = GLSContext(_t(Phi), 0.4, _t(XL), _t(y), block_cols=96, serial_stream=serial)
    (ref_b, _, _, ref_st), _ = ctx.stream(torch.tensor(G).pin_memory())
    res, stats = ctx.stream_file(f2, m, "u2", offset=7)
    b, st = res[0], res[3]
    assert stats.blocks == 11 and stats.file_bytes == ((n + 3) // 4) * m
    assert np.array_equal(b.numpy(), ref_b.numpy()) and np.array_equal(st.numpy(), ref_st.numpy())
    compare(as_numpy(res), O.gls_sequence(Phi, 0.4, XL, y, G.astype(np.float64)), 1e-10)
    with pytest.raises(GLSError) as e:
        ctx.stream_file(f2, m + 60, "u2", offset=7)   # file shorter than m columns
    assert e.value.status == -5


def test_u2_argument_errors():
    Phi, XL, y, G = _inputs(130, 4, 8, 2)
    ctx = GLSContext(_t(Phi), 0.4, _t(XL), _t(y), block_cols=8)
    Wd = _t(synth.pack_dosages_2bit(G))
    o = ctx._outputs(8, Wd.device)
    args = [ctypes.c_void_p(t.data_ptr()) for t in o]
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib().gls_block_u2(ctx.handle, 8, ctypes.c_void_p(Wd.data_ptr()), 32, args[0], 4, args[1], args[2], args[3], s)
    assert st == -1                                    # ld_g2 < ceil(130 / 4) = 33
    st = lib().gls_block_u2(ctx.handle, 9, ctypes.c_void_p(Wd.data_ptr()), 33, args[0], 4, args[1], args[2], args[3], s)
    assert st == -1                                    # mb > block_cols
    assert lib().gls_stream_file_host_bytes(ctx.handle, 4) == 0
    assert lib().gls_stream_file_host_bytes(ctx.handle, 2) == 3 * 4096


def test_u2_no_covariates_and_stream_resume():
    """p = 1 (the SNP alone) with int8 slices from packed dosages, and a packed
    stream resumed at col0: the columns before it untouched, the rest equal to
    the full stream."""
    n, m = 301, 500
    Phi = synth.kinship(n, 9)
    y = synth.phenotype(n, 9)
    G = synth.genotypes_u8(n, 0, m, 9)
    P = synth.pack_dosages_2bit(G)
    ctx = GLSContext(_t(Phi), 0.5, None, _t(y), block_cols=128, precision="int8_emu")
    a = _run_u8(ctx, G, 128)
    b = _collect([ctx.block_u2(_t(P[j:j + 128])) for j in range(0, m, 128)])
    for k in KEYS:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    Ph = torch.tensor(P).pin_memory()
    (full, *_), _ = ctx.stream(Ph, packed=True)
    f = torch.float64
    out = (torch.full((m, 1), -7.0, dtype=f).pin_memory(), torch.zeros(m, dtype=f).pin_memory(),
           torch.zeros(m, dtype=f).pin_memory(), torch.zeros(m, dtype=torch.int32).pin_memory())
    res, stats = ctx.stream(Ph, col0=333, out=out, packed=True)
    part = res[0]
    assert stats.h2d_bytes == ((n + 3) // 4) * (m - 333)
    assert (part.numpy()[:333] == -7.0).all() and np.array_equal(part.numpy()[333:], full.numpy()[333:])
    r = O.gls_sequence(Phi, 0.5, np.zeros((n, 0)), y, G[333:].astype(np.float64))
    compare(slice_out(as_numpy(res), 333), r, 1e-10)
