"""Streaming from storage (GPU, through the C-ABI): a reader thread and three
host buffers ahead of the two device buffers.  Results must be bitwise those
of the in-memory stream, with or without overlap, and resumable; every
streamed output is also held to the plain-FP64 bar against the CPU oracle
(per SNP max relative error of b <= 1e-10, sigma2 and v relative 1e-10,
status equal)."""
import os

import numpy as np
import pytest
import torch

from oracle import gls_oracle as O
from paper_1302_4332_amd import synth
from paper_1302_4332_amd.gls import GLSContext, GLSError
from parity_util import as_numpy, compare, slice_out

TOL = 1e-10

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


@pytest.fixture(scope="module")
def study(tmp_path_factory):
    n, m = 330, 1000
    Phi = synth.kinship(n, 31)
    XL = synth.covariates(n, 4, 31, "sex_age")
    y = synth.phenotype(n, 31)
    G = synth.genotypes_u8(n, 0, m, 31)
    d = tmp_path_factory.mktemp("snps")
    f64 = str(d / "x.f64")
    u8 = str(d / "x.u8")
    with open(f64, "wb") as f:
        f.write(b"\0" * 24)                 # a header the offset skips
        f.write(G.astype(np.float64).tobytes())
    G.tofile(u8)
    return Phi, XL, y, G, f64, u8


@pytest.mark.parametrize("serial", [False, True])
def test_file_stream_equals_memory_stream(study, serial):
    Phi, XL, y, G, f64, u8 = study
    m = G.shape[0]
    ctx = GLSContext(_t(Phi), 0.4, _t(XL), _t(y), block_cols=96, serial_stream=serial)
    (ref_b, ref_s2, _, ref_st), _ = ctx.stream(torch.tensor(G.astype(np.float64)).pin_memory())
    (b, s2, v, st), stats = ctx.stream_file(f64, m, torch.float64, offset=24)
    assert stats.blocks == 11 and stats.file_bytes == 8 * 330 * m
    assert np.array_equal(b.numpy(), ref_b.numpy()) and np.array_equal(st.numpy(), ref_st.numpy())
    out8, stats8 = ctx.stream_file(u8, m, torch.uint8)
    assert stats8.file_bytes == 330 * m
    assert np.array_equal(out8[0].numpy(), ref_b.numpy())
    r = O.gls_sequence(Phi, 0.4, XL, y, G.astype(np.float64))
    compare(as_numpy((b, s2, v, st)), r, TOL)
    compare(as_numpy(out8), r, TOL)


def test_file_stream_resume_and_errors(study):
    Phi, XL, y, G, f64, u8 = study
    m = G.shape[0]
    ctx = GLSContext(_t(Phi), 0.4, _t(XL), _t(y), block_cols=128)
    (ref, *_), _ = ctx.stream_file(u8, m, torch.uint8)
    f = torch.float64
    out = (torch.full((m, 4), -3.0, dtype=f).pin_memory(), torch.zeros(m, dtype=f).pin_memory(),
           torch.zeros(m, dtype=f).pin_memory(), torch.zeros(m, dtype=torch.int32).pin_memory())
    res, stats = ctx.stream_file(u8, m, torch.uint8, col0=600, out=out)
    b = res[0]
    assert stats.blocks == 4
    assert (b.numpy()[:600] == -3.0).all() and np.array_equal(b.numpy()[600:], ref.numpy()[600:])
    r = O.gls_sequence(Phi, 0.4, XL, y, G[600:].astype(np.float64))
    compare(slice_out(as_numpy(res), 600), r, TOL)
    with pytest.raises(GLSError) as e:
        ctx.stream_file(u8, m + 50, torch.uint8)          # file shorter than m columns
    assert e.value.status == -5
    with pytest.raises(GLSError) as e:
        ctx.stream_file(os.path.join(os.path.dirname(u8), "missing"), m, torch.uint8)
    assert e.value.status == -1


@pytest.mark.parametrize("serial", [False, True])
def test_file_stream_ramp_equals_memory_stream(tmp_path, serial):
    """Large blocks: the file stream opens with the same short blocks as the
    in-memory stream and gives bitwise its results."""
    n, m = 130, 5000
    Phi = synth.kinship(n, 41)
    XL = synth.covariates(n, 4, 41, "sex_age")
    y = synth.phenotype(n, 41)
    G = synth.genotypes_u8(n, 0, m, 41)
    path = str(tmp_path / "x.u8")
    G.tofile(path)
    ctx = GLSContext(_t(Phi), 0.4, _t(XL), _t(y), block_cols=2048, serial_stream=serial)
    (ref_b, _, _, ref_st), ref_stats = ctx.stream(torch.tensor(G).pin_memory())
    res, stats = ctx.stream_file(path, m, torch.uint8)
    b, st = res[0], res[3]
    assert stats.blocks == ref_stats.blocks > (m + 2047) // 2048    # the ramp adds blocks
    assert stats.file_bytes == n * m
    assert np.array_equal(b.numpy(), ref_b.numpy()) and np.array_equal(st.numpy(), ref_st.numpy())
    res2, stats2 = ctx.stream_file(path, m, torch.uint8, col0=1234)
    assert np.array_equal(res2[0].numpy()[1234:], ref_b.numpy()[1234:])
    r = O.gls_sequence(Phi, 0.4, XL, y, G.astype(np.float64))
    compare(as_numpy(res), r, TOL)
    compare(slice_out(as_numpy(res2), 1234), slice_out(r, 1234), TOL)
