"""The adjoint of a streamed study (GPU, through the C-ABI): gls_stream_backward
over SNP blocks held in page-locked host memory, then gls_backward_finish.

- Against the FP64 CPU autograd reference of Eq. 1 (loss sum_i t_i^2): every
  entry of the y and X_R gradients within 1e-8 element-wise (floor one
  millionth of the largest entry), the h2 gradient relative 1e-8; in FP64 and
  refined FP32, with p = 4, 3 and 1 (no covariates).
- Bitwise equal to the device-resident adjoint (GLSFunction, gls_backward_block
  per block), with and without the opening ramp of short blocks (every block
  but the last a multiple of 16 SNPs), when resumed with col0, in serial mode
  and on caller-given streams.
- Arbitrary cotangents of all three outputs against the reference VJP.
- Error paths: no GLS_KEEP_FOR_GRAD, col0 outside [0, m], a wrong shape.
- At n = 20,000, p = 8, blocks of 16,384 in refined FP32 x2 (the whole-study
  gradient's configuration): bitwise equal to the resident adjoint on the first
  block and the ragged last one.
"""
import numpy as np
import pytest
import torch

from oracle import gls_grad as G
from paper_1302_4332_amd import synth
from paper_1302_4332_amd.gls import GLSContext, GLSError, GLSFunction, stream_grad, stream_grad_file, t2_loss
from parity_util import elementwise_close

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL_G = 1e-8


def _t(a, grad=False):
    return torch.tensor(np.ascontiguousarray(a), device=DEV, requires_grad=grad)


def _problem(n, p, m, seed, h2):
    Phi = synth.kinship(n, seed)
    XL = synth.covariates(n, p, seed, "sex_age" if p == 4 else "gauss")
    y = synth.phenotype(n, seed)
    XR = synth.genotypes(n, 0, m, seed)
    return Phi, h2, XL, y, XR


def _resident(Phi, h2, XL, y, XR, bc, precision, sweeps):
    yt, XRt = _t(y, True), _t(XR, True)
    h2t = torch.tensor(h2, dtype=torch.float64, device=DEV, requires_grad=True)
    b, s2, v = GLSFunction.apply(yt, XRt, h2t, _t(Phi), _t(XL), bc, precision, sweeps)
    t2_loss(b, s2, v).backward()
    return yt.grad.cpu().numpy(), XRt.grad.cpu().numpy(), float(h2t.grad)


def _streamed(Phi, h2, XL, y, XR, bc, precision, sweeps):
    XR_host = torch.tensor(XR).pin_memory()
    XR_grad = torch.empty_like(XR_host).pin_memory()
    loss, gy, gh, outs = stream_grad(_t(Phi), h2, _t(XL), _t(y), XR_host, t2_loss, block_cols=bc,
                                     precision=precision, refine_sweeps=sweeps, XR_grad=XR_grad)
    return loss, gy.cpu().numpy(), XR_grad.numpy().copy(), float(gh), outs


def _cotangents(Phi, h2, XL, y, XR_host, bc, precision, sweeps, **kw):
    """Outputs of a streamed forward and the t^2 loss's cotangents (pinned)."""
    g = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=bc, precision=precision, refine_sweeps=sweeps,
                   keep_for_grad=True, **kw)
    outs, _ = g.stream(XR_host)
    leaves = [t.to(DEV).requires_grad_(True) for t in outs[:3]]
    grads = torch.autograd.grad(t2_loss(*leaves), leaves)
    return g, [c.detach().cpu().pin_memory() for c in grads]


@pytest.mark.parametrize("precision,sweeps", [("fp64", 0), ("fp32_ir", 2)])
@pytest.mark.parametrize("n,p,m,bc,h2", [(300, 4, 700, 128, 0.3), (257, 3, 333, 100, 0.6), (200, 1, 150, 64, 0.45)])
def test_streamed_adjoint_matches_reference(n, p, m, bc, h2, precision, sweeps):
    Phi, h2, XL, y, XR = _problem(n, p, m, seed=n + m, h2=h2)
    loss, gy, gX, gh, _ = _streamed(Phi, h2, XL, y, XR, bc, precision, sweeps)
    rloss, ry, rX, rh = G.loss_and_grads(Phi, h2, XL, y, XR.T)
    assert loss == pytest.approx(rloss, rel=1e-8)
    elementwise_close(gy, ry, TOL_G)
    elementwise_close(gX, rX.T, TOL_G)
    assert gh == pytest.approx(rh, rel=TOL_G)


@pytest.mark.parametrize("precision,sweeps", [("fp64", 0), ("fp32_ir", 2)])
@pytest.mark.parametrize("n,m,bc", [(300, 700, 128), (330, 5000, 2048)])
def test_streamed_adjoint_bitwise_equals_resident(n, m, bc, precision, sweeps):
    """bc = 128: the same blocks as the resident path.  bc = 2,048: the stream
    opens with blocks of 256, 320, 448, ... (multiples of 64), the resident path
    runs 2,048, 2,048, 904; the adjoint sums run in SNP order in groups of 16,
    so the gradients agree bitwise."""
    Phi, h2, XL, y, XR = _problem(n, 4, m, seed=11, h2=0.4)
    ry, rX, rh = _resident(Phi, h2, XL, y, XR, bc, precision, sweeps)
    _, gy, gX, gh, _ = _streamed(Phi, h2, XL, y, XR, bc, precision, sweeps)
    assert np.array_equal(gy, ry)
    assert np.array_equal(gX, rX)
    assert gh == rh


def test_resume_serial_and_caller_streams_bitwise():
    n, m, bc = 300, 3000, 2048
    Phi, h2, XL, y, XR = _problem(n, 4, m, seed=5, h2=0.45)
    XR_host = torch.tensor(XR).pin_memory()

    def run(split=None, serial=False, streams=False):
        g, (bb, sb, vb) = _cotangents(Phi, h2, XL, y, XR_host, bc, "fp64", 0, serial_stream=serial)
        XR_grad = torch.zeros_like(XR_host).pin_memory()
        kw = {}
        if streams:
            kw = {"compute_stream": torch.cuda.Stream(), "copy_stream": torch.cuda.Stream()}
        if split is None:
            s = g.stream_backward(XR_host, bb, sb, vb, XR_grad=XR_grad, **kw)
            assert s.h2d_bytes == 8 * m * (n + 4 + 2) and s.d2h_bytes == 8 * m * n
        else:   # the first `split` SNPs, then the rest with col0
            g.stream_backward(XR_host[:split], bb[:split], sb[:split], vb[:split], XR_grad=XR_grad[:split], **kw)
            g.stream_backward(XR_host, bb, sb, vb, col0=split, XR_grad=XR_grad, **kw)
        gy, gh = g.backward_finish()
        torch.cuda.synchronize()
        g.close()
        return gy.cpu().numpy(), XR_grad.numpy().copy(), float(gh)

    ref = run()
    for kw in ({"split": 1200}, {"split": 2048}, {"serial": True}, {"streams": True}):
        got = run(**kw)
        print(kw, flush=True)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]) and got[2] == ref[2], kw
    rloss, ry, rX, rh = G.loss_and_grads(Phi, h2, XL, y, XR.T)
    elementwise_close(ref[0], ry, TOL_G)
    elementwise_close(ref[1], rX.T, TOL_G)
    assert ref[2] == pytest.approx(rh, rel=TOL_G)


def test_streamed_vjp_arbitrary_cotangents_without_xr_grad():
    n, m = 280, 450
    Phi, h2, XL, y, XR = _problem(n, 4, m, seed=4, h2=0.35)
    rng = np.random.default_rng(1)
    bb, sb, vb = rng.standard_normal((m, 4)), rng.standard_normal(m), rng.standard_normal(m)
    g = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=64, keep_for_grad=True)
    XR_host = torch.tensor(XR).pin_memory()
    g.stream(XR_host)
    g.stream_backward(XR_host, *(torch.tensor(a).pin_memory() for a in (bb, sb, vb)))
    gy, gh = g.backward_finish()
    torch.cuda.synchronize()
    g.close()
    ry, _, rh = G.outputs_grads(Phi, h2, XL, y, XR.T, bb, sb, vb)
    elementwise_close(gy.cpu().numpy(), ry, TOL_G)
    assert float(gh) == pytest.approx(rh, rel=TOL_G)


def test_stream_backward_errors():
    Phi, h2, XL, y, XR = _problem(200, 4, 100, seed=2, h2=0.4)
    XR_host = torch.tensor(XR).pin_memory()
    z = [torch.zeros(100, 4, dtype=torch.float64), torch.zeros(100, dtype=torch.float64),
         torch.zeros(100, dtype=torch.float64)]
    g = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=64)
    with pytest.raises(GLSError) as e:
        g.stream_backward(XR_host, *z)
    assert "GLS_KEEP_FOR_GRAD" in str(e.value)
    g.close()
    g = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=64, keep_for_grad=True)
    with pytest.raises(GLSError):
        g.stream_backward(XR_host, *z, col0=101)
    with pytest.raises(ValueError):
        g.stream_backward(XR_host, z[0][:50], z[1], z[2])
    s = g.stream_backward(XR_host, *z, col0=100)   # empty: nothing streamed
    assert s.blocks == 0
    g.close()


@pytest.mark.timeout(900)
def test_full_size_streamed_gradient_equals_resident():
    """n = 20,000, p = 8, blocks of 16,384, refined FP32 x2 (the configuration of
    the bench's whole-study gradient): the study's first block and its ragged
    last 1,152 SNPs.  The stream opens with blocks of 2,048, 2,560, ... (all
    multiples of 16), the resident path runs 16,384 and 1,152, so y_grad and
    h2_grad agree bitwise; the resident h2 gradient of these SNPs is checked
    against the oracle's central differences in test_gpu_combined.py."""
    w = synth.WORKLOADS["c4_n20k_p8"]
    st = synth.make_study(w)
    bc, tail = w.block_cols, w.m % w.block_cols
    Xh = np.concatenate([st.snps(0, bc), st.snps(w.m - tail, w.m)])
    Phi, XL, y = _t(st.Phi), _t(st.XL), _t(st.y)
    yt, Xt = _t(st.y, True), _t(Xh)
    h2t = torch.tensor(w.h2, dtype=torch.float64, device=DEV, requires_grad=True)
    b, s2, v = GLSFunction.apply(yt, Xt, h2t, Phi, XL, bc, "fp32_ir", 2)
    t2_loss(b, s2, v).backward()
    ry, rh = yt.grad.cpu().numpy(), float(h2t.grad)
    del Xt, b, s2, v
    loss, gy, gh, outs = stream_grad(Phi, w.h2, XL, y, torch.tensor(Xh).pin_memory(), t2_loss, block_cols=bc,
                                     precision="fp32_ir", refine_sweeps=2)
    print(f"n = 20,000: d loss / d h2 resident {rh:.12e} streamed {float(gh):.12e}", flush=True)
    assert np.array_equal(gy.cpu().numpy(), ry)
    assert float(gh) == rh
    assert (outs[3].numpy() == 0).all()


@pytest.fixture(scope="module")
def snp_files(tmp_path_factory):
    """The same 2,600 SNPs at n = 330 as an FP64 file behind a 24-byte header,
    a byte file and a packed 2-bit file (blocks of 2,048: the opening ramp of
    256, 320, 448, ... runs through the file as in memory)."""
    n, m = 330, 2600
    Phi, h2, XL, y, XR = _problem(n, 4, m, seed=21, h2=0.35)
    G = XR.astype(np.uint8)
    d = tmp_path_factory.mktemp("adj")
    f64, u8, u2 = str(d / "x.f64"), str(d / "x.u8"), str(d / "x.u2")
    with open(f64, "wb") as f:
        f.write(b"\0" * 24)
        f.write(XR.tobytes())
    G.tofile(u8)
    synth.pack_dosages_2bit(G).tofile(u2)
    return Phi, h2, XL, y, XR, f64, u8, u2


def _file_grads(snp_files, fmt, path, offset=0, serial=False, split=None, with_xr=True):
    Phi, h2, XL, y, XR, *_ = snp_files
    m, n = XR.shape
    g, (bb, sb, vb) = _cotangents(Phi, h2, XL, y, torch.tensor(XR).pin_memory(), 2048, "fp64", 0,
                                  serial_stream=serial)
    XR_grad = torch.zeros((m, n), dtype=torch.float64).pin_memory() if with_xr else None
    if split is None:
        s = g.stream_backward_file(path, m, bb, sb, vb, fmt=fmt, offset=offset, XR_grad=XR_grad)
        assert s.file_bytes == m * {torch.float64: 8 * n, torch.uint8: n, "u2": (n + 3) // 4}[fmt]
    else:
        g.stream_backward_file(path, split, bb[:split], sb[:split], vb[:split], fmt=fmt, offset=offset,
                               XR_grad=XR_grad[:split] if with_xr else None)
        g.stream_backward_file(path, m, bb, sb, vb, fmt=fmt, offset=offset, col0=split, XR_grad=XR_grad)
    gy, gh = g.backward_finish()
    torch.cuda.synchronize()
    g.close()
    return gy.cpu().numpy(), (XR_grad.numpy().copy() if with_xr else None), float(gh)


def test_file_adjoint_equals_memory_adjoint(snp_files):
    """FP64, byte and packed files, overlapped, serial and resumed: bitwise the
    gradients of the in-memory streamed adjoint on the same values."""
    Phi, h2, XL, y, XR, f64, u8, u2 = snp_files
    g, (bb, sb, vb) = _cotangents(Phi, h2, XL, y, torch.tensor(XR).pin_memory(), 2048, "fp64", 0)
    XR_host = torch.tensor(XR).pin_memory()
    XR_grad = torch.zeros_like(XR_host).pin_memory()
    g.stream_backward(XR_host, bb, sb, vb, XR_grad=XR_grad)
    ry, rh = g.backward_finish()
    torch.cuda.synchronize()
    g.close()
    ref = (ry.cpu().numpy(), XR_grad.numpy().copy(), float(rh))
    cases = [dict(fmt=torch.float64, path=f64, offset=24), dict(fmt=torch.float64, path=f64, offset=24, serial=True),
             dict(fmt=torch.float64, path=f64, offset=24, split=1024), dict(fmt=torch.uint8, path=u8),
             dict(fmt="u2", path=u2), dict(fmt="u2", path=u2, serial=True, with_xr=False)]
    for kw in cases:
        gy, gX, gh = _file_grads(snp_files, **kw)
        print({k: str(v) for k, v in kw.items() if k != "path"}, flush=True)
        assert np.array_equal(gy, ref[0]) and gh == ref[2], kw
        if gX is not None:
            assert np.array_equal(gX, ref[1]), kw
    rloss, ry_o, rX_o, rh_o = G.loss_and_grads(Phi, h2, XL, y, XR.T)
    elementwise_close(ref[0], ry_o, TOL_G)
    elementwise_close(ref[1], rX_o.T, TOL_G)
    assert ref[2] == pytest.approx(rh_o, rel=TOL_G)


def test_file_adjoint_errors(snp_files, tmp_path):
    Phi, h2, XL, y, XR, f64, u8, u2 = snp_files
    m = XR.shape[0]
    z = [torch.zeros(m, 4, dtype=torch.float64), torch.zeros(m, dtype=torch.float64),
         torch.zeros(m, dtype=torch.float64)]
    g = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=2048)
    with pytest.raises(GLSError, match="GLS_KEEP_FOR_GRAD"):
        g.stream_backward_file(u8, m, *z, fmt=torch.uint8)
    g.close()
    g = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=2048, keep_for_grad=True)
    with pytest.raises(GLSError, match="cannot open"):
        g.stream_backward_file(str(tmp_path / "missing.u8"), m, *z, fmt=torch.uint8)
    short = str(tmp_path / "short.u8")
    XR[: m // 2].astype(np.uint8).tofile(short)
    with pytest.raises(GLSError, match="shorter"):
        g.stream_backward_file(short, m, *z, fmt=torch.uint8)
    with pytest.raises(GLSError):
        g.stream_backward_file(u8, m, *z, fmt=torch.uint8, col0=m + 1)
    assert g.stream_backward_file(u8, m, *z, fmt=torch.uint8, col0=m).blocks == 0
    g.close()


@pytest.mark.parametrize("fmt", [torch.float64, "u2"])
def test_stream_grad_file_equals_stream_grad(snp_files, fmt):
    """The whole file pipeline (forward from the file, the loss's cotangents,
    the adjoint from the file) against stream_grad on the same SNPs in memory,
    in refined FP32 x2: bitwise equal outputs and gradients."""
    Phi, h2, XL, y, XR, f64, u8, u2 = snp_files
    args = (_t(Phi), h2, _t(XL), _t(y))
    kw = dict(block_cols=2048, precision="fp32_ir", refine_sweeps=2)
    loss, gy, gh, outs = stream_grad(*args, torch.tensor(XR).pin_memory(), t2_loss, **kw)
    path, off = (f64, 24) if fmt is torch.float64 else (u2, 0)
    lf, fy, fh, fouts = stream_grad_file(*args, path, XR.shape[0], t2_loss, fmt=fmt, offset=off, **kw)
    assert lf == loss and float(fh) == float(gh)
    assert np.array_equal(fy.cpu().numpy(), gy.cpu().numpy())
    for a, b in zip(fouts, outs):
        assert np.array_equal(a.numpy(), b.numpy(), equal_nan=True)
