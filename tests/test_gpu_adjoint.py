"""The hand-written adjoint (GPU, through the C-ABI) against the FP64 CPU
autograd reference of Eq. 1 and against central finite differences.

Tolerances: element-wise relative 1e-8 against the reference gradient
(both FP64; the two differ only by rounding of different algorithms), and for
finite differences |FD - <g, u>| <= 1e-5 max(|FD|, |<g, u>|, 1e-3 |g| |u|).
"""
import numpy as np
import pytest
import torch

from oracle import gls_grad as G
from paper_1302_4332_amd import synth
from paper_1302_4332_amd.gls import GLSFunction, t2_loss

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a, grad=False):
    return torch.tensor(np.ascontiguousarray(a), device=DEV, requires_grad=grad)


def _problem(n, p, m, seed, h2):
    Phi = synth.kinship(n, seed)
    XL = synth.covariates(n, p, seed, "sex_age" if p == 4 else "gauss")
    y = synth.phenotype(n, seed)
    XR = synth.genotypes(n, 0, m, seed)
    return Phi, h2, XL, y, XR


def _gpu_grads(Phi, h2, XL, y, XR, bc, precision="fp64", sweeps=0):
    yt, XRt, h2t = _t(y, True), _t(XR, True), torch.tensor(h2, dtype=torch.float64, device=DEV, requires_grad=True)
    b, s2, v = GLSFunction.apply(yt, XRt, h2t, _t(Phi), _t(XL), bc, precision, sweeps)
    loss = t2_loss(b, s2, v)
    loss.backward()
    return loss.item(), yt.grad.cpu().numpy(), XRt.grad.cpu().numpy(), h2t.grad.item()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("n,p,m,bc,h2", [(300, 4, 200, 64, 0.3), (257, 3, 90, 90, 0.6), (520, 6, 130, 48, 0.45)])
def test_adjoint_matches_reference_gradient(n, p, m, bc, h2):
    Phi, h2, XL, y, XR = _problem(n, p, m, seed=n, h2=h2)
    loss, gy, gX, gh = _gpu_grads(Phi, h2, XL, y, XR, bc)
    rloss, ry, rX, rh = G.loss_and_grads(Phi, h2, XL, y, XR.T)
    assert loss == pytest.approx(rloss, rel=1e-10)
    assert _rel(gy, ry) < 1e-8
    assert _rel(gX, rX.T) < 1e-8
    assert gh == pytest.approx(rh, rel=1e-8)


def test_adjoint_vjp_arbitrary_cotangents():
    """All three outputs' cotangents, random: VJP against the reference."""
    Phi, h2, XL, y, XR = _problem(280, 4, 75, seed=4, h2=0.35)
    rng = np.random.default_rng(0)
    bb, sb, vb = rng.standard_normal((75, 4)), rng.standard_normal(75), rng.standard_normal(75)
    yt, XRt = _t(y, True), _t(XR, True)
    h2t = torch.tensor(h2, dtype=torch.float64, device=DEV, requires_grad=True)
    b, s2, v = GLSFunction.apply(yt, XRt, h2t, _t(Phi), _t(XL), 32, "fp64", 0)
    ((b * _t(bb)).sum() + (s2 * _t(sb)).sum() + (v * _t(vb)).sum()).backward()
    ry, rX, rh = G.outputs_grads(Phi, h2, XL, y, XR.T, bb, sb, vb)
    assert _rel(yt.grad.cpu().numpy(), ry) < 1e-8
    assert _rel(XRt.grad.cpu().numpy(), rX.T) < 1e-8
    assert float(h2t.grad) == pytest.approx(rh, rel=1e-8)


def test_adjoint_finite_differences_c3_shape():
    """n = 4096, p = 4, m = 16,384, h2 = 0.3: central differences (step 1e-6)
    of the GPU forward loss on 64 random directions split over y, X_R and h2."""
    w = synth.WORKLOADS["c3_grad_n4096"]
    st = synth.make_study(w)
    XR = st.snps(0, w.m)
    bc = w.block_cols
    loss, gy, gX, gh = _gpu_grads(st.Phi, w.h2, st.XL, st.y, XR, bc)
    Phi_d, XL_d = _t(st.Phi), _t(st.XL)

    def f(y, X, h2):
        with torch.no_grad():
            b, s2, v = GLSFunction.apply(_t(y), _t(X), torch.tensor(h2, dtype=torch.float64, device=DEV),
                                         Phi_d, XL_d, bc, "fp64", 0)
            return float(t2_loss(b, s2, v))

    rng = np.random.default_rng(7)
    eps = 1e-6
    worst = 0.0
    for k in range(64):
        which = k % 3
        if which == 0:
            u = rng.standard_normal(st.y.shape)
            fd = (f(st.y + eps * u, XR, w.h2) - f(st.y - eps * u, XR, w.h2)) / (2 * eps)
            an, gn, un = float(gy @ u), np.linalg.norm(gy), np.linalg.norm(u)
        elif which == 1:
            U = rng.standard_normal(XR.shape)
            fd = (f(st.y, XR + eps * U, w.h2) - f(st.y, XR - eps * U, w.h2)) / (2 * eps)
            an, gn, un = float(np.sum(gX * U)), np.linalg.norm(gX), np.linalg.norm(U)
        else:
            s = rng.choice([-1.0, 1.0])
            fd = (f(st.y, XR, w.h2 + eps * s) - f(st.y, XR, w.h2 - eps * s)) / (2 * eps)
            an, gn, un = gh * s, abs(gh), 1.0
        bound = 1e-5 * max(abs(fd), abs(an), 1e-3 * gn * un)
        worst = max(worst, abs(fd - an) / bound)
        assert abs(fd - an) <= bound, (k, which, fd, an)
    print(f"c3 FD: loss {loss:.6e}, worst |FD - <g,u>| / bound = {worst:.3f}")


def test_adjoint_c3_elementwise_subset():
    """n = 4096 with 2,048 SNPs of the same study: element-wise against the
    FP64 reference gradient."""
    w = synth.WORKLOADS["c3_grad_n4096"]
    st = synth.make_study(w)
    XR = st.snps(0, 2048)
    loss, gy, gX, gh = _gpu_grads(st.Phi, w.h2, st.XL, st.y, XR, 1024)
    rloss, ry, rX, rh = G.loss_and_grads(st.Phi, w.h2, st.XL, st.y, XR.T)
    assert loss == pytest.approx(rloss, rel=1e-10)
    assert _rel(gy, ry) < 1e-8 and _rel(gX, rX.T) < 1e-8
    assert gh == pytest.approx(rh, rel=1e-8)


@pytest.mark.parametrize("precision,sweeps", [("fp32_ir", 2), ("fp16_ir", 4)])
def test_adjoint_refined_mixed_matches_fp64(precision, sweeps):
    Phi, h2, XL, y, XR = _problem(300, 4, 150, seed=11, h2=0.3)
    _, gy, gX, gh = _gpu_grads(Phi, h2, XL, y, XR, 64)
    _, my, mX, mh = _gpu_grads(Phi, h2, XL, y, XR, 64, precision, sweeps)
    assert _rel(my, gy) < 1e-7 and _rel(mX, gX) < 1e-7
    assert mh == pytest.approx(gh, rel=1e-7)
