"""Pins of the reference gradient (oracle/gls_grad.py) by central finite
differences of the forward oracle's loss (Eq. 1 evaluated by the structured
algorithm, a different route from the dense autograd reference)."""
import numpy as np
import pytest

from oracle import gls_grad as G
from oracle import gls_oracle as O


def _problem(n=28, p=4, m=7, seed=3, h2=0.35):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, 2 * n))
    Phi = B @ B.T / (2 * n) + 1e-3 * np.eye(n)
    XL = np.column_stack([np.ones(n), rng.integers(0, 2, n), rng.normal(50, 10, n)])[:, :p - 1]
    y = rng.standard_normal(n)
    XR = rng.integers(0, 3, size=(m, n)).astype(float)
    return Phi, h2, XL, y, XR


def _loss(Phi, h2, XL, y, XR):
    o = O.gls_sequence(Phi, h2, XL, y, XR)
    return O.loss_t2(o["b"], o["sigma2"], o["v"])


def _check(fd, an, gnorm, vnorm):
    assert abs(fd - an) <= 1e-5 * max(abs(fd), abs(an), 1e-3 * gnorm * vnorm)


def test_reference_loss_matches_forward_oracle():
    Phi, h2, XL, y, XR = _problem()
    loss, *_ = G.loss_and_grads(Phi, h2, XL, y, XR.T)
    assert loss == pytest.approx(_loss(Phi, h2, XL, y, XR), rel=1e-11)


@pytest.mark.parametrize("seed", [0, 1])
def test_reference_gradient_vs_central_differences(seed):
    Phi, h2, XL, y, XR = _problem(seed=seed + 10)
    _, dy, dXR, dh2 = G.loss_and_grads(Phi, h2, XL, y, XR.T)
    rng = np.random.default_rng(seed)
    eps = 1e-6
    for _ in range(8):
        u = rng.standard_normal(y.shape)
        fd = (_loss(Phi, h2, XL, y + eps * u, XR) - _loss(Phi, h2, XL, y - eps * u, XR)) / (2 * eps)
        _check(fd, dy @ u, np.linalg.norm(dy), np.linalg.norm(u))
        W = rng.standard_normal(XR.shape)            # SNP-major direction
        fd = (_loss(Phi, h2, XL, y, XR + eps * W) - _loss(Phi, h2, XL, y, XR - eps * W)) / (2 * eps)
        _check(fd, np.sum(dXR.T * W), np.linalg.norm(dXR), np.linalg.norm(W))
    fd = (_loss(Phi, h2 + eps, XL, y, XR) - _loss(Phi, h2 - eps, XL, y, XR)) / (2 * eps)
    _check(fd, dh2, abs(dh2), 1.0)


def test_output_vjp_consistent_with_loss_gradient():
    """The VJP of (b, sigma2, v) with the loss's own cotangents equals the loss gradient."""
    Phi, h2, XL, y, XR = _problem(seed=5)
    o = O.gls_sequence(Phi, h2, XL, y, XR)
    b, s2, v = o["b"], o["sigma2"], o["v"]
    bbar = np.zeros_like(b)
    bbar[:, -1] = 2 * b[:, -1] / (s2 * v)
    s2bar = -b[:, -1] ** 2 / (s2 ** 2 * v)
    vbar = -b[:, -1] ** 2 / (s2 * v ** 2)
    dy, dXR, dh2 = G.outputs_grads(Phi, h2, XL, y, XR.T, bbar, s2bar, vbar)
    _, dy2, dXR2, dh22 = G.loss_and_grads(Phi, h2, XL, y, XR.T)
    assert np.allclose(dy, dy2, rtol=1e-9, atol=1e-12)
    assert np.allclose(dXR, dXR2, rtol=1e-9, atol=1e-12)
    assert dh2 == pytest.approx(dh22, rel=1e-9)


def test_h2_gradient_closed_form():
    """d loss / d h2 of the reference gradient against a closed form with no
    autograd and no differences: dM/dh2 = Phi - I, so d(M^-1) = -M^-1 (Phi - I)
    M^-1, and per SNP, with A = X^T M^-1 X and r = X^T M^-1 y,
        dA = -X^T M^-1 (Phi - I) M^-1 X,   dr = -X^T M^-1 (Phi - I) M^-1 y,
        db = A^-1 (dr - dA b),   dc = -y^T M^-1 (Phi - I) M^-1 y,
        dsigma2 = (dc - db.r - b.dr) / (n - p),   dv = -(A^-1 dA A^-1)_pp,
    chained into t^2 = b_p^2 / (sigma2 v)."""
    Phi, h2, XL, y, XR = _problem(seed=21)
    n, m = XR.shape[1], XR.shape[0]
    p = XL.shape[1] + 1
    M = h2 * Phi + (1 - h2) * np.eye(n)
    Mi = np.linalg.inv(M)
    D = Mi @ (Phi - np.eye(n)) @ Mi                   # -d(M^-1)/dh2
    c, dc = y @ Mi @ y, -(y @ D @ y)
    total = 0.0
    for i in range(m):
        X = np.column_stack([XL, XR[i]])
        A, r = X.T @ Mi @ X, X.T @ Mi @ y
        Ai = np.linalg.inv(A)
        b = Ai @ r
        dA, dr = -(X.T @ D @ X), -(X.T @ D @ y)
        db = Ai @ (dr - dA @ b)
        s2 = (c - b @ r) / (n - p)
        ds2 = (dc - db @ r - b @ dr) / (n - p)
        v, dv = Ai[-1, -1], -(Ai @ dA @ Ai)[-1, -1]
        total += 2 * b[-1] * db[-1] / (s2 * v) - b[-1] ** 2 * (ds2 * v + s2 * dv) / (s2 * v) ** 2
    _, _, _, dh2 = G.loss_and_grads(Phi, h2, XL, y, XR.T)
    assert dh2 == pytest.approx(total, rel=1e-9)
