"""Reference gradient of the squared-t loss (TEST INFRASTRUCTURE ONLY).

Dense FP64 CPU PyTorch autograd through Eq. 1 of Sec. 1.3 written out
directly, with M^-1 applied by a Cholesky solve:

    M     = h2 * Phi + (1 - h2) * I
    A_i   = X_i^T M^-1 X_i,   g_i = X_i^T M^-1 y,   b_i = A_i^-1 g_i
    sigma2_i = (y^T M^-1 y - b_i^T g_i) / (n - p)   (GLS residual over n - p)
    v_i   = (A_i^-1)_pp,      loss = sum_i b_i,p^2 / (sigma2_i * v_i)

It does not use the structured algorithm, the whitened quantities or any
hand-derived adjoint, so it is independent of the GPU backward.  Only
``tests/`` and ``bench.py``'s ``cpu_baseline`` leg may import it.
"""
from __future__ import annotations

import numpy as np
import torch


def eq1_outputs(Phi, h2, XL, y, XR):
    """b (m x p), sigma2 (m), v (m) as differentiable float64 CPU tensors.

    XR is n x m (one SNP per column).
    """
    n = Phi.shape[0]
    q = XL.shape[1]
    p = q + 1
    eye = torch.eye(n, dtype=torch.float64)
    M = h2 * Phi + (1.0 - h2) * eye
    C = torch.linalg.cholesky(M)
    MiXL = torch.cholesky_solve(XL, C)
    Miy = torch.cholesky_solve(y[:, None], C)[:, 0]
    MiXR = torch.cholesky_solve(XR, C)
    m = XR.shape[1]
    ATL = XL.T @ MiXL
    ABL = XR.T @ MiXL
    ABR = (XR * MiXR).sum(0)
    top = torch.cat([ATL.expand(m, q, q), ABL[:, None, :]], dim=1)      # rows 0..q, cols 0..q-1
    right = torch.cat([ABL[:, :, None], ABR[:, None, None]], dim=1)      # col q
    A = torch.cat([top, right], dim=2)
    g = torch.cat([(XL.T @ Miy).expand(m, q), (XR.T @ Miy)[:, None]], dim=1)
    b = torch.linalg.solve(A, g)
    yMy = y @ Miy
    sigma2 = (yMy - (b * g).sum(-1)) / float(n - p)
    v = torch.linalg.inv(A)[:, p - 1, p - 1]
    return b, sigma2, v


def loss_t2(b, sigma2, v):
    return (b[:, -1] ** 2 / (sigma2 * v)).sum()


def loss_and_grads(Phi, h2, XL, y, XR_cols):
    """Loss and its gradients with respect to y (n), X_R (n x m) and h2.

    Inputs are numpy float64; XR_cols is n x m.  Returns
    (loss, dy, dXR (n x m), dh2).
    """
    Phi_t = torch.as_tensor(np.asarray(Phi), dtype=torch.float64)
    XL_t = torch.as_tensor(np.asarray(XL), dtype=torch.float64)
    y_t = torch.tensor(np.asarray(y), dtype=torch.float64, requires_grad=True)
    XR_t = torch.tensor(np.asarray(XR_cols), dtype=torch.float64, requires_grad=True)
    h2_t = torch.tensor(float(h2), dtype=torch.float64, requires_grad=True)
    b, s2, v = eq1_outputs(Phi_t, h2_t, XL_t, y_t, XR_t)
    loss = loss_t2(b, s2, v)
    loss.backward()
    return (loss.item(), y_t.grad.numpy().copy(), XR_t.grad.numpy().copy(), h2_t.grad.item())


def outputs_grads(Phi, h2, XL, y, XR_cols, b_bar, s2_bar, v_bar):
    """Vector-Jacobian product of (b, sigma2, v) with given cotangents.

    Returns (dy, dXR (n x m), dh2) for the scalar sum(b*b_bar) + sum(s2*s2_bar) + sum(v*v_bar).
    """
    Phi_t = torch.as_tensor(np.asarray(Phi), dtype=torch.float64)
    XL_t = torch.as_tensor(np.asarray(XL), dtype=torch.float64)
    y_t = torch.tensor(np.asarray(y), dtype=torch.float64, requires_grad=True)
    XR_t = torch.tensor(np.asarray(XR_cols), dtype=torch.float64, requires_grad=True)
    h2_t = torch.tensor(float(h2), dtype=torch.float64, requires_grad=True)
    b, s2, v = eq1_outputs(Phi_t, h2_t, XL_t, y_t, XR_t)
    f = (b * torch.as_tensor(b_bar)).sum() + (s2 * torch.as_tensor(s2_bar)).sum() + (v * torch.as_tensor(v_bar)).sum()
    f.backward()
    return y_t.grad.numpy().copy(), XR_t.grad.numpy().copy(), h2_t.grad.item()
