"""Comparison of GPU outputs with the CPU oracle, shared by the GPU tests.

Bar (reading of the "1e-10 relative" target, where componentwise relative
error is undefined for coefficients near zero): per SNP
||b_i - b_i,oracle||_inf / ||b_i,oracle||_inf <= tol, relative tol on
sigma2_i and v_i, status bit-exact, NaN outputs where the status is 1.
"""
import numpy as np

KEYS = ("b", "sigma2", "v", "status")


def as_numpy(out):
    """(b, sigma2, v, status) tensors (host or device) -> dict of numpy arrays."""
    return {k: t.cpu().numpy() if hasattr(t, "cpu") else np.asarray(t) for k, t in zip(KEYS, out)}


def compare(g, r, tol):
    """Asserts the bar; returns the worst relative error of b."""
    assert np.array_equal(g["status"], r["status"]), "status differs from the oracle"
    ok = r["status"] == 0
    err = np.max(np.abs(g["b"][ok] - r["b"][ok]), axis=1) / np.max(np.abs(r["b"][ok]), axis=1)
    worst = float(err.max(initial=0.0))
    assert worst <= tol, f"max rel err b {worst:.3e} > {tol:g}"
    assert np.allclose(g["sigma2"][ok], r["sigma2"][ok], rtol=tol, atol=0), "sigma2"
    assert np.allclose(g["v"][ok], r["v"][ok], rtol=tol, atol=0), "v"
    assert np.isnan(g["b"][~ok]).all() and np.isnan(g["sigma2"][~ok]).all()
    return worst


def slice_out(d, j0, j1=None):
    return {k: v[j0:j1] for k, v in d.items()}


def elementwise_close(a, b, tol, floor=1e-6):
    """|a - b| <= tol * max(|b|, floor * max|b|) for every entry; returns the
    worst ratio |a - b| / (tol * max(|b|, floor * max|b|))."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.maximum(np.abs(b), floor * float(np.max(np.abs(b))))
    ratio = np.abs(a - b) / (tol * scale)
    worst = float(ratio.max(initial=0.0))
    assert worst <= 1.0, f"element-wise: worst |a - b| / bound = {worst:.3f} (tol {tol:g}, floor {floor:g})"
    return worst
