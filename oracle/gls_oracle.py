"""CPU oracle for the GWAS sequence of generalized least-squares problems.

TEST INFRASTRUCTURE ONLY.  This is the plain, slow, FP64 statement of what the
GPU path computes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product library never
does, and it shares no code with the HIP kernels.

What is computed (paper, Sec. 1.3, Eq. 1): for every SNP i = 1..m,

    b_i = (X_i^T M^-1 X_i)^-1 X_i^T M^-1 y,   X_i = [X_L | x_R,i]  (n x p),

with the variance-component covariance M = h2 * Phi + (1 - h2) * I.  The
steps follow the Cholesky rewrite (Sec. 2.1, Eq. 2) and the structured
algorithm of Sec. 2.1 (Listing 1), in the paper's order and notation:

    L        = chol(M)                  (potrf)
    X~_L     = L^-1 X_L                 (trsm)
    y~       = L^-1 y                   (trsv)
    r~_T     = X~_L^T y~                (gemv)
    S_TL     = X~_L^T X~_L              (syrk)
    per SNP block (Sec. 2.2: pack SNP vectors so trsv becomes one trsm):
      X~_R,b = L^-1 X_R,b               (trsm)
      per SNP:  S_BL,i = x~_i^T X~_L,  S_BR,i = x~_i^T x~_i,  r~_B,i = x~_i^T y~
                S_i = [[S_TL, S_BL,i^T], [S_BL,i, S_BR,i]],  r~_i = [r~_T; r~_B,i]
                b_i = S_i^-1 r~_i       (posv: Cholesky of S_i, two substitutions)

Additions the paper does not print (readings of the silent parts):

* residual variance  sigma2_i = (c - b_i^T r~_i) / (n - p),  c = y~^T y~,
  i.e. the GLS residual (y - X_i b_i)^T M^-1 (y - X_i b_i) over n - p;
* v_i = (S_i^-1)_pp, so that se_i = sqrt(sigma2_i * v_i) and t_i = b_i,p / se_i;
* status_i = 1 when S_i is numerically singular: its Cholesky fails or the
  last squared pivot d_i^2 is not above SINGULAR_REL * S_BR,i; then b_i,
  sigma2_i and v_i are NaN.  The coefficient order is [covariates..., SNP].

Parity pins live in ``tests/test_oracle.py`` (explicit-inverse Eq. 1, exact
rational arithmetic, ordinary least squares at h2 = 0, the Frisch-Waugh-Lovell
closed form, invariances, exact recovery).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

# S_i counts as singular when its last squared Cholesky pivot is at most this
# fraction of S_BR,i = ||x~_i||^2 (x~_i lies within ~1e-6 rad of span X~_L).
SINGULAR_REL = 2.0 ** -40


class NotSPDError(ValueError):
    """M (or S_TL) is not symmetric positive definite; ``pivot`` is 1-based."""

    def __init__(self, what: str, pivot: int):
        super().__init__(f"{what} is not positive definite (leading minor {pivot})")
        self.what = what
        self.pivot = pivot


def variance_component_matrix(Phi: np.ndarray, h2: float) -> np.ndarray:
    """M = h2 * Phi + (1 - h2) * I (the covariance of the variance-component model)."""
    n = Phi.shape[0]
    return h2 * np.asarray(Phi, dtype=np.float64) + (1.0 - h2) * np.eye(n)


def cholesky_lower(A: np.ndarray, what: str = "M") -> np.ndarray:
    """Lower Cholesky factor, A = L L^T (Sec. 2.1: potrf).  Raises NotSPDError."""
    c, info = scipy.linalg.lapack.dpotrf(np.asarray(A, dtype=np.float64), lower=1, clean=1)
    if info > 0:
        raise NotSPDError(what, int(info))
    if info < 0:
        raise ValueError("dpotrf argument error")
    return np.tril(c)


def covariate_terms(L: np.ndarray, XL: np.ndarray, y: np.ndarray):
    """Loop-invariant part of the structured algorithm (Sec. 2.1).

    Returns X~_L, y~, r~_T = X~_L^T y~, S_TL = X~_L^T X~_L and c = y~^T y~.
    """
    XLt = scipy.linalg.solve_triangular(L, XL, lower=True)
    yt = scipy.linalg.solve_triangular(L, y, lower=True)
    rT = XLt.T @ yt
    STL = XLt.T @ XLt
    c = float(yt @ yt)
    return XLt, yt, rT, STL, c


def whiten_block(L: np.ndarray, XRb: np.ndarray) -> np.ndarray:
    """X~_R,b = L^-1 X_R,b for an n x mb block (Sec. 2.2: one trsm per block)."""
    return scipy.linalg.solve_triangular(L, XRb, lower=True, check_finite=False)


def snp_terms(XRt: np.ndarray, XLt: np.ndarray, yt: np.ndarray):
    """Per-SNP products: S_BL,i = x~_i^T X~_L, S_BR,i = x~_i^T x~_i, r~_B,i = x~_i^T y~."""
    SBL = XRt.T @ XLt
    SBR = np.einsum("ij,ij->j", XRt, XRt)
    rB = XRt.T @ yt
    return SBL, SBR, rB


def assemble(STL, rT, SBL, SBR, rB):
    """Stack S_i = [[S_TL, S_BL,i^T], [S_BL,i, S_BR,i]] and r~_i = [r~_T; r~_B,i]."""
    mb = SBR.shape[0]
    q = STL.shape[0]
    S = np.empty((mb, q + 1, q + 1))
    S[:, :q, :q] = STL
    S[:, q, :q] = SBL
    S[:, :q, q] = SBL
    S[:, q, q] = SBR
    r = np.empty((mb, q + 1))
    r[:, :q] = rT
    r[:, q] = rB
    return S, r


def _chol_stack(S: np.ndarray):
    """Cholesky of each p x p S_i; failing ones get NaN factors."""
    try:
        return np.linalg.cholesky(S), np.zeros(S.shape[0], dtype=bool)
    except np.linalg.LinAlgError:
        Ls = np.full_like(S, np.nan)
        bad = np.zeros(S.shape[0], dtype=bool)
        for i in range(S.shape[0]):
            try:
                Ls[i] = np.linalg.cholesky(S[i])
            except np.linalg.LinAlgError:
                bad[i] = True
        return Ls, bad


def _forward(Ls, r):
    p = r.shape[1]
    z = np.empty_like(r)
    for k in range(p):
        z[:, k] = (r[:, k] - np.einsum("ij,ij->i", Ls[:, k, :k], z[:, :k])) / Ls[:, k, k]
    return z


def _backward(Ls, z):
    p = z.shape[1]
    b = np.empty_like(z)
    for k in range(p - 1, -1, -1):
        b[:, k] = (z[:, k] - np.einsum("ij,ij->i", Ls[:, k + 1:, k], b[:, k + 1:])) / Ls[:, k, k]
    return b


def solve_small(S: np.ndarray, r: np.ndarray, SBR: np.ndarray):
    """posv per SNP: b_i = S_i^-1 r~_i by Cholesky; also v_i = (S_i^-1)_pp and status."""
    mb, p, _ = S.shape
    Ls, bad = _chol_stack(S)
    with np.errstate(invalid="ignore", divide="ignore"):
        b = _backward(Ls, _forward(Ls, r))
        e = np.zeros((mb, p))
        e[:, p - 1] = 1.0
        v = _backward(Ls, _forward(Ls, e))[:, p - 1]
        d2 = Ls[:, p - 1, p - 1] ** 2
        singular = bad | ~(d2 > SINGULAR_REL * SBR)
    b[singular] = np.nan
    v[singular] = np.nan
    return b, v, singular.astype(np.int32)


def residual_variance(c: float, b: np.ndarray, r: np.ndarray, n: int) -> np.ndarray:
    """sigma2_i = (c - b_i^T r~_i) / (n - p)."""
    p = b.shape[1]
    return (c - np.einsum("ij,ij->i", b, r)) / float(n - p)


class Study:
    """Setup of one study (Cholesky and covariate terms), then SNP blocks."""

    def __init__(self, Phi, h2, XL, y, M=None):
        XL = np.asarray(XL, dtype=np.float64)
        if XL.ndim == 1:
            XL = XL[:, None]
        self.n = XL.shape[0]
        self.p = XL.shape[1] + 1
        self.M = variance_component_matrix(Phi, h2) if M is None else np.asarray(M, dtype=np.float64)
        self.L = cholesky_lower(self.M, "M")
        self.XLt, self.yt, self.rT, self.STL, self.c = covariate_terms(self.L, XL, np.asarray(y, dtype=np.float64))
        if self.p > 1:
            cholesky_lower(self.STL, "S_TL")

    def block(self, XRb: np.ndarray, keep: bool = False):
        """One SNP block: XRb is n x mb (column-major SNPs).  Returns a dict."""
        XRt = whiten_block(self.L, np.asarray(XRb, dtype=np.float64))
        SBL, SBR, rB = snp_terms(XRt, self.XLt, self.yt)
        S, r = assemble(self.STL, self.rT, SBL, SBR, rB)
        b, v, status = solve_small(S, r, SBR)
        sigma2 = residual_variance(self.c, b, r, self.n)
        out = {"b": b, "sigma2": sigma2, "v": v, "status": status}
        if keep:
            out.update(XRt=XRt, SBL=SBL, SBR=SBR, rB=rB, S=S, r=r)
        return out


def gls_sequence(Phi, h2, XL, y, XR_snp_major, block_cols=None, M=None):
    """Whole study.  XR_snp_major has shape (m, n): row j is SNP j's n samples
    (the same memory as a column-major n x m matrix).  Returns b (m x p),
    sigma2, v, status (m,)."""
    st = Study(Phi, h2, XL, y, M=M)
    XR = np.asarray(XR_snp_major, dtype=np.float64)
    m = XR.shape[0]
    mb = m if block_cols is None else block_cols
    outs = [st.block(XR[j:j + mb].T) for j in range(0, m, max(mb, 1))] if m else []
    if not outs:
        return {"b": np.zeros((0, st.p)), "sigma2": np.zeros(0), "v": np.zeros(0),
                "status": np.zeros(0, dtype=np.int32)}
    return {k: np.concatenate([o[k] for o in outs]) for k in outs[0]}


def t_squared(b, sigma2, v):
    """t_i^2 = b_i,p^2 / (sigma2_i * v_i): the squared t-statistic of the SNP coefficient."""
    return b[:, -1] ** 2 / (sigma2 * v)


def loss_t2(b, sigma2, v) -> float:
    """Scalar loss: sum over SNPs of squared t-statistics."""
    return float(np.sum(t_squared(b, sigma2, v)))
