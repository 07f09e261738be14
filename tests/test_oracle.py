"""Pins of the CPU oracle against mathematics it does not itself use.

Each test names what fixes the expected value: an exact rational solution of
Eq. 1, a textbook closed form, a library routine for a special case, an
invariance of the GLS solution, or brute force on tiny inputs.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import gls_oracle as O
from oracle.exact import gls_exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_problem(n=40, p=4, m=16, seed=0, h2=0.45):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, 3 * n))
    Phi = G @ G.T / (3 * n) + 1e-3 * np.eye(n)
    XL = np.column_stack([np.ones(n)] + [rng.standard_normal(n) for _ in range(p - 2)])
    y = rng.standard_normal(n)
    XR = rng.integers(0, 3, size=(m, n)).astype(np.float64)   # SNP-major
    return Phi, h2, XL, y, XR


def _relerr(a, b):
    return np.max(np.abs(a - b), axis=-1) / np.max(np.abs(b), axis=-1)


def _frac(s):
    return Fraction(s)


# -- exact rational pins (Eq. 1) -------------------------------------------

def test_golden_exact_fixture():
    """Eq. 1 in exact arithmetic (tests/golden/eq1_exact_tiny.json)."""
    doc = json.load(open(os.path.join(GOLDEN, "eq1_exact_tiny.json")))
    M = np.array(doc["M"], dtype=np.float64)
    XL = np.array(doc["XL"], dtype=np.float64)
    y = np.array(doc["y"], dtype=np.float64)
    XR = np.array(doc["XR_cols"], dtype=np.float64)
    out = O.gls_sequence(None, 0.0, XL, y, XR, M=M)
    b_ex = np.array([[float(_frac(v)) for v in row] for row in doc["b"]])
    s_ex = np.array([float(_frac(v)) for v in doc["sigma2"]])
    v_ex = np.array([float(_frac(v)) for v in doc["v"]])
    assert np.all(_relerr(out["b"], b_ex) < 1e-13)
    assert np.allclose(out["sigma2"], s_ex, rtol=1e-13, atol=0)
    assert np.allclose(out["v"], v_ex, rtol=1e-13, atol=0)
    assert not out["status"].any()


def test_golden_fixture_reproducible():
    doc = json.load(open(os.path.join(GOLDEN, "eq1_exact_tiny.json")))
    res = gls_exact(doc["M"], doc["XL"], doc["y"], doc["XR_cols"])
    for (b, s, v), b_g, s_g, v_g in zip(res, doc["b"], doc["sigma2"], doc["v"]):
        assert b == [_frac(v) for v in b_g]
        assert s == _frac(s_g) and v == _frac(v_g)


def test_hand_example_single_regressor():
    """p = 1, M = I: b = x.y / x.x; x=(1,2,3), y=(1,0,2) gives b = 1/2,
    residual (1/2, -1, 1/2), sigma2 = (3/2)/2 = 3/4, v = 1/14."""
    (b, s2, v), = gls_exact([[1, 0, 0], [0, 1, 0], [0, 0, 1]], [[], [], []], [1, 0, 2], [[1, 2, 3]])
    assert b == [Fraction(1, 2)] and s2 == Fraction(3, 4) and v == Fraction(1, 14)
    out = O.gls_sequence(None, 0.0, np.zeros((3, 0)), np.array([1.0, 0, 2]),
                         np.array([[1.0, 2, 3]]), M=np.eye(3))
    assert out["b"][0, 0] == pytest.approx(0.5, rel=1e-15)
    assert out["sigma2"][0] == pytest.approx(0.75, rel=1e-15)
    assert out["v"][0] == pytest.approx(1 / 14, rel=1e-15)


def test_simple_linear_regression_closed_form():
    """M = I, X_i = [1 | x]: slope = Sxy/Sxx, intercept = ybar - slope*xbar,
    v = 1/Sxx, sigma2 = (Syy - Sxy^2/Sxx)/(n-2)  (textbook OLS)."""
    rng = np.random.default_rng(3)
    n = 50
    x = rng.integers(0, 3, n).astype(float)
    y = 0.7 * x + rng.standard_normal(n)
    xb, yb = x.mean(), y.mean()
    Sxx = np.sum((x - xb) ** 2)
    Sxy = np.sum((x - xb) * (y - yb))
    Syy = np.sum((y - yb) ** 2)
    out = O.gls_sequence(None, 0.0, np.ones((n, 1)), y, x[None, :], M=np.eye(n))
    assert out["b"][0, 1] == pytest.approx(Sxy / Sxx, rel=1e-12)
    assert out["b"][0, 0] == pytest.approx(yb - Sxy / Sxx * xb, rel=1e-12)
    assert out["v"][0] == pytest.approx(1 / Sxx, rel=1e-12)
    assert out["sigma2"][0] == pytest.approx((Syy - Sxy ** 2 / Sxx) / (n - 2), rel=1e-11)


def test_exact_rational_random_small():
    """Brute force: exact Eq. 1 on small random integer problems vs the FP64 oracle."""
    rng = np.random.default_rng(11)
    n, q = 9, 2
    B = rng.integers(-2, 3, size=(n, n))
    M = (B @ B.T + 3 * np.eye(n, dtype=int)).tolist()
    XL = np.column_stack([np.ones(n, int), rng.integers(0, 2, n)]).tolist()
    y = rng.integers(-5, 6, n).tolist()
    XR = rng.integers(0, 3, size=(4, n)).tolist()
    res = gls_exact(M, XL, y, XR)
    out = O.gls_sequence(None, 0.0, np.array(XL, float), np.array(y, float),
                         np.array(XR, float), M=np.array(M, float))
    b_ex = np.array([[float(v) for v in b] for b, _, _ in res])
    assert np.all(_relerr(out["b"], b_ex) < 1e-12)
    assert np.allclose(out["sigma2"], [float(s) for _, s, _ in res], rtol=1e-11, atol=0)
    assert np.allclose(out["v"], [float(v) for _, _, v in res], rtol=1e-12, atol=0)


# -- Eq. 1 with explicit inverses (brute force) -----------------------------

def test_eq1_explicit_inverse():
    Phi, h2, XL, y, XR = _rand_problem()
    n = Phi.shape[0]
    M = h2 * Phi + (1 - h2) * np.eye(n)
    Mi = np.linalg.inv(M)
    out = O.gls_sequence(Phi, h2, XL, y, XR, block_cols=5)
    for i in range(XR.shape[0]):
        X = np.column_stack([XL, XR[i]])
        A = X.T @ Mi @ X
        b = np.linalg.inv(A) @ (X.T @ Mi @ y)
        res = y - X @ b
        assert _relerr(out["b"][i], b) < 1e-10
        assert out["sigma2"][i] == pytest.approx(res @ Mi @ res / (n - X.shape[1]), rel=1e-9)
        assert out["v"][i] == pytest.approx(np.linalg.inv(A)[-1, -1], rel=1e-10)


def test_h2_zero_is_ordinary_least_squares():
    """h2 = 0 makes M = I, so b_i is the OLS fit (numpy.linalg.lstsq)."""
    Phi, _, XL, y, XR = _rand_problem(n=60, seed=2)
    out = O.gls_sequence(Phi, 0.0, XL, y, XR)
    for i in range(XR.shape[0]):
        X = np.column_stack([XL, XR[i]])
        b, rss, *_ = np.linalg.lstsq(X, y, rcond=None)
        assert _relerr(out["b"][i], b) < 1e-11
        assert out["sigma2"][i] == pytest.approx(rss[0] / (60 - X.shape[1]), rel=1e-10)


def test_h2_one_uses_phi():
    """h2 = 1 makes M = Phi: compare with explicit Phi^-1 normal equations."""
    Phi, _, XL, y, XR = _rand_problem(n=30, m=4, seed=5)
    Pi = np.linalg.inv(Phi)
    out = O.gls_sequence(Phi, 1.0, XL, y, XR)
    for i in range(4):
        X = np.column_stack([XL, XR[i]])
        b = np.linalg.solve(X.T @ Pi @ X, X.T @ Pi @ y)
        assert _relerr(out["b"][i], b) < 1e-9


# -- closed form via partitioned (Frisch-Waugh-Lovell) regression -----------

def test_frisch_waugh_lovell_closed_form():
    Phi, h2, XL, y, XR = _rand_problem(n=50, m=20, seed=7)
    st = O.Study(Phi, h2, XL, y)
    blk = st.block(XR.T, keep=True)
    STL, rT, c, n, p = st.STL, st.rT, st.c, st.n, st.p
    a = np.linalg.solve(STL, rT)
    q = c - rT @ a
    for i in range(XR.shape[0]):
        sbl = blk["SBL"][i]
        w = np.linalg.solve(STL, sbl)
        schur = blk["SBR"][i] - sbl @ w
        num = blk["rB"][i] - sbl @ a
        bp = num / schur
        assert blk["b"][i, -1] == pytest.approx(bp, rel=1e-10)
        assert np.allclose(blk["b"][i, :-1], a - w * bp, rtol=1e-10, atol=1e-12 * np.abs(a).max())
        assert blk["v"][i] == pytest.approx(1 / schur, rel=1e-10)
        assert blk["sigma2"][i] == pytest.approx((q - num ** 2 / schur) / (n - p), rel=1e-10)
        rho = num ** 2 / (schur * q)
        t2 = O.t_squared(blk["b"][i:i + 1], blk["sigma2"][i:i + 1], blk["v"][i:i + 1])[0]
        assert t2 == pytest.approx((n - p) * rho / (1 - rho), rel=1e-9)


def test_sigma2_two_ways_and_alternative_products():
    """sigma2 from c - b^T r equals ||y~ - X~_i b_i||^2/(n-p); S_BL and r~_B equal
    x_i^T M^-1 X_L and x_i^T M^-1 y computed without the triangular solve."""
    Phi, h2, XL, y, XR = _rand_problem(n=45, m=8, seed=9)
    st = O.Study(Phi, h2, XL, y)
    blk = st.block(XR.T, keep=True)
    M = h2 * Phi + (1 - h2) * np.eye(45)
    MiXL = np.linalg.solve(M, XL)
    Miy = np.linalg.solve(M, y)
    for i in range(8):
        Xt = np.column_stack([st.XLt, blk["XRt"][:, i]])
        rss = np.sum((st.yt - Xt @ blk["b"][i]) ** 2)
        assert blk["sigma2"][i] == pytest.approx(rss / (45 - 4), rel=1e-9)
        assert np.allclose(blk["SBL"][i], XR[i] @ MiXL, rtol=1e-10)
        assert blk["rB"][i] == pytest.approx(XR[i] @ Miy, rel=1e-9, abs=1e-12)


# -- invariances of the GLS solution ---------------------------------------

def test_invariance_snp_scaling():
    Phi, h2, XL, y, XR = _rand_problem(seed=13)
    base = O.gls_sequence(Phi, h2, XL, y, XR)
    sc = O.gls_sequence(Phi, h2, XL, y, 3.0 * XR)
    assert np.allclose(sc["b"][:, -1], base["b"][:, -1] / 3.0, rtol=1e-11)
    assert np.allclose(sc["b"][:, :-1], base["b"][:, :-1], rtol=1e-10)
    assert np.allclose(sc["sigma2"], base["sigma2"], rtol=1e-10)
    assert np.allclose(O.t_squared(sc["b"], sc["sigma2"], sc["v"]),
                       O.t_squared(base["b"], base["sigma2"], base["v"]), rtol=1e-9)


def test_invariance_sample_permutation():
    """Reordering individuals consistently (rows of y, X_L, X_R; rows and
    columns of Phi) changes L but not the GLS solution."""
    Phi, h2, XL, y, XR = _rand_problem(seed=17)
    perm = np.random.default_rng(1).permutation(Phi.shape[0])
    base = O.gls_sequence(Phi, h2, XL, y, XR)
    pr = O.gls_sequence(Phi[np.ix_(perm, perm)], h2, XL[perm], y[perm], XR[:, perm])
    assert np.all(_relerr(pr["b"], base["b"]) < 1e-10)
    assert np.allclose(pr["sigma2"], base["sigma2"], rtol=1e-10)
    assert np.allclose(pr["v"], base["v"], rtol=1e-10)


def test_invariance_covariate_shift_and_phenotype_transform():
    Phi, h2, XL, y, XR = _rand_problem(seed=19)
    base = O.gls_sequence(Phi, h2, XL, y, XR)
    gamma = np.array([0.5, -1.5, 2.0])
    sh = O.gls_sequence(Phi, h2, XL, y, XR + (XL @ gamma)[None, :])
    assert np.allclose(sh["b"][:, -1], base["b"][:, -1], rtol=1e-9)
    assert np.allclose(sh["sigma2"], base["sigma2"], rtol=1e-9)
    yt = O.gls_sequence(Phi, h2, XL, -2.5 * y + XL @ gamma, XR)
    assert np.allclose(yt["b"][:, -1], -2.5 * base["b"][:, -1], rtol=1e-9)


def test_invariance_covariance_scaling():
    Phi, h2, XL, y, XR = _rand_problem(seed=23)
    M = h2 * Phi + (1 - h2) * np.eye(Phi.shape[0])
    base = O.gls_sequence(None, 0, XL, y, XR, M=M)
    sc = O.gls_sequence(None, 0, XL, y, XR, M=7.0 * M)
    assert np.all(_relerr(sc["b"], base["b"]) < 1e-11)
    assert np.allclose(sc["sigma2"], base["sigma2"] / 7.0, rtol=1e-10)


def test_exact_recovery():
    """y = X_j beta exactly: b_j = beta and sigma2_j ~ 0."""
    Phi, h2, XL, _, XR = _rand_problem(seed=29)
    beta = np.array([1.0, -0.5, 0.25, 2.0])
    y = np.column_stack([XL, XR[3]]) @ beta
    out = O.gls_sequence(Phi, h2, XL, y, XR)
    assert np.allclose(out["b"][3], beta, rtol=1e-10, atol=1e-12)
    assert abs(out["sigma2"][3]) < 1e-20 * max(1.0, y @ y) + 1e-24


def test_block_size_independence():
    Phi, h2, XL, y, XR = _rand_problem(m=23, seed=31)
    a = O.gls_sequence(Phi, h2, XL, y, XR, block_cols=4)
    b = O.gls_sequence(Phi, h2, XL, y, XR, block_cols=23)
    assert np.all(_relerr(a["b"], b["b"]) < 1e-13)


# -- failure handling ------------------------------------------------------

def test_degenerate_snp_flags_status():
    """A SNP collinear with the covariates (constant column with an intercept)
    or all zero makes S_i singular: status 1, NaN outputs, others untouched."""
    Phi, h2, XL, y, XR = _rand_problem(seed=37)
    XR[2] = 2.0
    XR[5] = 0.0
    XR[6] = XL[:, 1] * 4.0
    out = O.gls_sequence(Phi, h2, XL, y, XR)
    assert list(np.nonzero(out["status"])[0]) == [2, 5, 6]
    assert np.isnan(out["b"][[2, 5, 6]]).all() and np.isnan(out["sigma2"][[2, 5, 6]]).all()
    assert np.isfinite(out["b"][[0, 1, 3, 4, 7]]).all()


def test_not_spd_reports_pivot():
    Phi, _, XL, y, XR = _rand_problem(n=12, seed=41)
    M = np.eye(12)
    M[4, 4] = -1.0
    with pytest.raises(O.NotSPDError) as e:
        O.gls_sequence(None, 0, XL, y, XR, M=M)
    assert e.value.pivot == 5


def test_loss_is_sum_of_t_squared():
    Phi, h2, XL, y, XR = _rand_problem(seed=43)
    out = O.gls_sequence(Phi, h2, XL, y, XR)
    se = np.sqrt(out["sigma2"] * out["v"])
    assert O.loss_t2(out["b"], out["sigma2"], out["v"]) == pytest.approx(np.sum((out["b"][:, -1] / se) ** 2), rel=1e-13)
