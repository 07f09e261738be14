"""Seeded synthetic GWAS inputs.

This module only draws inputs; it holds none of the GLS method's arithmetic
(no M, no Cholesky, no solves).  The same host arrays feed the HIP path and
the CPU oracle, so both sides always see bit-identical inputs.

Workloads (Sec. 1.3-1.4 fix n ~ 10,000 samples, p between 4 and 20, m in the
millions; the recipe below fills in what the paper leaves open):

* kinship Phi = G G^T / n_markers + ridge * I, with G an n x 2000 matrix of
  Binomial(2, f) genotypes (f ~ U(0.05, 0.5) per marker) whose columns are
  standardised with the empirical mean and population s.d.;
* covariates X_L = [1, sex ~ Bernoulli(0.5), age ~ N(50, 10)] (p = 4), or
  [1, N(0,1) x (p-2)] for the Gaussian kind;
* SNP dosages x_R,j ~ Binomial(2, f_j), f_j ~ U(0.05, 0.5) per SNP, stored as
  float64 (or uint8, or packed four to a byte) with each SNP's n samples
  contiguous, i.e. column-major n x m;
* phenotype y ~ N(0, 1), optionally plus effect * x_R,c for one causal SNP c.

Randomness is counter-addressed: SNP chunk k of a study draws from
``default_rng([seed, STREAM_XR, k])``, so any column range is reproducible on
its own, whatever block size a caller streams with.
"""
from __future__ import annotations

import concurrent.futures as _cf
import dataclasses
import os

import numpy as np

STREAM_KIN = 1
STREAM_XL = 2
STREAM_XR = 3
STREAM_Y = 4
STREAM_CAUSAL = 5
STREAM_JITTER = 6
SNP_CHUNK = 1024
BASE_SEED = 4332


@dataclasses.dataclass(frozen=True)
class Workload:
    """One study shape: sizes, heritability and generator options."""

    name: str
    n: int
    p: int
    m: int
    h2: float
    block_cols: int
    covariates: str = "sex_age"     # or "gauss"
    causal: bool = False
    effect: float = 0.3
    seed: int = BASE_SEED
    n_markers: int = 2000
    ridge: float = 1e-3


WORKLOADS = {
    "c0_small": Workload("c0_small", n=512, p=4, m=2048, h2=0.5, block_cols=2048,
                         seed=BASE_SEED + 0),
    "c1_n10k_m100k": Workload("c1_n10k_m100k", n=10000, p=4, m=100000, h2=0.4,
                              block_cols=8192, causal=True, seed=BASE_SEED + 1),
    "c2_n10k_m1M": Workload("c2_n10k_m1M", n=10000, p=4, m=1000000, h2=0.4,
                            block_cols=8192, seed=BASE_SEED + 2),
    "c3_grad_n4096": Workload("c3_grad_n4096", n=4096, p=4, m=16384, h2=0.3,
                              block_cols=8192, seed=BASE_SEED + 3),
    "c4_n20k_p8": Workload("c4_n20k_p8", n=20000, p=8, m=2000000, h2=0.4,
                           block_cols=16384, covariates="gauss", seed=BASE_SEED + 4),
}


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def kinship(n: int, seed: int, n_markers: int = 2000, ridge: float = 1e-3) -> np.ndarray:
    """Phi = G G^T / n_markers + ridge * I from standardised Binomial(2,f) markers."""
    rng = np.random.default_rng([seed, STREAM_KIN])
    f = rng.uniform(0.05, 0.5, size=n_markers)
    u1 = rng.random((n, n_markers))
    u2 = rng.random((n, n_markers))
    G = (u1 < f).astype(np.float64) + (u2 < f)
    mu = G.mean(axis=0)
    sd = G.std(axis=0)
    bad = sd == 0.0
    # a constant marker column cannot be standardised: redraw it
    while bad.any():
        k = int(bad.sum())
        G[:, bad] = (rng.random((n, k)) < f[bad]).astype(np.float64) + (rng.random((n, k)) < f[bad])
        mu = G.mean(axis=0)
        sd = G.std(axis=0)
        bad = sd == 0.0
    G = (G - mu) / sd
    Phi = (G @ G.T) / float(n_markers)
    Phi = 0.5 * (Phi + Phi.T)
    Phi[np.diag_indices(n)] += ridge
    return np.ascontiguousarray(Phi)


def covariates(n: int, p: int, seed: int, kind: str = "sex_age") -> np.ndarray:
    """X_L, n x (p-1), column-major (Fortran order)."""
    rng = np.random.default_rng([seed, STREAM_XL])
    XL = np.empty((n, p - 1), dtype=np.float64, order="F")
    if p == 1:
        return XL
    XL[:, 0] = 1.0
    if kind == "sex_age":
        if p != 4:
            raise ValueError("the sex/age covariate set has p = 4")
        XL[:, 1] = (rng.random(n) < 0.5).astype(np.float64)
        XL[:, 2] = rng.normal(50.0, 10.0, size=n)
    elif kind == "gauss":
        XL[:, 1:] = rng.standard_normal((n, p - 2))
    else:
        raise ValueError(kind)
    return XL


def _chunk(n: int, seed: int, k: int) -> np.ndarray:
    """SNP chunk k as uint8 dosages, shape (SNP_CHUNK, n) (one SNP per row)."""
    rng = np.random.default_rng([seed, STREAM_XR, k])
    f = rng.uniform(0.05, 0.5, size=SNP_CHUNK).astype(np.float32)[:, None]
    a = rng.random((SNP_CHUNK, n), dtype=np.float32) < f
    b = rng.random((SNP_CHUNK, n), dtype=np.float32) < f
    return a.astype(np.uint8) + b.astype(np.uint8)


def genotypes_u8(n: int, j0: int, j1: int, seed: int, out: np.ndarray | None = None) -> np.ndarray:
    """SNPs [j0, j1) as uint8 dosages, shape (j1-j0, n): SNP-major, samples contiguous."""
    cols = j1 - j0
    if out is None:
        out = np.empty((cols, n), dtype=np.uint8)
    k0, k1 = j0 // SNP_CHUNK, (j1 - 1) // SNP_CHUNK + 1 if cols > 0 else j0 // SNP_CHUNK

    def work(k):
        c = _chunk(n, seed, k)
        lo = max(j0, k * SNP_CHUNK)
        hi = min(j1, (k + 1) * SNP_CHUNK)
        out[lo - j0:hi - j0] = c[lo - k * SNP_CHUNK:hi - k * SNP_CHUNK]

    if k1 - k0 <= 2:
        for k in range(k0, k1):
            work(k)
    else:
        with _cf.ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(k0, k1)))
    return out


def genotypes(n: int, j0: int, j1: int, seed: int, out: np.ndarray | None = None) -> np.ndarray:
    """SNPs [j0, j1) as float64 dosages, shape (j1-j0, n) == column-major n x (j1-j0)."""
    g = genotypes_u8(n, j0, j1, seed)
    if out is None:
        return g.astype(np.float64)
    out[...] = g
    return out


def imputed_dosages(n: int, j0: int, j1: int, seed: int, kind: str = "jitter") -> np.ndarray:
    """Real-valued SNP columns [j0, j1), shape (j1-j0, n): the dosages of
    ``genotypes`` made non-integer, as imputed or normalised genotype data are.

    kind "jitter": dosage + U(-0.5, 0.5) (imputation-like expected dosages);
    kind "standardized": each SNP column centred and scaled to unit population
    s.d. (a constant column is left at zero)."""
    g = genotypes(n, j0, j1, seed)
    if kind == "jitter":
        for k in range(j0 // SNP_CHUNK, (j1 - 1) // SNP_CHUNK + 1 if j1 > j0 else 0):
            rng = np.random.default_rng([seed, STREAM_JITTER, k])
            u = rng.uniform(-0.5, 0.5, size=(SNP_CHUNK, n))
            lo, hi = max(j0, k * SNP_CHUNK), min(j1, (k + 1) * SNP_CHUNK)
            g[lo - j0:hi - j0] += u[lo - k * SNP_CHUNK:hi - k * SNP_CHUNK]
        return g
    if kind == "standardized":
        mu = g.mean(axis=1, keepdims=True)
        sd = g.std(axis=1, keepdims=True)
        return np.where(sd > 0, (g - mu) / np.where(sd > 0, sd, 1.0), 0.0)
    raise ValueError(kind)


def pack_dosages_2bit(g: np.ndarray) -> np.ndarray:
    """Packs uint8 dosages 0..3 of shape (cols, n) four to a byte, shape
    (cols, ceil(n / 4)): sample k in bits [2 (k % 4), 2 (k % 4) + 2) of byte
    k // 4; pad bits are zero.  A storage format only (the library's 2-bit
    entry points read it)."""
    g = np.ascontiguousarray(g, dtype=np.uint8)
    if g.ndim != 2:
        raise ValueError("g must be (cols, n)")
    if g.size and int(g.max()) > 3:
        raise ValueError("2-bit packing holds dosages 0..3 only")
    cols, n = g.shape
    q = (n + 3) // 4
    pad = np.zeros((cols, 4 * q), dtype=np.uint8)
    pad[:, :n] = g
    t = pad.reshape(cols, q, 4)
    return (t[:, :, 0] | (t[:, :, 1] << 2) | (t[:, :, 2] << 4) | (t[:, :, 3] << 6)).astype(np.uint8)


def phenotype(n: int, seed: int, x_causal: np.ndarray | None = None, effect: float = 0.3) -> np.ndarray:
    rng = np.random.default_rng([seed, STREAM_Y])
    y = rng.standard_normal(n)
    if x_causal is not None:
        y = y + effect * x_causal
    return y


def causal_index(m: int, seed: int) -> int:
    return int(np.random.default_rng([seed, STREAM_CAUSAL]).integers(0, m))


@dataclasses.dataclass
class Study:
    """The fixed per-study inputs plus a handle to draw SNP columns on demand."""

    w: Workload
    Phi: np.ndarray
    XL: np.ndarray
    y: np.ndarray
    causal: int | None

    def snps(self, j0: int, j1: int) -> np.ndarray:
        return genotypes(self.w.n, j0, j1, self.w.seed)

    def snps_u8(self, j0: int, j1: int) -> np.ndarray:
        return genotypes_u8(self.w.n, j0, j1, self.w.seed)

    def snps_u2(self, j0: int, j1: int) -> np.ndarray:
        return pack_dosages_2bit(genotypes_u8(self.w.n, j0, j1, self.w.seed))


def make_study(w: Workload | str, *, n: int | None = None, m: int | None = None,
               p: int | None = None, seed: int | None = None) -> Study:
    """Build the fixed inputs of a workload; n, m, p, seed may be overridden."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    kw = {}
    if n is not None:
        kw["n"] = n
    if m is not None:
        kw["m"] = m
    if p is not None:
        kw["p"] = p
    if seed is not None:
        kw["seed"] = seed
    if kw:
        w = dataclasses.replace(w, **kw)
    Phi = kinship(w.n, w.seed, w.n_markers, w.ridge)
    XL = covariates(w.n, w.p, w.seed, w.covariates)
    c = None
    xc = None
    if w.causal:
        c = causal_index(w.m, w.seed)
        xc = genotypes(w.n, c, c + 1, w.seed)[0]
    y = phenotype(w.n, w.seed, xc, w.effect)
    return Study(w, Phi, XL, y, c)
