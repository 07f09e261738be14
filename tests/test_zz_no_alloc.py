"""The allocation-free entry point gls_solve_noalloc (GPU, through the C-ABI).

It runs gls_setup + gls_block with the library's static device scratch as
workspace.  Checked against gls_setup + gls_block through their own entry
points on the same inputs: b, sigma2, v and status bitwise equal, and both
against the CPU oracle at the plain-FP64 bar (per SNP, ||b_i - b_i,oracle||_inf
/ ||b_i,oracle||_inf <= 1e-10, relative 1e-10 on sigma2 and v, status exact).
Two calls in a row, the second a smaller study, so that what the first call
left in the shared scratch must not reach the second's results; then a
refined-FP32 call, and the size limit and argument errors.
"""
import numpy as np
import pytest
import torch

from oracle import gls_oracle as O
from paper_1302_4332_amd import synth
from paper_1302_4332_amd.gls import GLSContext, GLSError, NOALLOC_SCRATCH_BYTES, make_opts, solve_noalloc, \
    workspace_bytes
from parity_util import as_numpy, compare

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


def _problem(n, p, m, seed, h2):
    Phi = synth.kinship(n, seed)
    XL = synth.covariates(n, p, seed, "gauss")
    XL[:, 0] = 1.0
    y = synth.phenotype(n, seed)
    XR = synth.genotypes(n, 0, m, seed)
    return Phi, h2, XL, y, XR


def _outputs(m, p):
    return (torch.full((m, p), 7.0, dtype=torch.float64, device=DEV),
            torch.full((m,), 7.0, dtype=torch.float64, device=DEV),
            torch.full((m,), 7.0, dtype=torch.float64, device=DEV),
            torch.full((m,), 9, dtype=torch.int32, device=DEV))


def _noalloc(Phi, h2, XL, y, XR, bc, **kw):
    m, p = XR.shape[0], XL.shape[1] + 1
    out = _outputs(m, p)
    solve_noalloc(_t(Phi), h2, _t(XL), _t(y), _t(XR), *out, block_cols=bc, **kw)
    return as_numpy(out)


def _setup_block(Phi, h2, XL, y, XR, bc, **kw):
    ctx = GLSContext(_t(Phi), h2, _t(XL), _t(y), block_cols=bc, **kw)
    X = _t(XR)
    outs = [ctx.block(X[j:j + bc]) for j in range(0, X.shape[0], bc)]
    torch.cuda.synchronize()
    ctx.close()
    return as_numpy(tuple(torch.cat([o[i] for o in outs]) for i in range(4)))


def _bitwise(a, b):
    for k in ("b", "sigma2", "v", "status"):
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), f"{k} differs from gls_setup + gls_block"


@pytest.mark.parametrize("n,p,m,bc,h2", [
    (1100, 6, 700, 256, 0.5),   # several blocks, ragged last block
    (300, 3, 130, 64, 0.3),     # then a smaller study on the same scratch
])
def test_noalloc_matches_setup_block(n, p, m, bc, h2):
    Phi, h2, XL, y, XR = _problem(n, p, m, seed=n + 31, h2=h2)
    assert workspace_bytes(n, p, make_opts(bc)) <= NOALLOC_SCRATCH_BYTES
    g = _noalloc(Phi, h2, XL, y, XR, bc)
    ref = _setup_block(Phi, h2, XL, y, XR, bc)
    _bitwise(g, ref)
    err = compare(g, O.gls_sequence(Phi, h2, XL, y, XR), 1e-10)
    print(f"noalloc n={n} p={p} m={m}: bitwise equal to gls_setup + gls_block, max rel err b {err:.2e}", flush=True)


def test_noalloc_two_calls_in_a_row():
    big = _problem(1024, 4, 600, seed=5, h2=0.6)
    small = _problem(200, 2, 90, seed=6, h2=0.4)
    g1 = _noalloc(*big, 512)
    g2 = _noalloc(*small, 64)
    _bitwise(g1, _setup_block(*big, 512))
    _bitwise(g2, _setup_block(*small, 64))
    compare(g2, O.gls_sequence(*small), 1e-10)


def test_noalloc_refined_fp32():
    Phi, h2, XL, y, XR = _problem(700, 4, 300, seed=11, h2=0.45)
    g = _noalloc(Phi, h2, XL, y, XR, 128, precision="fp32_ir", refine_sweeps=2)
    _bitwise(g, _setup_block(Phi, h2, XL, y, XR, 128, precision="fp32_ir", refine_sweeps=2))
    compare(g, O.gls_sequence(Phi, h2, XL, y, XR), 1e-8)


def test_noalloc_limits_and_errors():
    Phi, h2, XL, y, XR = _problem(1600, 4, 8, seed=3, h2=0.5)
    assert workspace_bytes(1600, 4, make_opts(1024)) > NOALLOC_SCRATCH_BYTES
    with pytest.raises(GLSError) as e:
        _noalloc(Phi, h2, XL, y, XR, 1024)
    assert e.value.status == -4   # GLS_ERR_WORKSPACE
    with pytest.raises(GLSError) as e:
        _noalloc(Phi, 1.5, XL, y, XR, 8)
    assert e.value.status == -1
    # a non-SPD M reports its pivot, and the next call still works
    n = 64
    bad = np.eye(n)
    bad[10, 10] = -1.0
    with pytest.raises(GLSError) as e:
        _noalloc(bad, 1.0, XL[:n], y[:n], XR[:, :n], 8)
    assert e.value.status == -2 and e.value.info == 11
    small = _problem(150, 3, 20, seed=8, h2=0.5)
    compare(_noalloc(*small, 16), O.gls_sequence(*small), 1e-10)
    # m = 0: setup only, nothing written
    _noalloc(Phi[:300, :300], h2, XL[:300], y[:300], XR[:0, :300], 16)
