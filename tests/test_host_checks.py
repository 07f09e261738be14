"""CPU checks of host-side behaviour that runs before any GPU call: the
binding's argument checks and bench.py's refusal of several GPUs."""
import os
import subprocess
import sys

import pytest
import torch

from paper_1302_4332_amd.gls import GLSContext, stream_grad, t2_loss

ROOT = os.path.join(os.path.dirname(__file__), "..")


def test_context_needs_device_tensors():
    Phi = torch.eye(8, dtype=torch.float64)
    with pytest.raises(TypeError, match="Phi must be a CUDA"):
        GLSContext(Phi, 0.5, None, torch.zeros(8, dtype=torch.float64), block_cols=4)


def test_stream_grad_needs_fp64_snps():
    Phi = torch.eye(8, dtype=torch.float64)
    y = torch.zeros(8, dtype=torch.float64)
    with pytest.raises(TypeError, match="XR_host must be torch.float64"):
        stream_grad(Phi, 0.5, None, y, torch.zeros((4, 8), dtype=torch.uint8), t2_loss, block_cols=4)


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_bench_refuses_several_gpus(argv, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], cwd=ROOT, capture_output=True,
                       text=True, timeout=120, env={**os.environ, **env})
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
