"""Copies overlap the solves in every streamed pass (Sec. 3.1, double buffering).

A streamed study given no copy stream runs on the handle's own compute and copy
streams, which gls_setup checks do not share a hardware queue.  Were copies and
solves on streams that share a queue, each block's copy would run after the
solve before it and a pass's device wall would approach its copies plus its
solves, about twice the solves at n = 10,000, where a block's copy takes about
as long as its product (a second live handle with an unchecked pair did exactly
that).
Here every pass of two live handles, used in turn, must stay within 1.4 times
its summed solve time (plus 5 ms for the opening copy), and all passes give
bitwise the same outputs.
"""
import numpy as np
import pytest
import torch

from paper_1302_4332_amd import synth
from paper_1302_4332_amd.gls import GLSContext

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_every_pass_overlaps_copies_and_solves():
    m = 24576
    st = synth.make_study("c1_n10k_m100k", m=m)
    Phi, XL, y = (torch.tensor(np.ascontiguousarray(a), device=DEV) for a in (st.Phi, st.XL, st.y))
    host = torch.from_numpy(st.snps(0, m)).pin_memory()
    ctxs = [GLSContext(Phi, st.w.h2, XL, y, block_cols=8192) for _ in range(2)]
    ref = None
    for k in range(8):
        ctx = ctxs[k % 2]
        out, stats = ctx.stream(host)
        print(f"pass {k}: wall {stats.wall_ms:.1f} ms, solves {stats.compute_ms:.1f} ms, {stats.blocks} blocks",
              flush=True)
        assert stats.blocks > 1
        assert stats.wall_ms <= 1.4 * stats.compute_ms + 5.0, "copies did not overlap the solves"
        got = [t.numpy().copy() for t in out]
        if ref is None:
            ref = got
        else:
            for a, b in zip(got, ref):
                assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    for ctx in ctxs:
        ctx.close()


def test_caller_streams_give_the_same_outputs():
    """A caller-given copy stream (and compute stream) runs the same kernels on
    the caller's streams: bitwise the outputs of the handle's own pair."""
    m = 3000
    st = synth.make_study("c0_small", m=m)
    Phi, XL, y = (torch.tensor(np.ascontiguousarray(a), device=DEV) for a in (st.Phi, st.XL, st.y))
    host = torch.from_numpy(st.snps(0, m)).pin_memory()
    ctx = GLSContext(Phi, st.w.h2, XL, y, block_cols=512)
    ref, _ = ctx.stream(host)
    cs, xs = torch.cuda.Stream(), torch.cuda.Stream()
    for kw in ({"copy_stream": xs}, {"compute_stream": cs, "copy_stream": xs}):
        got, stats = ctx.stream(host, **kw)
        assert stats.blocks == 6
        for a, b in zip(got, ref):
            assert np.array_equal(a.numpy().view(np.uint8), b.numpy().view(np.uint8))
    ctx.close()
