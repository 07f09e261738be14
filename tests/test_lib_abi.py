"""CPU checks of the C-ABI library: it loads, exports what include/gls.h
declares, and its host-only planning calls behave (no GPU needed)."""
import os
import re

import pytest

from paper_1302_4332_amd import gls

HEADER = os.path.join(os.path.dirname(__file__), "..", "include", "gls.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gls_[a-z0-9_]+)\s*\(", text)))


def test_header_matches_binding():
    assert set(_declared()) == set(gls.SIGNATURES)


def test_library_exports_every_declared_symbol():
    L = gls.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_workspace_planning():
    o = gls.make_opts(8192)
    assert gls.workspace_bytes(10000, 4, o) > 2 * 8 * 10240 * 10240
    assert gls.workspace_bytes(10000, 4, o) % 256 == 0
    assert gls.workspace_bytes(10, 10, o) == 0          # n <= p
    assert gls.workspace_bytes(100, 0, o) == 0          # p < 1
    assert gls.workspace_bytes(100, 21, o) == 0         # p > 20
    assert gls.workspace_bytes(2 ** 20 + 1, 4, o) == 0  # n above the supported 2^20
    assert gls.workspace_bytes(100, 20, o) > 0          # p = 20, the largest supported
    assert gls.workspace_bytes(100, 4, gls.make_opts(0)) == 0
    assert gls.workspace_bytes(100, 4, gls.make_opts(16, refine_sweeps=9)) == 0
    small = gls.workspace_bytes(512, 4, gls.make_opts(64))
    big = gls.workspace_bytes(512, 4, gls.make_opts(4096))
    assert big > small


def test_status_strings():
    L = gls.lib()
    for code in gls.STATUS:
        assert L.gls_status_string(code)
