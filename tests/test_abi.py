"""The C ABI: the built library loads and exports every function include/cc.h declares,
and the ctypes binding covers all of them (no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cc.h")
LIB = os.path.join(ROOT, "paper_1711_11361_amd", "libcutcell.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cc_[a-z_]+)\s*\(", src)))


def test_header_declares_the_step_api():
    names = declared()
    for n in ("cc_geometry", "cc_sweep", "cc_step", "cc_cfl_dt", "cc_create", "cc_workspace_bytes"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_covers_every_symbol_and_workspace_query():
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W
    assert set(declared()) == set(cc.EXPORTED)
    w = W.cylinder()
    cfg = cc.make_config(w["grid"])
    body, keep = cc.make_body(w["body"])
    n64 = cc.cc_workspace_bytes(cfg, body)
    cfg32 = cc.make_config(w["grid"], cc.CC_FP32_GEOM64)
    n32 = cc.cc_workspace_bytes(cfg32, body)
    nc = 1024 * 512
    # two FP64 state buffers plus three geometry levels at least
    assert n64 >= 2 * 32 * nc + 3 * (8 + 16 + 16) * nc
    assert n64 - n32 == pytest.approx(2 * 16 * nc, rel=0.01)
