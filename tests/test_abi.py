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


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("case", ["clockwise", "non_convex", "two_vertices", "wound_twice"])
def test_create_refuses_a_body_that_is_not_convex_and_counter_clockwise(case):
    """Argument checks run before any device call: a clockwise, non-convex, degenerate or
    doubly wound body polygon is refused with CC_ERR_ARG (its cut-cell geometry would be
    wrong without any error otherwise)."""
    import numpy as np
    from paper_1711_11361_amd import cc
    from paper_1711_11361_amd import workloads as W
    w = W.cylinder(nx=64, ny=32)
    if case == "clockwise":
        verts = W.triangle(0.2)[::-1]
    elif case == "non_convex":
        verts = np.array([[0.0, 0.0], [0.2, 0.0], [0.05, 0.05], [0.2, 0.2], [0.0, 0.2]])
    elif case == "two_vertices":
        verts = np.array([[0.0, 0.0], [0.2, 0.0]])
    else:
        a = 4.0 * np.pi * np.arange(10) / 10  # a decagon's vertices visited twice round
        verts = 0.1 * np.stack([np.cos(a), np.sin(a)], axis=1)
    b = dict(w["body"], verts=np.ascontiguousarray(verts, dtype=np.float64))
    cfg = cc.make_config(w["grid"])
    body, keep = cc.make_body(b)
    with pytest.raises(cc.CCError) as e:
        cc.cc_create(cfg, body, 0, 0, 0)
    assert e.value.status == cc.CC_ERR_ARG
    # the workload polygons themselves pass the same check
    for good in (W.circle(0.1, 1024), W.triangle(0.2), W.naca00(0.12, 1.0, 512, 0.25), W.half_plane_quad(2.0)):
        body, keep = cc.make_body(dict(w["body"], verts=good))
        with pytest.raises(cc.CCError) as e:
            cc.cc_create(cfg, body, 0, 0, 0)  # refused for the missing workspace, not the body
        assert e.value.status == cc.CC_ERR_WORKSPACE
