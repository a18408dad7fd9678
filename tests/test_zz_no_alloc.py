"""cc_totals_state, the entry point that allocates nothing (its partial sums live in the
library's per-device scratch array), against cc_totals of the same state: bit for bit,
on two calls in a row, the second with a smaller state, in both precisions."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_1711_11361_amd import cc  # noqa: E402
from paper_1711_11361_amd import workloads as W  # noqa: E402


def stepped(w, precision, nsteps):
    s = cc.Solver(w["grid"], w["body"], precision=precision)
    s.set_prim(w["prim"])
    for _ in range(nsteps):
        s.step(s.cfl_dt(w["cfl"]))
    return s


def cell_sizes(g):
    return (g["x_hi"] - g["x_lo"]) / g["nx"], (g["y_hi"] - g["y_lo"]) / g["ny"]


def test_totals_without_allocation_equal_cc_totals():
    cases = [(W.cylinder(nx=256, ny=128), cc.CC_FP32_GEOM64, 5),  # first call: the larger state
             (W.piston(nx=61, ny=17), cc.CC_FP64, 4)]             # second call: a smaller one
    stream = torch.cuda.Stream()
    for w, prec, n in cases:
        s = stepped(w, prec, n)
        want = s.totals()
        U64 = s.get_u_tensor()  # the state as FP64 planes (exact for FP32 state)
        torch.cuda.synchronize()
        nx, ny = w["grid"]["nx"], w["grid"]["ny"]
        hx, hy = cell_sizes(w["grid"])
        inputs = [(U64, cc.CC_FP64)]
        if prec == cc.CC_FP32_GEOM64:
            inputs.append((U64.to(torch.float32), cc.CC_FP32_GEOM64))  # the FP32 planes themselves
        for U, p in inputs:
            out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                cc.cc_totals_state(U.data_ptr(), p, nx, ny, hx, hy, stream.cuda_stream, out.data_ptr())
            stream.synchronize()
            got = out.cpu().numpy()
            assert np.array_equal(got, want), (w["name"], p, got, want)
        s.close()


def test_refusals():
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    u = torch.zeros(4 * 8, dtype=torch.float64, device="cuda")
    for args, st in (((0, cc.CC_FP64, 2, 4), cc.CC_ERR_ARG), ((u.data_ptr(), 7, 2, 4), cc.CC_ERR_ARG),
                     ((u.data_ptr(), cc.CC_FP64, 0, 4), cc.CC_ERR_ARG),
                     ((u.data_ptr(), cc.CC_FP64, 65536, 65536), cc.CC_ERR_UNSUPPORTED)):
        with pytest.raises(cc.CCError) as e:
            cc.cc_totals_state(*args, 1.0, 1.0, 0, out.data_ptr())
        assert e.value.status == st
