"""ctypes binding of libcutcell.so (C ABI in include/cc.h), with the same function names.

Only argument marshalling happens here: device memory comes from torch tensors (their
data pointers and the current HIP stream are passed through); every step of the method
runs in the library's kernels.  Importing fails loudly when the library is missing.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libcutcell.so")

CC_OK, CC_ERR_ARG, CC_ERR_DEVICE, CC_ERR_WORKSPACE, CC_ERR_STATE, CC_ERR_MOTION, CC_ERR_UNSUPPORTED = range(7)
CC_FP64, CC_FP32_GEOM64 = 0, 1
STATUS_NAMES = {0: "CC_OK", 1: "CC_ERR_ARG", 2: "CC_ERR_DEVICE", 3: "CC_ERR_WORKSPACE", 4: "CC_ERR_STATE",
                5: "CC_ERR_MOTION", 6: "CC_ERR_UNSUPPORTED"}


class cc_config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("bc", C.c_int32 * 4), ("precision", C.c_int32),
                ("options", C.c_int32), ("x_lo", C.c_double), ("x_hi", C.c_double), ("y_lo", C.c_double),
                ("y_hi", C.c_double), ("gamma", C.c_double), ("alpha_min", C.c_double)]


class cc_body(C.Structure):
    _fields_ = [("nverts", C.c_int32), ("pad_", C.c_int32), ("verts", C.POINTER(C.c_double)),
                ("ref_x", C.c_double), ("ref_y", C.c_double), ("theta0", C.c_double), ("vx", C.c_double),
                ("vy", C.c_double), ("pitch_amp", C.c_double), ("pitch_omega", C.c_double)]


class CCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIBPATH):
    raise ImportError(f"libcutcell.so not built ({LIBPATH}); run paper_1711_11361_amd/build.py")

# torch brings its own HIP runtime; load it first so that the library binds to the same
# runtime instance (a second instance would not see the device).
import torch  # noqa: E402,F401

_lib = C.CDLL(LIBPATH)
_vp, _d, _i32 = C.c_void_p, C.c_double, C.c_int32
_sig = {
    "cc_workspace_bytes": (C.c_size_t, [C.POINTER(cc_config), C.POINTER(cc_body)]),
    "cc_create": (C.c_int, [C.POINTER(cc_config), C.POINTER(cc_body), _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "cc_workspace_bytes_bodies": (C.c_size_t, [C.POINTER(cc_config), C.POINTER(cc_body), _i32]),
    "cc_create_bodies": (C.c_int, [C.POINTER(cc_config), C.POINTER(cc_body), _i32, _vp, C.c_size_t, _vp,
                                   C.POINTER(_vp)]),
    "cc_destroy": (C.c_int, [_vp]),
    "cc_set_state": (C.c_int, [_vp, _vp, _d]),
    "cc_set_clock": (C.c_int, [_vp, _d, C.c_int64]),
    "cc_set_u": (C.c_int, [_vp, _vp]),
    "cc_get_state": (C.c_int, [_vp, _vp, _i32]),
    "cc_geometry": (C.c_int, [_vp, _d, _i32]),
    "cc_geometry_dump": (C.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cc_begin_step": (C.c_int, [_vp, _d]),
    "cc_sweep": (C.c_int, [_vp, _i32, _d]),
    "cc_end_step": (C.c_int, [_vp]),
    "cc_step": (C.c_int, [_vp, _d]),
    "cc_cfl_dt": (C.c_int, [_vp, _d, C.POINTER(_d), _vp]),
    "cc_advance": (C.c_int, [_vp, _i32, _d, C.POINTER(_d), C.POINTER(C.c_float), C.POINTER(_i32)]),
    "cc_totals": (C.c_int, [_vp, C.POINTER(_d), C.POINTER(_d)]),
    "cc_set_budget": (C.c_int, [_vp, _i32]),
    "cc_totals_state": (C.c_int, [_vp, _i32, _i32, _i32, _d, _d, _vp, _vp]),
    "cc_surface_loads": (C.c_int, [_vp, C.POINTER(_d)]),
    "cc_body_loads": (C.c_int, [_vp, _i32, C.POINTER(_d)]),
    "cc_surface_pressure": (C.c_int, [_vp, C.c_void_p, _i32, C.POINTER(_i32)]),
    "cc_info": (C.c_int, [_vp, C.POINTER(_d), _i32]),
    "cc_autotune": (C.c_int, [_vp, _i32, C.POINTER(_i32), C.c_char_p]),
    "cc_set_tiles": (C.c_int, [_vp, _i32, _i32]),
    "cc_set_launch_mode": (C.c_int, [_vp, _i32]),
    "cc_timing": (C.c_int, [_vp, _i32]),
    "cc_timing_read": (C.c_int, [_vp, C.POINTER(_d), _i32]),
    "cc_last_error": (C.c_char_p, [_vp]),
    "cc_batch_workspace_bytes": (C.c_size_t, [_i32]),
    "cc_batch_create": (C.c_int, [_i32, _i32, _vp, C.c_size_t, _vp, C.POINTER(_vp)]),
    "cc_batch_destroy": (C.c_int, [_vp]),
    "cc_batch_add": (C.c_int, [_vp, _vp]),
    "cc_batch_remove": (C.c_int, [_vp, _vp]),
    "cc_batch_size": (_i32, [_vp]),
    "cc_batch_set_tiles": (C.c_int, [_vp, _i32, _i32]),
    "cc_batch_autotune": (C.c_int, [_vp, _i32, C.POINTER(_i32), C.c_char_p]),
    "cc_batch_set_launch_mode": (C.c_int, [_vp, _i32]),
    "cc_batch_step": (C.c_int, [_vp, C.POINTER(_d), C.POINTER(_i32)]),
    "cc_batch_last_dt": (C.c_int, [_vp, _d, C.POINTER(_d), C.POINTER(_i32)]),
    "cc_batch_cfl_dt": (C.c_int, [_vp, _d, C.POINTER(_d)]),
    "cc_batch_advance": (C.c_int, [_vp, _i32, _d, C.POINTER(_d), C.POINTER(C.c_float), C.POINTER(_i32)]),
    "cc_batch_last_error": (C.c_char_p, [_vp]),
    "cc_batch_timing": (C.c_int, [_vp, _i32]),
    "cc_batch_timing_read": (C.c_int, [_vp, C.POINTER(_d), _i32]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


def _check(ctx, st):
    if st != CC_OK:
        raw = _lib.cc_last_error(ctx)
        raise CCError(st, raw.decode() if raw else "")


def make_config(grid, precision=CC_FP64):
    c = cc_config()
    c.nx, c.ny = grid["nx"], grid["ny"]
    for k, v in enumerate(grid.get("bc", (0, 0, 0, 0))):
        c.bc[k] = v
    c.precision = precision
    c.options = 1 if grid.get("axisymmetric", False) else 0
    c.x_lo, c.x_hi, c.y_lo, c.y_hi = grid["x_lo"], grid["x_hi"], grid["y_lo"], grid["y_hi"]
    c.gamma = grid.get("gamma", 1.4)
    c.alpha_min = grid.get("alpha_min", 0.0)
    return c


def make_body(body):
    b = cc_body()
    keep = None
    if body is not None and len(body["verts"]) > 0:
        keep = np.ascontiguousarray(np.asarray(body["verts"], dtype=np.float64).reshape(-1))
        b.nverts = len(keep) // 2
        b.verts = keep.ctypes.data_as(C.POINTER(C.c_double))
        b.ref_x, b.ref_y = body.get("ref", (0.0, 0.0))
        b.theta0 = body.get("theta0", 0.0)
        b.vx, b.vy = body.get("vel", (0.0, 0.0))
        b.pitch_amp = body.get("pitch_amp", 0.0)
        b.pitch_omega = body.get("pitch_omega", 0.0)
    return b, keep


def make_bodies(bodies):
    """A cc_body array for several bodies (and the vertex arrays it points to)."""
    arr = (cc_body * len(bodies))()
    keep = []
    for k, bd in enumerate(bodies):
        b, v = make_body(bd)
        arr[k] = b
        keep.append(v)
    return arr, keep


# ----------------------------------------------------------------- C-ABI mirrors
def cc_workspace_bytes(cfg, body):
    return _lib.cc_workspace_bytes(C.byref(cfg), C.byref(body))


def cc_workspace_bytes_bodies(cfg, bodies, n):
    return _lib.cc_workspace_bytes_bodies(C.byref(cfg), bodies, n)


def cc_create_bodies(cfg, bodies, n, d_ws, ws_bytes, stream):
    out = _vp()
    _check(None, _lib.cc_create_bodies(C.byref(cfg), bodies, n, _vp(d_ws), ws_bytes, _vp(stream), C.byref(out)))
    return out


def cc_create(cfg, body, d_ws, ws_bytes, stream):
    out = _vp()
    _check(None, _lib.cc_create(C.byref(cfg), C.byref(body), _vp(d_ws), ws_bytes, _vp(stream), C.byref(out)))
    return out


def cc_destroy(ctx):
    _check(None, _lib.cc_destroy(ctx))


def cc_set_state(ctx, d_prim, t0):
    _check(ctx, _lib.cc_set_state(ctx, _vp(d_prim), t0))


def cc_set_clock(ctx, t, step):
    _check(ctx, _lib.cc_set_clock(ctx, float(t), int(step)))


def cc_set_u(ctx, d_u):
    _check(ctx, _lib.cc_set_u(ctx, _vp(d_u)))


def cc_get_state(ctx, d_out, what):
    _check(ctx, _lib.cc_get_state(ctx, _vp(d_out), what))


def cc_geometry(ctx, t, level):
    _check(ctx, _lib.cc_geometry(ctx, t, level))


def cc_geometry_dump(ctx, level, d_vcls, d_alpha, d_bx, d_by, d_cut=None, d_ncut=None):
    _check(ctx, _lib.cc_geometry_dump(ctx, level, _vp(d_vcls), _vp(d_alpha), _vp(d_bx), _vp(d_by), _vp(d_cut),
                                      _vp(d_ncut)))


def cc_begin_step(ctx, dt):
    _check(ctx, _lib.cc_begin_step(ctx, dt))


def cc_sweep(ctx, d, dt):
    _check(ctx, _lib.cc_sweep(ctx, d, dt))


def cc_end_step(ctx):
    _check(ctx, _lib.cc_end_step(ctx))


def cc_step(ctx, dt):
    _check(ctx, _lib.cc_step(ctx, dt))


def cc_cfl_dt(ctx, cfl, d_dt=None):
    """Host time step; with d_dt (a device pointer) only the asynchronous device output."""
    if d_dt is not None:
        _check(ctx, _lib.cc_cfl_dt(ctx, cfl, None, _vp(d_dt)))
        return None
    out = _d()
    _check(ctx, _lib.cc_cfl_dt(ctx, cfl, C.byref(out), None))
    return out.value


def cc_advance(ctx, nsteps, cfl, want_dt=True, want_ms=False):
    """Returns (steps done, dts or None, per-step device ms or None); raises CCError when a
    step is refused (the exception carries .done, the steps completed before it)."""
    dts = (_d * max(nsteps, 1))() if want_dt else None
    ms = (C.c_float * max(nsteps, 1))() if want_ms else None
    done = _i32()
    st = _lib.cc_advance(ctx, nsteps, cfl, dts, ms, C.byref(done))
    if st != CC_OK:
        raw = _lib.cc_last_error(ctx)
        err = CCError(st, raw.decode() if raw else "")
        err.done = done.value
        raise err
    n = done.value
    return n, (np.array(dts[:n]) if want_dt else None), (np.array(ms[:n]) if want_ms else None)


def cc_surface_loads(ctx):
    out = (_d * 4)()
    _check(ctx, _lib.cc_surface_loads(ctx, out))
    return np.array(out[:])


def cc_surface_pressure(ctx, d_out, max_records):
    """Number of wall cells at level n; the first max_records records (6 doubles each) go to
    device pointer d_out."""
    n = _i32(0)
    _check(ctx, _lib.cc_surface_pressure(ctx, d_out, int(max_records), C.byref(n)))
    return n.value


def cc_totals(ctx, with_budget=False):
    """Totals (4 components); with_budget: also (boundary, wall, lost), 4 components each."""
    out = (_d * 4)()
    bud = (_d * 12)() if with_budget else None
    _check(ctx, _lib.cc_totals(ctx, out, bud))
    if not with_budget:
        return np.array(out[:])
    b = np.array(bud[:])
    return np.array(out[:]), (b[0:4], b[4:8], b[8:12])


def cc_set_budget(ctx, on):
    _check(ctx, _lib.cc_set_budget(ctx, int(bool(on))))


def cc_totals_state(d_u, precision, nx, ny, hx, hy, stream, d_out4):
    """Totals of a state held outside any context (device pointers), asynchronous on
    `stream`; allocates nothing."""
    _check(None, _lib.cc_totals_state(_vp(d_u), int(precision), int(nx), int(ny), float(hx), float(hy),
                                      _vp(stream), _vp(d_out4)))


def cc_info(ctx):
    out = (_d * 11)()
    _check(ctx, _lib.cc_info(ctx, out, 11))
    v = out[:]
    return {"t": v[0], "steps": int(v[1]), "parity": int(v[2]), "status": int(v[3]), "collapses": int(v[4]),
            "box_cells": int(v[5]), "capacity": int(v[6]), "tile_x_rows": int(v[7]), "tile_y_rows": int(v[8]),
            "tile_y_walk": bool(v[9]), "x_with_box": bool(v[10])}


def cc_set_tiles(ctx, tile_x, tile_y):
    _check(ctx, _lib.cc_set_tiles(ctx, int(tile_x), int(tile_y)))


def cc_autotune(ctx, reps=20, cache_path=None):
    out = (_i32 * 2)()
    _check(ctx, _lib.cc_autotune(ctx, int(reps), out, cache_path.encode() if cache_path else None))
    return out[0], out[1]


def cc_batch_autotune(b, reps=20, cache_path=None):
    out = (_i32 * 2)()
    _bcheck(b, _lib.cc_batch_autotune(b, int(reps), out, cache_path.encode() if cache_path else None))
    return out[0], out[1]


CC_LAUNCH_PER_PHASE, CC_LAUNCH_PERSISTENT = 0, 1


def cc_set_launch_mode(ctx, mode):
    _check(ctx, _lib.cc_set_launch_mode(ctx, int(mode)))


def cc_batch_set_launch_mode(b, mode):
    _bcheck(b, _lib.cc_batch_set_launch_mode(b, int(mode)))


def cc_timing(ctx, enable):
    _check(ctx, _lib.cc_timing(ctx, int(enable)))


def cc_timing_read(ctx):
    out = (_d * 8)()
    _check(ctx, _lib.cc_timing_read(ctx, out, 8))
    v = out[:]
    return {"dense_x": (v[0], v[1]), "dense_y": (v[2], v[3]), "box": (v[4], v[5]), "geometry": (v[6], v[7])}


def cc_batch_timing(b, enable):
    _bcheck(b, _lib.cc_batch_timing(b, int(enable)))


def cc_batch_timing_read(b):
    out = (_d * 8)()
    _bcheck(b, _lib.cc_batch_timing_read(b, out, 8))
    v = out[:]
    return {"dense_x": (v[0], v[1]), "dense_y": (v[2], v[3]), "box": (v[4], v[5]), "geometry": (v[6], v[7])}


def _bcheck(b, st):
    if st != CC_OK:
        raw = _lib.cc_batch_last_error(b)
        raise CCError(st, raw.decode() if raw else "")


def cc_batch_workspace_bytes(max_instances):
    return _lib.cc_batch_workspace_bytes(int(max_instances))


def cc_batch_create(max_instances, precision, d_ws, ws_bytes, stream):
    out = _vp()
    _bcheck(None, _lib.cc_batch_create(int(max_instances), int(precision), _vp(d_ws), ws_bytes, _vp(stream),
                                       C.byref(out)))
    return out


def cc_batch_destroy(b):
    _bcheck(b, _lib.cc_batch_destroy(b))


def cc_batch_add(b, ctx):
    _bcheck(b, _lib.cc_batch_add(b, ctx))


def cc_batch_remove(b, ctx):
    _bcheck(b, _lib.cc_batch_remove(b, ctx))


def cc_batch_size(b):
    return int(_lib.cc_batch_size(b))


def cc_batch_set_tiles(b, tile_x, tile_y):
    _bcheck(b, _lib.cc_batch_set_tiles(b, int(tile_x), int(tile_y)))


def cc_batch_step(b, dts):
    n = len(dts)
    d = (_d * max(n, 1))(*dts)
    st = (_i32 * max(n, 1))()
    _bcheck(b, _lib.cc_batch_step(b, d, st))
    return list(st[:n])


def cc_batch_last_dt(b, cfl, n):
    d = (_d * max(n, 1))()
    st = (_i32 * max(n, 1))()
    _bcheck(b, _lib.cc_batch_last_dt(b, cfl, d, st))
    return list(d[:n]), list(st[:n])


def cc_batch_advance(b, nsteps, cfl, n, want_ms=False):
    """Returns (per-member time steps as a list of arrays, per-step ms or None, done list);
    raises CCError on a refused step (with .done, the per-member steps completed)."""
    dts = (_d * max(n * nsteps, 1))()
    ms = (C.c_float * max(nsteps, 1))() if want_ms else None
    done = (_i32 * max(n, 1))()
    st = _lib.cc_batch_advance(b, nsteps, cfl, dts, ms, done)
    dn = list(done[:n])
    if st != CC_OK:
        raw = _lib.cc_batch_last_error(b)
        err = CCError(st, raw.decode() if raw else "")
        err.done = dn
        raise err
    out = [np.array(dts[k * nsteps: k * nsteps + dn[k]]) for k in range(n)]
    return out, (np.array(ms[:nsteps]) if want_ms else None), dn


def cc_batch_cfl_dt(b, cfl, n):
    d = (_d * max(n, 1))()
    _bcheck(b, _lib.cc_batch_cfl_dt(b, cfl, d))
    return list(d[:n])


# ----------------------------------------------------------------- torch-backed solver
class Solver:
    """A simulation context whose device memory (workspace, I/O buffers) is owned by torch
    on `device`.  It runs on a stream of its own (a captured step needs a stream other than
    the null stream); the binding's tensor copies run on that stream too."""

    def __init__(self, grid, body=None, precision=CC_FP64, device="cuda:0", bodies=None):
        """bodies: a list of two to four body dicts, each with its own motion (instead of
        `body`)."""
        import torch
        self.torch = torch
        self.grid = dict(grid)
        self.nx, self.ny = grid["nx"], grid["ny"]
        self.precision = precision
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)
        self._cfg = make_config(grid, precision)
        if bodies is not None:
            self._body, self._verts = make_bodies(bodies)
            self.ws_bytes = cc_workspace_bytes_bodies(self._cfg, self._body, len(bodies))
        else:
            self._body, self._verts = make_body(body)
            self.ws_bytes = cc_workspace_bytes(self._cfg, self._body)
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            self._io = torch.empty((4, self.ny, self.nx), dtype=torch.float64, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        if bodies is not None:
            self.ctx = cc_create_bodies(self._cfg, self._body, len(bodies), self._ws_ptr, self.ws_bytes,
                                        self.stream.cuda_stream)
        else:
            self.ctx = cc_create(self._cfg, self._body, self._ws_ptr, self.ws_bytes, self.stream.cuda_stream)

    @staticmethod
    def device_bytes(grid, body=None, precision=CC_FP64):
        """Device memory one Solver allocates: the library's workspace (plus the alignment
        pad) and the FP64 input/output buffer of four planes."""
        cfg = make_config(grid, precision)
        b, _ = make_body(body)
        return cc_workspace_bytes(cfg, b) + 256 + 4 * 8 * grid["nx"] * grid["ny"]

    def close(self):
        if getattr(self, "ctx", None):
            cc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _on_stream(self):
        return self.torch.cuda.stream(self.stream)

    def set_prim(self, prim, t0=0.0):
        with self._on_stream():
            self._io.copy_(self.torch.as_tensor(np.asarray(prim, dtype=np.float64).reshape(4, self.ny, self.nx)))
            cc_set_state(self.ctx, self._io.data_ptr(), t0)

    def set_clock(self, t, step):
        """Resume at time t after `step` split steps; set the state afterwards."""
        cc_set_clock(self.ctx, t, step)

    def set_u(self, U):
        with self._on_stream():
            self._io.copy_(self.torch.as_tensor(np.asarray(U, dtype=np.float64).reshape(4, self.ny, self.nx)))
            cc_set_u(self.ctx, self._io.data_ptr())

    def get_u_tensor(self):
        """Conserved state as an FP64 tensor, valid on this solver's stream."""
        with self._on_stream():
            out = self.torch.empty((4, self.ny, self.nx), dtype=self.torch.float64, device=self.device)
            cc_get_state(self.ctx, out.data_ptr(), 1)
        return out

    def get_u(self):
        with self._on_stream():
            return self.get_u_tensor().cpu().numpy()

    def get_prim(self):
        with self._on_stream():
            out = self.torch.empty((4, self.ny, self.nx), dtype=self.torch.float64, device=self.device)
            cc_get_state(self.ctx, out.data_ptr(), 0)
            return out.cpu().numpy()

    def geometry(self, t, level=0):
        cc_geometry(self.ctx, t, level)

    def geometry_dump(self, level=0):
        t = self.torch
        nx, ny = self.nx, self.ny
        with self._on_stream():
            vc = t.empty((ny + 1, nx + 1), dtype=t.int8, device=self.device)
            al = t.empty((ny, nx), dtype=t.float64, device=self.device)
            bx = t.empty((ny, nx + 1), dtype=t.float64, device=self.device)
            by = t.empty((ny + 1, nx), dtype=t.float64, device=self.device)
            cut = t.empty(nx * ny, dtype=t.int32, device=self.device)
            ncut = t.empty(1, dtype=t.int32, device=self.device)
            cc_geometry_dump(self.ctx, level, vc.data_ptr(), al.data_ptr(), bx.data_ptr(), by.data_ptr(),
                             cut.data_ptr(), ncut.data_ptr())
            n = int(ncut.cpu().item())
            return {"vcls": vc.cpu().numpy(), "alpha": al.cpu().numpy(), "bx": bx.cpu().numpy(),
                    "by": by.cpu().numpy(), "cut": cut[:n].cpu().numpy()}

    def begin_step(self, dt):
        cc_begin_step(self.ctx, dt)

    def sweep(self, d, dt):
        cc_sweep(self.ctx, d, dt)

    def end_step(self):
        cc_end_step(self.ctx)

    def step(self, dt):
        cc_step(self.ctx, dt)

    def cfl_dt(self, cfl):
        return cc_cfl_dt(self.ctx, cfl)

    def advance(self, nsteps, cfl, want_ms=False):
        """nsteps CFL steps planned on the device; returns (dts, per-step ms or None)."""
        _, dts, ms = cc_advance(self.ctx, nsteps, cfl, True, want_ms)
        return dts, ms

    def totals(self):
        return cc_totals(self.ctx)

    def set_budget(self, on=True):
        """Track the conservation budget from now on (resets it)."""
        cc_set_budget(self.ctx, on)

    def budget(self):
        """(boundary, wall, lost) since the state was set, as the oracle's budget()."""
        return cc_totals(self.ctx, True)[1]

    def surface_loads(self):
        """(Fx, Fy, Mz about the pose origin, sum p*|N|) of the gas on the body at level n."""
        return cc_surface_loads(self.ctx)

    def body_loads(self, body):
        """surface_loads of one body of several (the wall cells it cuts; moment about its origin)."""
        out = np.zeros(4)
        _check(self.ctx, _lib.cc_body_loads(self.ctx, int(body), out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def surface_pressure(self):
        """Wall cells at level n in increasing index: rows (index, wall x, wall y, p*, Nx, Ny)."""
        n = cc_surface_pressure(self.ctx, None, 0)
        with self._on_stream():
            out = self.torch.empty((max(n, 1), 6), dtype=self.torch.float64, device=self.device)
            n2 = cc_surface_pressure(self.ctx, out.data_ptr(), n)
            assert n2 == n
            return out[:n].cpu().numpy()

    def info(self):
        return cc_info(self.ctx)

    def set_tiles(self, tile_x, tile_y):
        cc_set_tiles(self.ctx, tile_x, tile_y)

    def set_launch_mode(self, mode):
        cc_set_launch_mode(self.ctx, mode)

    def autotune(self, reps=20, cache_path=None):
        """Pick the fastest dense-sweep tile shapes for this grid (needs a state); with a
        cache file, a configuration tuned before is taken from it."""
        return cc_autotune(self.ctx, reps, cache_path)

    def cfl_dt_device(self, cfl, out):
        """The time step into a one-element FP64 device tensor, asynchronously."""
        cc_cfl_dt(self.ctx, cfl, out.data_ptr())

    @property
    def parity(self):
        return self.info()["parity"]

    def run(self, cfl, nsteps=None, t_end=None, dts=None):
        used = []
        k = 0
        while True:
            if dts is not None:
                if k >= len(dts):
                    break
                dt = dts[k]
            else:
                if nsteps is not None and k >= nsteps:
                    break
                dt = self.cfl_dt(cfl)
                if t_end is not None:
                    t = self.info()["t"]
                    if t >= t_end * (1 - 1e-14):
                        break
                    dt = min(dt, t_end - t)
            self.step(dt)
            used.append(dt)
            k += 1
        return used


class Batch:
    """Contexts of one precision stepped together (continuous batching): one launch per
    phase over all members, a captured graph per membership.  Device memory is owned by
    torch; the batch runs on a stream of its own."""

    def __init__(self, max_instances, precision=CC_FP64, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)
        self.max_instances = int(max_instances)
        nbytes = cc_batch_workspace_bytes(max_instances)
        with torch.cuda.stream(self.stream):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        self.b = cc_batch_create(max_instances, precision, ptr, nbytes, self.stream.cuda_stream)
        self.members = []

    def close(self):
        if getattr(self, "b", None):
            cc_batch_destroy(self.b)
            self.b = None
            self.members = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, solver):
        cc_batch_add(self.b, solver.ctx)
        self.members.append(solver)

    def remove(self, solver):
        cc_batch_remove(self.b, solver.ctx)
        self.members.remove(solver)

    def set_tiles(self, tile_x, tile_y):
        cc_batch_set_tiles(self.b, tile_x, tile_y)

    def autotune(self, reps=20, cache_path=None):
        return cc_batch_autotune(self.b, reps, cache_path)

    def set_launch_mode(self, mode):
        cc_batch_set_launch_mode(self.b, mode)

    def step(self, dts):
        """One step of every member (member k with dts[k]); returns the status words."""
        return cc_batch_step(self.b, list(dts))

    def last_dt(self, cfl):
        """Next time steps from the speeds reduced by the last step, and status words."""
        return cc_batch_last_dt(self.b, cfl, len(self.members))

    def cfl_dt(self, cfl):
        return cc_batch_cfl_dt(self.b, cfl, len(self.members))

    def advance(self, nsteps, cfl, want_ms=False):
        """nsteps CFL steps of every member planned on the device; returns (per-member
        time steps, per-step ms or None)."""
        dts, ms, _ = cc_batch_advance(self.b, nsteps, cfl, len(self.members), want_ms)
        return dts, ms
