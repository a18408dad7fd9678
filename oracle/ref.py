"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

A workload is described by plain Python data (see paper_1711_11361_amd.workloads): a grid
dict, a body dict and primitive initial fields.  This module turns them into the oracle's
own C structs; it does not share any code with the GPU binding.
"""
import ctypes as C

import numpy as np

from . import build as _build


class _Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("bc", C.c_int32 * 4),
                ("precision", C.c_int32), ("options", C.c_int32),
                ("x_lo", C.c_double), ("x_hi", C.c_double), ("y_lo", C.c_double),
                ("y_hi", C.c_double), ("gamma", C.c_double), ("alpha_min", C.c_double)]


class _Body(C.Structure):
    _fields_ = [("nverts", C.c_int32), ("pad_", C.c_int32), ("verts", C.POINTER(C.c_double)),
                ("ref_x", C.c_double), ("ref_y", C.c_double), ("theta0", C.c_double),
                ("vx", C.c_double), ("vy", C.c_double), ("pitch_amp", C.c_double),
                ("pitch_omega", C.c_double)]


_libs = {}


def lib(parallel=False):
    """The oracle library: the plain build, or (parallel) the OpenMP build of the same
    source, which gives identical results on all host cores."""
    L = _libs.get(parallel)
    if L is None:
        L = C.CDLL(_build.ensure_built(parallel))
        _libs[parallel] = L
        d, i, p, vp = C.c_double, C.c_int, C.POINTER(C.c_double), C.c_void_p
        L.ccref_create.restype = vp
        L.ccref_create.argtypes = [C.POINTER(_Config), C.POINTER(_Body)]
        L.ccref_create_bodies.restype = vp
        L.ccref_create_bodies.argtypes = [C.POINTER(_Config), C.POINTER(_Body), i]
        L.ccref_surface_loads_body.argtypes = [vp, i, p]
        L.ccref_nbodies.argtypes = [vp]
        L.ccref_cell_bodies.argtypes = [vp, i, C.POINTER(C.c_int8)]
        L.ccref_destroy.argtypes = [vp]
        L.ccref_set_prim.argtypes = [vp, p, d]
        L.ccref_set_u.argtypes = [vp, p]
        L.ccref_set_clock.argtypes = [vp, d, C.c_int64]
        L.ccref_get_u.argtypes = [vp, p]
        L.ccref_get_prim.argtypes = [vp, p]
        L.ccref_time.restype = d
        L.ccref_time.argtypes = [vp]
        L.ccref_steps.restype = C.c_int64
        L.ccref_steps.argtypes = [vp]
        L.ccref_parity.argtypes = [vp]
        L.ccref_status.argtypes = [vp]
        L.ccref_collapses.restype = C.c_int64
        L.ccref_collapses.argtypes = [vp]
        L.ccref_pose.argtypes = [vp, d, p]
        L.ccref_geometry_poly.argtypes = [vp, p, i, i]
        L.ccref_geometry.argtypes = [vp, d, i]
        L.ccref_geometry_dump.argtypes = [vp, i, C.POINTER(C.c_int8), p, p, p]
        L.ccref_wall_point.argtypes = [vp, i, i, i, p]
        L.ccref_wave_speeds.argtypes = [vp, p]
        L.ccref_cfl_dt.restype = d
        L.ccref_cfl_dt.argtypes = [vp, d]
        L.ccref_totals.argtypes = [vp, p]
        L.ccref_surface_loads.argtypes = [vp, p]
        L.ccref_surface_pressure.restype = i
        L.ccref_surface_pressure.argtypes = [vp, p, i]
        L.ccref_budget.argtypes = [vp, p, p, p]
        L.ccref_sweep.argtypes = [vp, i, d]
        L.ccref_begin_step.argtypes = [vp, d]
        L.ccref_end_step.argtypes = [vp]
        L.ccref_step.argtypes = [vp, d]
        L.ccref_hllc.argtypes = [p, p, i, d, p]
        L.ccref_hllc.restype = None
        L.ccref_flux.argtypes = [p, i, d, p]
        L.ccref_flux.restype = None
        L.ccref_vanleer.restype = d
        L.ccref_vanleer.argtypes = [d, d]
        L.ccref_muscl.argtypes = [p, p, p, i, d, i, d, p, p]
        L.ccref_muscl.restype = None
        L.ccref_wall_riemann.argtypes = [p, d, d, d, d, d, p]
        L.ccref_wall_riemann.restype = None
        L.ccref_clip_area.restype = d
        L.ccref_clip_area.argtypes = [p, i, d, d, d, d]
        L.ccref_face_intervals.argtypes = [vp, i, p, p]
        L.ccref_body_velocity.argtypes = [vp, d, d, d, p]
        L.ccref_body_velocity.restype = None
        L.ccref_step_disp.argtypes = [vp, i, d, d]
        L.ccref_step_disp.restype = d
        L.ccref_trace.argtypes = [vp, i, i]
        L.ccref_trace_get.argtypes = [vp, p]
        L.ccref_set_option.argtypes = [vp, i, i]
        L.ccref_cut_list.argtypes = [vp, i, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- pure building blocks
def hllc(ql, qr, d, gamma=1.4):
    ql, qr = _f64(ql), _f64(qr)
    f = np.zeros(4)
    lib().ccref_hllc(_dp(ql), _dp(qr), d, gamma, _dp(f))
    return f


def flux(q, d, gamma=1.4):
    q = _f64(q)
    f = np.zeros(4)
    lib().ccref_flux(_dp(q), d, gamma, _dp(f))
    return f


def vanleer(a, b):
    return lib().ccref_vanleer(a, b)


def muscl(qm, q, qp, ok, lam, d, gamma=1.4):
    qm, q, qp = _f64(qm), _f64(q), _f64(qp)
    el, er = np.zeros(4), np.zeros(4)
    lib().ccref_muscl(_dp(qm), _dp(q), _dp(qp), int(ok), lam, d, gamma, _dp(el), _dp(er))
    return el, er


def clip_area(poly, x0, y0, w, h):
    poly = _f64(np.asarray(poly).reshape(-1))
    return lib().ccref_clip_area(_dp(poly), len(poly) // 2, x0, y0, w, h)


def wall_riemann(q, n, uw, gamma=1.4):
    q = _f64(q)
    out = np.zeros(2)
    lib().ccref_wall_riemann(_dp(q), n[0], n[1], uw[0], uw[1], gamma, _dp(out))
    return out[0], out[1]


# ---------------------------------------------------------------- simulation context
def _fill_body(b, body):
    """Fill a _Body from a body dict; returns the vertex array it points to."""
    verts = _f64(np.asarray(body["verts"]).reshape(-1))
    b.nverts = len(verts) // 2
    b.verts = _dp(verts)
    b.ref_x, b.ref_y = body.get("ref", (0.0, 0.0))
    b.theta0 = body.get("theta0", 0.0)
    b.vx, b.vy = body.get("vel", (0.0, 0.0))
    b.pitch_amp = body.get("pitch_amp", 0.0)
    b.pitch_omega = body.get("pitch_omega", 0.0)
    return verts


class Oracle:
    """One oracle simulation: a grid, a rigid body (or `bodies`, a list of up to four
    body dicts, each with its own motion) and the level-n state."""

    def __init__(self, grid, body=None, parallel=False, bodies=None):
        self._L = lib(parallel)
        self.grid = dict(grid)
        cfg = _Config()
        cfg.nx, cfg.ny = grid["nx"], grid["ny"]
        for k, v in enumerate(grid.get("bc", (0, 0, 0, 0))):
            cfg.bc[k] = v
        cfg.precision = 0
        cfg.x_lo, cfg.x_hi = grid["x_lo"], grid["x_hi"]
        cfg.y_lo, cfg.y_hi = grid["y_lo"], grid["y_hi"]
        cfg.gamma = grid.get("gamma", 1.4)
        cfg.alpha_min = grid.get("alpha_min", 0.0)
        cfg.options = 1 if grid.get("axisymmetric", False) else 0
        self.nx, self.ny = cfg.nx, cfg.ny
        self.gamma = cfg.gamma
        if bodies is not None:
            arr = (_Body * len(bodies))()
            self._verts = [_fill_body(arr[k], bd) for k, bd in enumerate(bodies)]
            self.m = sum(arr[k].nverts for k in range(len(bodies)))
            h = self._L.ccref_create_bodies(C.byref(cfg), arr, len(bodies))
            if not h:
                raise ValueError("oracle: invalid configuration")
            self._h = C.c_void_p(h)
            return
        b = _Body()
        self._verts = None
        if body is not None and len(body["verts"]) > 0:
            self._verts = _f64(np.asarray(body["verts"]).reshape(-1))
            b.nverts = len(self._verts) // 2
            b.verts = _dp(self._verts)
            b.ref_x, b.ref_y = body.get("ref", (0.0, 0.0))
            b.theta0 = body.get("theta0", 0.0)
            b.vx, b.vy = body.get("vel", (0.0, 0.0))
            b.pitch_amp = body.get("pitch_amp", 0.0)
            b.pitch_omega = body.get("pitch_omega", 0.0)
        else:
            b.nverts = 0
        self.m = b.nverts
        h = self._L.ccref_create(C.byref(cfg), C.byref(b))
        if not h:
            raise ValueError("oracle: invalid configuration")
        self._h = C.c_void_p(h)

    def close(self):
        if getattr(self, "_h", None):
            self._L.ccref_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # state
    def set_prim(self, prim, t0=0.0):
        prim = _f64(prim).reshape(4, self.ny, self.nx)
        self._L.ccref_set_prim(self._h, _dp(prim), t0)

    def set_clock(self, t, step):
        """Resume at time t after `step` split steps (sweep order and level-n geometry of an
        uninterrupted run); set the state afterwards."""
        if self._L.ccref_set_clock(self._h, float(t), int(step)) != 0:
            raise ValueError("bad step count")

    def set_u(self, U):
        U = _f64(U).reshape(4, self.ny, self.nx)
        self._L.ccref_set_u(self._h, _dp(U))

    def get_u(self):
        U = np.zeros((4, self.ny, self.nx))
        self._L.ccref_get_u(self._h, _dp(U))
        return U

    def get_prim(self):
        P = np.zeros((4, self.ny, self.nx))
        self._L.ccref_get_prim(self._h, _dp(P))
        return P

    @property
    def t(self):
        return self._L.ccref_time(self._h)

    @property
    def steps(self):
        return self._L.ccref_steps(self._h)

    @property
    def parity(self):
        return self._L.ccref_parity(self._h)

    @property
    def status(self):
        return self._L.ccref_status(self._h)

    @property
    def collapses(self):
        return self._L.ccref_collapses(self._h)

    # geometry
    def pose(self, t):
        out = np.zeros(2 * max(self.m, 1))
        self._L.ccref_pose(self._h, t, _dp(out))
        return out[: 2 * self.m].reshape(-1, 2)

    def geometry(self, t, which=0):
        if self._L.ccref_geometry(self._h, t, which):
            raise ValueError("bad level")

    def geometry_poly(self, posed, which=0):
        posed = _f64(np.asarray(posed).reshape(-1))
        if self._L.ccref_geometry_poly(self._h, _dp(posed), len(posed) // 2, which):
            raise ValueError("bad level")

    def geometry_dump(self, which=0):
        nx, ny = self.nx, self.ny
        vc = np.zeros((ny + 1, nx + 1), dtype=np.int8)
        al = np.zeros((ny, nx))
        bx = np.zeros((ny, nx + 1))
        by = np.zeros((ny + 1, nx))
        self._L.ccref_geometry_dump(self._h, which, vc.ctypes.data_as(C.POINTER(C.c_int8)),
                                  _dp(al), _dp(bx), _dp(by))
        return {"vcls": vc, "alpha": al, "bx": bx, "by": by}

    def cut_list(self, which=0):
        """Linear indices (j nx + i, increasing) of the level's cut cells."""
        out = np.zeros(self.nx * self.ny, dtype=np.int32)
        n = C.c_int32()
        self._L.ccref_cut_list(self._h, which, out.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(n))
        return out[: n.value].copy()

    def wall_point(self, i, j, which=0):
        out = np.zeros(2)
        ok = self._L.ccref_wall_point(self._h, which, i, j, _dp(out))
        return out if ok else None

    def face_intervals(self, which=0):
        nx, ny = self.nx, self.ny
        fx = np.zeros((ny, nx + 1, 2))
        fy = np.zeros((ny + 1, nx, 2))
        self._L.ccref_face_intervals(self._h, which, _dp(fx), _dp(fy))
        return fx, fy

    # time stepping
    def wave_speeds(self):
        out = np.zeros(2)
        self._L.ccref_wave_speeds(self._h, _dp(out))
        return out

    def cfl_dt(self, cfl):
        return self._L.ccref_cfl_dt(self._h, cfl)

    def begin_step(self, dt):
        if self._L.ccref_begin_step(self._h, dt):
            raise RuntimeError("begin_step refused")

    def sweep(self, d, dt):
        if self._L.ccref_sweep(self._h, d, dt):
            raise RuntimeError("sweep refused")

    def end_step(self):
        if self._L.ccref_end_step(self._h):
            raise RuntimeError("end_step refused")

    def step(self, dt):
        if self._L.ccref_step(self._h, dt):
            raise RuntimeError("step refused")

    def totals(self):
        out = np.zeros(4)
        self._L.ccref_totals(self._h, _dp(out))
        return out

    def surface_loads(self):
        """(Fx, Fy, Mz about the pose origin, sum p*|N|) of the gas on the body at level n."""
        out = np.zeros(4)
        self._L.ccref_surface_loads(self._h, _dp(out))
        return out

    def body_loads(self, b):
        """surface_loads of body b of a context with several bodies (the wall cells it cuts)."""
        out = np.zeros(4)
        if self._L.ccref_surface_loads_body(self._h, int(b), _dp(out)) != 0:
            raise ValueError("no such body")
        return out

    @property
    def nbodies(self):
        return self._L.ccref_nbodies(self._h)

    def cell_bodies(self, which=0):
        """Body cutting each cut cell of a level (-1 elsewhere); several bodies only."""
        out = np.zeros((self.ny, self.nx), dtype=np.int8)
        if self._L.ccref_cell_bodies(self._h, which, out.ctypes.data_as(C.POINTER(C.c_int8))) != 0:
            raise ValueError("one body: no cell bodies")
        return out

    def surface_pressure(self):
        """Wall cells at level n in increasing index: rows (index, wall x, wall y, p*, Nx, Ny)."""
        n = self._L.ccref_surface_pressure(self._h, None, 0)
        out = np.zeros((max(n, 1), 6))
        self._L.ccref_surface_pressure(self._h, _dp(out), n)
        return out[:n]

    def budget(self):
        b, w, l = np.zeros(4), np.zeros(4), np.zeros(4)
        self._L.ccref_budget(self._h, _dp(b), _dp(w), _dp(l))
        return b, w, l

    # test hooks
    def body_velocity(self, t, x, y):
        out = np.zeros(2)
        self._L.ccref_body_velocity(self._h, t, x, y, _dp(out))
        return out

    def step_disp(self, d, x, y):
        """Displacement along d of (x, y) under the rigid map of the open step."""
        return self._L.ccref_step_disp(self._h, d, x, y)

    def trace(self, i, j):
        """Record the sweep quantities of cell (i, j) in the following sweeps."""
        self._L.ccref_trace(self._h, i, j)

    def trace_get(self):
        r = np.zeros(31)
        self._L.ccref_trace_get(self._h, _dp(r))
        return {"F_lo": r[0:4], "F_hi": r[4:8], "phi_lo": r[8:12], "phi_hi": r[12:16], "FB": r[16:20],
                "Q": r[20:24], "alpha_s": r[24], "alpha_e": r[25], "bt_lo": r[26], "bt_hi": r[27],
                "ahat": r[28], "wall": bool(r[29]), "has": bool(r[30])}

    def set_uncover_moves_content(self, on):
        """Oracle-only: cells that become fluid take content from their donors as printed
        (instead of a state only, reading R13)."""
        self._L.ccref_set_option(self._h, 1, int(bool(on)))

    def run(self, cfl, nsteps=None, t_end=None, dts=None):
        """Advance with the CFL time step; returns the list of dt used."""
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
                    if self.t >= t_end * (1 - 1e-14):
                        break
                    dt = min(dt, t_end - self.t)
            self.step(dt)
            used.append(dt)
            k += 1
        return used
