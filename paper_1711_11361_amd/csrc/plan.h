// Step planning on the device: the time step from the CFL condition of the current state
// (Sec. 4, global step from the regular cell size) and the host part of a split step (the
// rigid poses at the step's start, stage and end, Sec. 2.3.4; level regions, sweep boxes,
// motion), computed by one block at the head of each captured step, so that a run of steps
// is queued without waiting for the host between them.  The arithmetic is that of the host
// planner, in the same order (bit-identical for a body that does not turn; a turning body's
// angles come from the device's sin and cos).
#pragma once
#include "engine.h"

namespace cc {

// Rigid pose: x = cs bx - sn by + cx, y = sn bx + cs by + cy.
struct Pose {
    double cs, sn, cx, cy;
};

// Certificate discs of a posed polygon: points closer than sqrt(rin2) to (cx, cy) are
// inside it, points farther than sqrt(rout2) outside; rin2 < 0: no discs.
struct Cert {
    double cx, cy, rin2, rout2;
};

__host__ __device__ inline bool box_empty(const Box& b) { return b.i0 >= b.i1 || b.j0 >= b.j1; }

__host__ __device__ inline Box box_union(const Box& a, const Box& b) {
    if (box_empty(a)) return b;
    if (box_empty(b)) return a;
    return Box{a.i0 < b.i0 ? a.i0 : b.i0, a.i1 > b.i1 ? a.i1 : b.i1, a.j0 < b.j0 ? a.j0 : b.j0,
               a.j1 > b.j1 ? a.j1 : b.j1};
}

// Cells that a polygon with bounding box [xmin, xmax] x [ymin, ymax] may touch, with a
// margin of two cells (empty when it lies outside the domain).
__host__ __device__ inline Box cells_of_bbox(double xmin, double xmax, double ymin, double ymax, double x_lo,
                                             double x_hi, double y_lo, double y_hi, double hx, double hy, int nx,
                                             int ny) {
    if (xmax < x_lo || xmin > x_hi || ymax < y_lo || ymin > y_hi) return Box{0, 0, 0, 0};
    int i0 = (int)floor((xmin - x_lo) / hx) - 2;
    int i1 = (int)floor((xmax - x_lo) / hx) + 3;
    int j0 = (int)floor((ymin - y_lo) / hy) - 2;
    int j1 = (int)floor((ymax - y_lo) / hy) + 3;
    Box c{i0 > 0 ? i0 : 0, i1 < nx ? i1 : nx, j0 > 0 ? j0 : 0, j1 < ny ? j1 : ny};
    if (c.i0 >= c.i1 || c.j0 >= c.j1) c = Box{0, 0, 0, 0};
    return c;
}

// Sweep box: the union of the start and end cells the body may touch, grown by three.
__host__ __device__ inline Box sweep_box_of(const Box& a, const Box& b, int nx, int ny) {
    Box ub = box_union(a, b);
    Box B{0, 0, 0, 0};
    if (!box_empty(ub)) {
        B.i0 = ub.i0 - 3 > 0 ? ub.i0 - 3 : 0;
        B.i1 = ub.i1 + 3 < nx ? ub.i1 + 3 : nx;
        B.j0 = ub.j0 - 3 > 0 ? ub.j0 - 3 : 0;
        B.j1 = ub.j1 + 3 < ny ? ub.j1 + 3 : ny;
    }
    return B;
}

// Why a planned run stopped (PlanState::halt).
enum HaltCode {
    HALT_NONE = 0,
    HALT_STATUS = 1,     // the status word of the last step has an error bit
    HALT_SPEEDS = 2,     // the wave speeds of the state are not finite
    HALT_DT = 3,         // the time step is not positive and finite
    HALT_MOTION = 4,     // the body moves a cell or more within one sweep
    HALT_REGION = 5,     // a geometry region exceeds its capacity
    HALT_SWEEP_CAP = 6,  // a sweep box exceeds the staging capacity
};

// Constant planning data of a context.
struct PlanConst {
    StepArgs base;  // the constant part of every step's arguments
    const double* body;
    int m;
    double ref_x, ref_y, theta0, vx, vy, amp, omega;
    double cs0, sn0;  // cos and sin of theta0 (the pose of a body that does not turn)
    Cert cert0;       // discs of the body turned by theta0 about the pose origin
    double x_lo, x_hi, y_lo, y_hi, hx, hy;
    int nx, ny, gw, gh, capw, caph;
    char* u[2];  // the two state buffers
    double cfl;
};

// Bookkeeping that steps advance (the host's copy is written before a run and read after).
struct PlanState {
    double t, step_dt;
    long long step;
    int parity, s0, sm, s1, cur;
    int halt, steps;  // halt code; steps planned in this run
    Box lbox[3];
    Level lev[3];
    Motion mot;
    Box last_sweep_box;
};

__device__ inline Pose pose_at_dev(const PlanConst& P, double t) {
    if (P.amp == 0.0) return Pose{P.cs0, P.sn0, P.ref_x + P.vx * t, P.ref_y + P.vy * t};
    double th = P.theta0 + P.amp * sin(P.omega * t);
    return Pose{cos(th), sin(th), P.ref_x + P.vx * t, P.ref_y + P.vy * t};
}

// Per-thread partial results over the body's vertices.
struct VAcc {
    int bad;
    double sx, sy;  // vertex speeds at the step's start
    double xmin[2], xmax[2], ymin[2], ymax[2];  // stage polygon (0) and end polygon (1)
    double yb[2], yt[2], xl[2], xr[2];
    int ib[2], it[2], il[2], ir[2];
    double sumx[2], sumy[2];
};

__device__ inline void vacc_init(VAcc& a, double sx, double sy) {
    a.bad = 0;
    a.sx = sx;
    a.sy = sy;
    for (int q = 0; q < 2; q++) {
        a.xmin[q] = a.ymin[q] = INFINITY;
        a.xmax[q] = a.ymax[q] = -INFINITY;
        a.yb[q] = a.xl[q] = INFINITY;
        a.yt[q] = a.xr[q] = -INFINITY;
        a.ib[q] = a.it[q] = a.il[q] = a.ir[q] = 0x7fffffff;
        a.sumx[q] = a.sumy[q] = 0.0;
    }
}

// Least value, then least index (the first vertex among equals, as a sequential scan with
// strict comparisons keeps).
__device__ inline void arg_lo(double& v, int& k, double v2, int k2) {
    if (v2 < v || (v2 == v && k2 < k)) {
        v = v2;
        k = k2;
    }
}
__device__ inline void arg_hi(double& v, int& k, double v2, int k2) {
    if (v2 > v || (v2 == v && k2 < k)) {
        v = v2;
        k = k2;
    }
}

__device__ inline void vacc_merge(VAcc& a, const VAcc& b) {
    a.bad |= b.bad;
    a.sx = fmax(a.sx, b.sx);
    a.sy = fmax(a.sy, b.sy);
    for (int q = 0; q < 2; q++) {
        a.xmin[q] = fmin(a.xmin[q], b.xmin[q]);
        a.xmax[q] = fmax(a.xmax[q], b.xmax[q]);
        a.ymin[q] = fmin(a.ymin[q], b.ymin[q]);
        a.ymax[q] = fmax(a.ymax[q], b.ymax[q]);
        arg_lo(a.yb[q], a.ib[q], b.yb[q], b.ib[q]);
        arg_hi(a.yt[q], a.it[q], b.yt[q], b.it[q]);
        arg_lo(a.xl[q], a.il[q], b.xl[q], b.il[q]);
        arg_hi(a.xr[q], a.ir[q], b.xr[q], b.ir[q]);
        a.sumx[q] += b.sumx[q];
        a.sumy[q] += b.sumy[q];
    }
}

constexpr int T_PLAN = 256;

// Block reduction of a trivially copyable accumulator through LDS (every thread calls it;
// thread 0 holds the result).
template <class A, class F>
__device__ inline void block_reduce(A& a, A* sh, F merge) {
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = T_PLAN / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) merge(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    a = sh[0];
    __syncthreads();
}

// Certificate discs of a turning body's posed polygon (the host's formula; the centroid
// sum is taken in another order, which moves the discs by rounding only, far inside their
// margins).
struct CAcc {
    double rin, rr;
};

__device__ inline void posed(const PlanConst& P, const Pose& px, const Pose& py, int k, double& x, double& y) {
    double bx = P.body[2 * k], by = P.body[2 * k + 1];
    x = (px.cs * bx - px.sn * by) + px.cx;
    y = (py.sn * bx + py.cs * by) + py.cy;
}

// A step that does nothing: no geometry jobs, empty sweep boxes, no dense direction.
__device__ inline void null_step(const PlanConst& P, const PlanState& S, StepArgs& a) {
    a = P.base;
    a.geo[0].active = a.geo[1].active = 0;
    for (int s = 0; s < 2; s++) {
        a.sw[s].B = Box{0, 0, 0, 0};
        a.sw[s].dir = 2;
        a.sw[s].Uin = a.sw[s].Uout = P.u[S.cur];
    }
}

// One step's planning: dt from the speeds the last step left (cfl_out), then the poses,
// regions, boxes and motion of the step, then the bookkeeping of its end (slots swapped,
// clock advanced, direction order reversed).  One block of T_PLAN threads.
__global__ __launch_bounds__(T_PLAN) void kb_plan(const PlanConst* __restrict__ PC, PlanState* __restrict__ PS,
                                                  StepArgs* __restrict__ out, double* __restrict__ dt_log) {
    const PlanConst& P = *PC;
    __shared__ PlanState S;
    __shared__ VAcc sh[T_PLAN];
    __shared__ double sdt;
    __shared__ int halt;
    if (threadIdx.x == 0) {
        S = *PS;
        halt = S.halt;
        if (!halt) {
            unsigned int st = __hip_atomic_load(P.base.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (st & (1u | 2u | 8u)) halt = HALT_STATUS;
        }
    }
    __syncthreads();
    double sx = __longlong_as_double((long long)P.base.cfl_out[0]);
    double sy = __longlong_as_double((long long)P.base.cfl_out[1]);
    if (!halt && threadIdx.x == 0 && !(isfinite(sx) && isfinite(sy))) halt = HALT_SPEEDS;
    __syncthreads();
    int m = P.m;
    double t0 = S.t;
    Pose q0 = pose_at_dev(P, t0);
    // vertex speeds at t^n (the rigid velocity of each vertex of the posed body)
    if (!halt && m > 0) {
        double thd = P.amp * P.omega * cos(P.omega * t0);
        double cx = P.ref_x + P.vx * t0, cy = P.ref_y + P.vy * t0;
        VAcc a;
        vacc_init(a, sx, sy);
        for (int k = threadIdx.x; k < m; k += T_PLAN) {
            double x, y;
            posed(P, q0, q0, k, x, y);
            double ux = P.vx - thd * (y - cy);
            double uy = P.vy + thd * (x - cx);
            a.sx = fmax(a.sx, fabs(ux));
            a.sy = fmax(a.sy, fabs(uy));
        }
        block_reduce(a, sh, vacc_merge);
        sx = a.sx;
        sy = a.sy;
    }
    if (threadIdx.x == 0) {
        double dt = P.cfl * fmin(P.hx / sx, P.hy / sy);
        if (!halt && (!(dt > 0.0) || !isfinite(dt))) halt = HALT_DT;
        sdt = dt;
    }
    __syncthreads();
    double dt = sdt;
    double t1 = t0 + dt;
    Pose q1 = pose_at_dev(P, t1);
    // stage polygon: the first sweep's coordinate at t^{n+1}, the other at t^n
    Pose mx = S.parity == 0 ? q1 : q0, my = S.parity == 0 ? q0 : q1;
    VAcc a;
    vacc_init(a, 0.0, 0.0);
    if (!halt && m > 0) {
        for (int k = threadIdx.x; k < m; k += T_PLAN) {
            double x0, y0, x1, y1, xm, ym;
            posed(P, q0, q0, k, x0, y0);
            posed(P, q1, q1, k, x1, y1);
            posed(P, mx, my, k, xm, ym);
            if (!(fabs(x1 - x0) < P.hx) || !(fabs(y1 - y0) < P.hy)) a.bad = 1;
            double xs[2] = {xm, x1}, ys[2] = {ym, y1};
            for (int q = 0; q < 2; q++) {
                a.xmin[q] = fmin(a.xmin[q], xs[q]);
                a.xmax[q] = fmax(a.xmax[q], xs[q]);
                a.ymin[q] = fmin(a.ymin[q], ys[q]);
                a.ymax[q] = fmax(a.ymax[q], ys[q]);
                arg_lo(a.yb[q], a.ib[q], ys[q], k);
                arg_hi(a.yt[q], a.it[q], ys[q], k);
                arg_lo(a.xl[q], a.il[q], xs[q], k);
                arg_hi(a.xr[q], a.ir[q], xs[q], k);
                a.sumx[q] += xs[q];
                a.sumy[q] += ys[q];
            }
        }
        block_reduce(a, sh, vacc_merge);
    }
    // discs of a turning body's polygons
    Cert cq[2] = {P.cert0, P.cert0};
    if (!halt && m > 0) {
        if (P.amp == 0.0) {
            if (P.cert0.rin2 >= 0.0) {
                cq[0].cx += mx.cx;
                cq[0].cy += my.cy;
                cq[1].cx += q1.cx;
                cq[1].cy += q1.cy;
            }
        } else {
            for (int q = 0; q < 2; q++) {
                cq[q] = Cert{0.0, 0.0, -1.0, 0.0};
                if (m < 8) continue;
                double cx = a.sumx[q] / m, cy = a.sumy[q] / m;
                const Pose& px = q == 0 ? mx : q1;
                const Pose& py = q == 0 ? my : q1;
                CAcc c{INFINITY, 0.0};
                for (int k = threadIdx.x; k < m; k += T_PLAN) {
                    int k1 = k + 1 == m ? 0 : k + 1;
                    double x, y, x1, y1;
                    posed(P, px, py, k, x, y);
                    posed(P, px, py, k1, x1, y1);
                    double ex = x1 - x, ey = y1 - y;
                    double l2 = ex * ex + ey * ey;
                    if (l2 > 0.0) c.rin = fmin(c.rin, (ex * (cy - y) - ey * (cx - x)) / sqrt(l2));
                    double dx = x - cx, dy = y - cy;
                    c.rr = fmax(c.rr, dx * dx + dy * dy);
                }
                CAcc* shc = reinterpret_cast<CAcc*>(sh);
                block_reduce(c, shc, [](CAcc& u, const CAcc& v) {
                    u.rin = fmin(u.rin, v.rin);
                    u.rr = fmax(u.rr, v.rr);
                });
                double rout = sqrt(c.rr);
                if (c.rin > 1e-7 * rout && isfinite(c.rin)) {
                    cq[q].cx = cx;
                    cq[q].cy = cy;
                    cq[q].rin2 = (c.rin * (1.0 - 1e-6)) * (c.rin * (1.0 - 1e-6));
                    cq[q].rout2 = (rout * (1.0 + 1e-6)) * (rout * (1.0 + 1e-6));
                }
            }
        }
    }
    if (threadIdx.x != 0) return;
    if (!halt && m > 0 && a.bad) halt = HALT_MOTION;
    StepArgs& A = *out;
    if (halt) {
        null_step(P, S, A);
        S.halt = halt;
        *PS = S;
        return;
    }
    A = P.base;
    if (m > 0) {
        Poly pl[2];
        Box cb[2];
        for (int q = 0; q < 2; q++) {
            Poly& Q = pl[q];
            Q = S.lev[q == 0 ? S.sm : S.s1].poly;
            Q.m = m;
            Q.xmin = a.xmin[q];
            Q.xmax = a.xmax[q];
            Q.ymin = a.ymin[q];
            Q.ymax = a.ymax[q];
            Q.ib = a.ib[q];
            Q.it = a.it[q];
            Q.il = a.il[q];
            Q.ir = a.ir[q];
            Q.cx = cq[q].cx;
            Q.cy = cq[q].cy;
            Q.rin2 = cq[q].rin2;
            Q.rout2 = cq[q].rout2;
            cb[q] = cells_of_bbox(Q.xmin, Q.xmax, Q.ymin, Q.ymax, P.x_lo, P.x_hi, P.y_lo, P.y_hi, P.hx, P.hy, P.nx,
                                  P.ny);
        }
        Box rm = box_union(S.lbox[S.sm], cb[0]), r1 = box_union(S.lbox[S.s1], cb[1]);
        auto fits = [&](const Box& r) { return box_empty(r) || (r.w() <= P.gw && r.h() <= P.gh); };
        if (!fits(rm) || !fits(r1)) {
            null_step(P, S, A);
            S.halt = HALT_REGION;
            *PS = S;
            return;
        }
        S.lev[S.sm].poly = pl[0];
        S.lev[S.s1].poly = pl[1];
        S.lbox[S.sm] = cb[0];
        S.lbox[S.s1] = cb[1];
        const int slot[2] = {S.sm, S.s1};
        const Box reg[2] = {rm, r1};
        const Pose px[2] = {mx, q1}, py[2] = {my, q1};
        for (int k = 0; k < 2; k++) {
            GeoJob& J = A.geo[k];
            J.L = S.lev[slot[k]];
            J.reg = reg[k];
            J.cs_x = px[k].cs;
            J.sn_x = px[k].sn;
            J.cx_x = px[k].cx;
            J.cs_y = py[k].cs;
            J.sn_y = py[k].sn;
            J.cy_y = py[k].cy;
            J.active = !box_empty(reg[k]);
        }
        // rigid map of the step and the wall velocity at mid-step
        double th0 = P.amp == 0.0 ? P.theta0 : P.theta0 + P.amp * sin(P.omega * t0);
        double th1 = P.amp == 0.0 ? P.theta0 : P.theta0 + P.amp * sin(P.omega * t1);
        Motion& M = S.mot;
        M.cosd = cos(th1 - th0);
        M.sind = sin(th1 - th0);
        M.c0x = P.ref_x + P.vx * t0;
        M.c0y = P.ref_y + P.vy * t0;
        M.c1x = P.ref_x + P.vx * t1;
        M.c1y = P.ref_y + P.vy * t1;
        double th = t0 + 0.5 * dt;
        M.vx = P.vx;
        M.vy = P.vy;
        M.thd = P.amp * P.omega * cos(P.omega * th);
        M.chx = P.ref_x + P.vx * th;
        M.chy = P.ref_y + P.vy * th;
    }
    A.mot = S.mot;
    for (int s = 0; s < 2; s++) {
        SweepJob& J = A.sw[s];
        int first = s == 0;
        int sl = first ? S.s0 : S.sm, el = first ? S.sm : S.s1;
        J.Ls = S.lev[sl];
        J.Le = S.lev[el];
        J.B = sweep_box_of(S.lbox[sl], S.lbox[el], P.nx, P.ny);
        J.dir = first ? S.parity : 1 - S.parity;
        J.first = first;
        J.lam = dt / (J.dir == 0 ? P.hx : P.hy);
        int rin = first ? S.cur : 1 - S.cur;
        J.Uin = P.u[rin];
        J.Uout = P.u[1 - rin];
        if (!box_empty(J.B) && (J.B.w() > P.capw || J.B.h() > P.caph)) {
            null_step(P, S, A);
            S.halt = HALT_SWEEP_CAP;
            *PS = S;
            return;
        }
    }
    A.step_id = (int32_t)(S.step & 0x7fffffff);
    A.cfl_alpha = S.lev[S.s1].alpha;
    A.cfl_U = P.u[S.cur];
    S.last_sweep_box = A.sw[1].B;
    // the step's end: slots swapped, clock advanced, the direction order reversed
    dt_log[S.steps] = dt;
    S.step_dt = dt;
    int tmp = S.s0;
    S.s0 = S.s1;
    S.s1 = tmp;
    S.t = t0 + dt;
    S.step++;
    S.parity ^= 1;
    S.steps++;
    *PS = S;
}

}  // namespace cc
